// Internal declarations shared by the host runtime and the HIP kernels of the
// boundary-element library.  Not part of the C ABI (that is include/bem.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/bem.h"

namespace bem {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

struct Error {
    bem_status status;
    std::string msg;
};

void set_error(const std::string &msg);

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------

// The library's device memory is stream-ordered (hipMallocAsync /
// hipFreeAsync) on the stream of the work at hand, so that one problem's
// allocations and frees never wait for the whole device, and requests served
// side by side on their own streams do not stall each other.  Each entry
// point sets the calling thread's allocation stream (AllocScope) to its
// problem's stream.
hipStream_t &alloc_stream();
void dmalloc(void **p, size_t bytes);
void dfree(void *p);
struct AllocScope {
    hipStream_t saved;
    explicit AllocScope(hipStream_t s) : saved(alloc_stream()) { alloc_stream() = s; }
    ~AllocScope() { alloc_stream() = saved; }
    AllocScope(const AllocScope &) = delete;
    AllocScope &operator=(const AllocScope &) = delete;
};

#define BEM_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::bem::Error{e_ == hipErrorOutOfMemory ? BEM_ERR_OOM : BEM_ERR_DEVICE,       \
                               std::string(#call) + ": " + hipGetErrorString(e_)};            \
    } while (0)

// ---------------------------------------------------------------------------
// quadrature constants (shared by the kernels through these definitions)
// ---------------------------------------------------------------------------

// Pair classes of two triangles of one boundary.
enum PairClass : int { FAR = 0, VERTEX = 1, EDGE = 2, COINCIDENT = 3 };

// Far-field work: one wavenumber pass of the pair kernel over a test range and
// a trial range of quadrature points.
struct PassDesc {
    int64_t test_begin, test_end;    // quadrature-point range of test points
    int64_t trial_begin, trial_end;  // quadrature-point range of trial points
    double kre, kim;                 // wavenumber of the pass
    double sV, sW;                   // density scalings of V and W (PMCHWT interior blocks)
    int slot;                        // partial-sum slot (0: exterior pass, 1: interior pass)
    int pad;
};

// Kernel-side copy of a pass (FP32 constants + ranges).
struct PassDev {
    long long test_begin, test_end, trial_begin, trial_end;
    float k, k_over_2pi, kim, sV;
    float sW, k2re, k2im, pad;       // k^2 (complex) for the W normal term
    int slot, pad2, pad3, pad4;
};

// One ordered touching pair (test triangle t, trial triangle s) of the singular
// pass.  pt/ps: local vertex orders that put the shared vertices first.
struct SingularItem {
    int t, s;
    int cls;
    int pass;          // index into the pass table (wavenumber and scalings)
    int pt[3], ps[3];
};

// Launch plan of the multi-right-hand-side GEMM (k_gemm.hip).
struct GemmPlan {
    int R;             // right-hand sides
    bool bf16;         // split-BF16 3-term (true) or FP32 MFMA (false)
    int shape;         // split-BF16 tile: 0 = 256 x 128 (4 waves), 1 = 384 x 128 (8 waves)
    int block;         // threads per workgroup
    int64_t Kp, Np;    // padded K (= 2n) and N (= 2R)
    int n_m, n_n, n_s; // m-tiles, n-tiles, K slices
    int64_t kslice;
    int n_wg;
    size_t bytes_x, bytes_c;
};

// One problem's share of a grouped pair-kernel launch (k_farfield.hip): its
// work list and the arrays the kernel reads and writes.
struct PairMember {
    const int4 *work;
    const PassDev *passes;
    const float *pts, *tnrm;
    const float4 *trial;
    double *part;
    int64_t M, nt;
    int n_split, pad;
};
constexpr int PAIR_GROUP_MAX = 16;
// Member table of a grouped launch, passed by value as the kernel argument:
// workgroups [start[m], start[m + 1]) run member m's work items.
struct PairGroup {
    int n, pad;
    int start[PAIR_GROUP_MAX + 1];
    PairMember m[PAIR_GROUP_MAX];
};

// OSRC preconditioner parameters (k_osrc.hip).
struct OsrcParams {
    int n_pade;
    double r_eps, theta;
    double cg_tol;     // relative tolerance of the inner COCG solves
    int cg_maxit;
};

// One block of the hierarchical matrix.  Vertices are reordered so that every
// cluster is a contiguous range; a block couples row vertices [r0, r1) and
// column vertices [c0, c1) of that order as a (2 m) x (2 n) complex matrix in
// interleaved (vertex, D/N) order.
struct HBlock {
    int32_t r0, r1, c0, c1;
    int32_t rank;      // -1: dense block D; else U V with this rank
    int32_t pad;
    float2 *U;         // (2 m) x rank, column-major
    float2 *V;         // rank x (2 n), row-major
    float2 *D;         // (2 m) x (2 n), column-major
    int64_t zoff;      // offset of the block's 2 m products in the product buffer
};
struct HMatrix;
struct OsrcWork;   // per-problem OSRC workspace (k_osrc.hip)

struct DomInfo {
    int64_t nv, nt;        // vertices / triangles of the domain
    int64_t v_off, t_off;  // offsets in the global vertex / triangle arrays
    double kre, kim, rho;
};

}  // namespace bem

// ---------------------------------------------------------------------------
// problem state (opaque handle of the C ABI)
// ---------------------------------------------------------------------------

struct bem_problem {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    int mode = BEM_OTF;
    int ss_order = 6;

    std::vector<bem::DomInfo> doms;
    double k0re = 0, k0im = 0, rho0 = 1;
    int64_t NV = 0, NT = 0, M = 0, N = 0;   // vertices, triangles, quadrature points, unknowns

    // host copies
    std::vector<double> h_verts;           // [NV][3]
    std::vector<int32_t> h_tris;           // [NT][3] global vertex indices
    std::vector<int32_t> h_rowD, h_rowN;   // unknown index of u_D / u_N per global vertex
    std::vector<bem::PassDesc> passes;

    // device geometry
    double *d_verts = nullptr;      // [NV][3]
    int32_t *d_tris = nullptr;      // [NT][3]
    int32_t *d_rowD = nullptr, *d_rowN = nullptr;
    double *d_area = nullptr;       // [NT]
    double *d_normal = nullptr;     // [NT][3]
    double *d_curl = nullptr;       // [NT][3][3]
    float *d_pts = nullptr;         // [3][M] FP32 quadrature points (SoA)
    float *d_tnrm = nullptr;        // [3][NT] FP32 triangle normals (SoA)
    int32_t *d_v2t_ptr = nullptr;   // [NV + 1]
    int32_t *d_v2t = nullptr;       // [3 NT]  (triangle * 3 + corner)

    // far-field pass
    bem::PassDev *d_pass = nullptr;
    int n_pass = 0;
    int4 *d_work = nullptr;         // (pass, test block, split, 0)
    int n_work = 0;
    int n_split = 8;
    int tpl = 1;                    // test points per lane of the pair kernel
    bool wrap_phase = true;         // phases k r / 2 pi may reach 256 revolutions: reduce them in the kernel
    float4 *d_trial = nullptr;      // trial records: [M][2] per point, then [NT][3] per triangle
    double *d_part = nullptr;       // [2][n_split][10][M]
    double *d_pot = nullptr;        // [M][10]

    // singular correction: vertex-level CSR with 4 complex blocks (DD, DN, ND, NN)
    int32_t *d_cptr = nullptr, *d_ccol = nullptr;
    double2 *d_cval = nullptr;      // [nnz][4]
    int64_t nnz = 0;
    // the same for the single-layer operator alone (pass 0 only; built on first use)
    int32_t *d_sl_cptr = nullptr, *d_sl_ccol = nullptr;
    double2 *d_sl_cval = nullptr;   // [nnz][4], block 1 = V
    int64_t sl_nnz = 0;
    bool sl_ready = false;
    int sl_tpl = 0, sl_split = 8;   // launch shape of the single-layer pair kernel (0: not chosen yet)

    // assembled mode: dense complex64 matrix, row-major [N][N]; BF16 planes
    // of its real view [N][2N] (hi and lo) for the split-BF16 GEMM
    float2 *d_A = nullptr;
    uint16_t *d_Ahi = nullptr, *d_Alo = nullptr;
    void *d_gx = nullptr;           // packed right-hand sides of the GEMM
    float *d_gc = nullptr;          // K-slice partial products of the GEMM
    size_t gx_bytes = 0, gc_bytes = 0;
    bool timed_gemm = false;

    // OSRC: vertex adjacency CSR with P1 mass and stiffness values
    int32_t *d_aptr = nullptr, *d_acol = nullptr;
    int32_t *d_adiag = nullptr;     // position of the diagonal entry of every row
    int2 *d_drange = nullptr;       // vertex range [begin, end) of every domain
    double *d_Mv = nullptr, *d_Sv = nullptr;
    int64_t a_nnz = 0;
    int *d_cg_chunks = nullptr;     // [chunks][8] row chunks of the batched COCG (domain, rows, first, count)
    int32_t *d_ell_col = nullptr;   // [9][NV] first entries of every row of the CSR above, slot-major
    double *d_ell_mv = nullptr, *d_ell_sv = nullptr;   // (padded with the row's own index and zeros)
    double2 *d_mdiag = nullptr;     // [NV] diagonal entries (M_ii, S_ii) of every row
    int cg_n_chunks = 0;
    bem::OsrcWork *osrc = nullptr;  // buffers, coefficients and captured COCG iterations of the last OSRC form

    // hierarchical matrix (bem_hmatrix_build)
    bem::HMatrix *hm = nullptr;

    // continuous batching (serving.cpp): the batch that launches this problem's
    // operator applies inside solves, and the events that order its stream and
    // the batch's around each apply
    bem_batch *batch = nullptr;
    hipEvent_t batch_ready = nullptr, batch_done = nullptr;

    // scratch vectors
    double2 *d_x = nullptr, *d_y = nullptr;
    int64_t scratch_rhs = 0;

    // timing
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
};

namespace bem {

// ---------------------------------------------------------------------------
// host-side mesh topology (mesh.cpp)
// ---------------------------------------------------------------------------

// Validate one domain's mesh; throws Error{BEM_ERR_MESH} with a message.
void validate_mesh(const double *v, int64_t nv, const int32_t *t, int64_t nt, int dom);
// Check that no two domains share or nearly share vertices (disjoint domains).
void validate_disjoint(const std::vector<DomInfo> &doms, const std::vector<double> &verts);
// Ordered touching pairs of every domain (sorted by class), for every pass that
// covers the domain (exterior pass 0 and the domain's own interior pass).
void touching_pairs(const bem_problem &p, std::vector<SingularItem> &items);
// Vertex-level pattern of the singular correction and the slot of every
// (item, a, b) contribution; contributions per slot are listed in item order.
void correction_pattern(const bem_problem &p, const std::vector<SingularItem> &items,
                        std::vector<int32_t> &cptr, std::vector<int32_t> &ccol,
                        std::vector<int32_t> &contrib_ptr, std::vector<int32_t> &contrib_idx);

// Sauter-Schwab rule of one class at order n on T x T, T = {0 <= s2 <= s1 <= 1}:
// rows (x1, x2, y1, y2, w).  Independent implementation of the library.
std::vector<double> singular_rule(int cls, int n);

// ---------------------------------------------------------------------------
// kernel launchers (k_*.hip)
// ---------------------------------------------------------------------------

void launch_geometry(bem_problem &p);
void launch_gather(bem_problem &p, const double2 *x);
void launch_pairs(bem_problem &p);
// kernel variant of a problem's pair kernel (problems of one variant can share a
// grouped launch) and the grouped launch of several problems' pair kernels
int pair_variant(const bem_problem &p);
void launch_pairs_group(hipStream_t s, const std::vector<bem_problem *> &ps);
void launch_reduce(bem_problem &p);
void launch_scatter(bem_problem &p, const double2 *x, double2 *y, int parts);
void launch_assemble_dense(bem_problem &p);
void launch_gemv(bem_problem &p, const double2 *x, double2 *y);
void split_matrix_bf16(bem_problem &p);
GemmPlan gemm_plan(const bem_problem &p, int R, bool bf16, int force_slices, int shape = 0);
void launch_gemm(bem_problem &p, const GemmPlan &g, const double2 *X, double2 *Y, void *xbuf, float *cbuf);
void launch_gemm_kernel(bem_problem &p, const GemmPlan &g, void *xbuf, float *cbuf);
void launch_unpack(bem_problem &p, const GemmPlan &g, const float *cbuf, double2 *Y);

// Blocks of a 1-D launch over `items` work items.  A dispatch counts its work
// items in 32 bits: kernels whose item count can exceed that loop over a capped
// grid (grid-stride) and pass capped = true; every other launch is checked.
// A uniform value (kernel argument, constant) copied into a VGPR.  On gfx950 a
// VALU instruction with an SGPR operand issues at half the rate of one whose
// operands are all VGPRs, so hot loops read their constants through this.
__device__ __forceinline__ float in_vgpr(float s)
{
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// Two complex64 matrix entries (16 bytes, 16-byte aligned) that a kernel reads
// once: a non-temporal load, so the streamed matrix does not displace what the
// caches hold (the GEMV runs 5 % faster than with cached loads).
__device__ __forceinline__ float4 load_streamed(const float2 *p)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}

inline unsigned blocks_1d(int64_t items, int block, bool capped = false)
{
    const int64_t b = (items + block - 1) / block;
    if (capped) return unsigned(std::max<int64_t>(1, std::min<int64_t>(b, int64_t(1) << 20)));
    if (b * block >= (int64_t(1) << 32)) throw Error{BEM_ERR_UNSUPPORTED, "launch exceeds 2^32 work items"};
    return unsigned(std::max<int64_t>(1, b));
}

// autotuner (autotune.cpp)
int tune_pairs(bem_problem &p, void (*rebuild)(bem_problem &), int max_split);
int tune_gemm_slices(bem_problem &p, int R, bool bf16, void *xbuf, float *cbuf, double2 *Y);
int cached_gemm_slices(bem_problem &p, int R, bool bf16);   // 0 when the bucket is untuned
// Singular correction of the given touching pairs into a vertex-level CSR with
// 4 complex blocks per entry (device arrays allocated here).
void run_singular(bem_problem &p, const std::vector<SingularItem> &items, int32_t **cptr, int32_t **ccol,
                  double2 **cval, int64_t *nnz);
// hierarchical matrix: block entries and the singular correction of near
// blocks (k_dense.hip), build and apply (hmatrix.cpp, k_hmatrix.hip)
struct EntryCtx;   // device inputs of the entry kernel (vertex records, domain constants)
EntryCtx *entry_ctx_create(bem_problem &p);
void entry_ctx_free(EntryCtx *c);
void launch_hblock_entries(bem_problem &p, EntryCtx *ctx, const int32_t *perm, const int4 *tiles, int64_t n_tiles,
                           const HBlock *blocks, float2 *const *out);
void launch_aca_partial(bem_problem &p, EntryCtx *ctx, const int32_t *perm, const HBlock *blocks, const int32_t *ids,
                        int n, float2 *const *U, float2 *const *V, const int32_t *kmax, float eps, int32_t *rank,
                        int max_side);
void launch_hblock_correction(bem_problem &p, const int2 *rows, int64_t n_rows, const HBlock *blocks,
                              float2 *const *out, const int32_t *perm, const int32_t *iperm);
void hmatrix_free(HMatrix *h);
HMatrix *hmatrix_build(bem_problem &p, double eps, int leaf, double eta, bem_hmatrix_info *info);
// Host-only plan of the hierarchical matrix's trees: out = {blocks, admissible
// blocks, entries of the singular pattern, of those the ones in admissible blocks}.
void hmatrix_plan(const bem_problem &p, int leaf, double eta, int64_t out[4]);
void hmatrix_apply(bem_problem &p, const double2 *x, double2 *y, int n_rhs, bool record);
// y = V_k0 x on the union of all boundaries (k_single_layer.hip); events as in the apply
void launch_single_layer(bem_problem &p, const double2 *x, double2 *y, bool record);

// FP64 complex vector helpers for GMRES (k_linalg.hip)
void zdot_multi(hipStream_t s, const double2 *V, int64_t ld, int nvec, const double2 *w, int64_t n,
                double2 *partials, int nblk, double2 *out_dev);
void zaxpy_multi(hipStream_t s, const double2 *V, int64_t ld, int nvec, const double2 *h_dev, double2 *w,
                 int64_t n, double sign);
void zscale_copy(hipStream_t s, const double2 *x, double2 *y, int64_t n, double2 a);
void zaxpy(hipStream_t s, double2 *y, const double2 *x, int64_t n, double2 a);

// batched FP64 complex kernels: R vectors of length n, bases [i][R][n] (k_linalg.hip)
// chunks of the batched dot products: partial buffers hold R * nvec * bdot_chunks(n) entries
constexpr int BD_CHUNK = 2048;
inline int bdot_chunks(int64_t n) { return int(std::max<int64_t>(1, (n + BD_CHUNK - 1) / BD_CHUNK)); }
void bdot(hipStream_t s, const double2 *V, int64_t ldv, int nvec, const double2 *w, int64_t n, int R,
          double2 *partials, int nblk, double2 *out_dev);
void baxpy(hipStream_t s, const double2 *V, int64_t ldv, int nvec, const double2 *h_dev, double2 *w, int64_t n, int R,
           double sign);
void bscale(hipStream_t s, const double2 *x, double2 *y, int64_t n, int R, const double2 *a_dev);

// batched (flexible) GMRES (krylov.cpp)
using ApplyFn = std::function<void(const double2 *X, double2 *Y, int R)>;
struct KrylovOpts {
    double tol;
    int restart;
    int max_iter;
    int progress = 0;             // print a line every `progress` Arnoldi steps (0: silent)
    const char *label = "gmres";
};
void gmres_batch(bem_problem &p, int64_t n, int R, const double2 *B, double2 *X, const KrylovOpts &o,
                 const ApplyFn &A, const ApplyFn *M, bem_solve_info *info);

// allocation-free apply (noalloc.hip): the file-scope scratch array of this
// many bytes; its device address on `device` (which must be current; looked up
// on first use), and a fill kernel that clears FP64 words
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
void *noalloc_scratch(int device);
void launch_zero_f64(hipStream_t s, double *p, int64_t n);

// continuous batching (serving.cpp): kinds of operator apply a problem hands
// to its batch, the hand-over (returns once the apply is launched and the
// problem's stream waits for it), and the count of problems inside a solve
enum BatchKind : int { BATCH_OTF = 0, BATCH_GEMV = 1, BATCH_GEMM_BF16 = 2, BATCH_GEMM_F32 = 3, BATCH_HMATRIX = 4 };
void batch_apply(bem_problem &p, int kind, const double2 *X, double2 *Y, int R);
void batch_enter(bem_batch &b);
void batch_leave(bem_batch &b);
void batch_detach(bem_problem &p);

// OSRC preconditioner (k_osrc.hip): Out = P Y for R residual vectors
void osrc_setup(bem_problem &p);
// enqueued on the problem's stream (the host waits only for the COCG convergence tests)
void osrc_apply(bem_problem &p, const OsrcParams &o, const double2 *Y, double2 *Out, int R);
void osrc_free(OsrcWork *w, hipStream_t s);

// incident fields and right-hand sides (k_field.hip)
void launch_rhs(bem_problem &p, const bem_incident &inc, double2 *b);
void launch_field(bem_problem &p, const double2 *u, const bem_incident *inc, int n_fields,
                  const double *pts, int64_t np, double2 *field, int32_t *region);

}  // namespace bem
