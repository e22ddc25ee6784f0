// Assembled mode: the dense complex64 PMCHWT matrix and its single-vector apply.
//
// Entry (row g, column h) of the four blocks (DD, DN, ND, NN) is the sum over
// the quadrature points q of the triangles at vertex g and p of the triangles
// at vertex h of the same pair integrands as the on-the-fly kernel, weighted by
// w_q lambda_g(q) w_p lambda_h(p) (curl term: w_q w_p curl_g . curl_h), for the
// exterior wavenumber and, when g and h lie on the same boundary, the interior
// one (paper eqs. Form1_calderon_sys_int_ptot and Form2_calderon_sys_simp3).
// Point-with-itself pairs are skipped (r = 0); the FP64 singular CSR is added
// afterwards, as in the on-the-fly apply.  Row-major storage: A[r * n + c],
// complex64 interleaved.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bem_internal.h"
#include "rule6.h"

namespace bem {

// Per (vertex, incident triangle corner, point) record, 3 x float4:
//   r0 = (x, w lambda_a(x) / (4 pi))   r1 = (n, w / (4 pi))   r2 = (curl lambda_a, 0)
// grouped by vertex: records [6 v2t_ptr[g], 6 v2t_ptr[g+1]).
__global__ void k_vertex_points(const int32_t *__restrict__ v2t, int64_t n_corner, const double *__restrict__ area,
                                const double *__restrict__ normal, const double *__restrict__ curl,
                                const float *__restrict__ pts, int64_t M, float4 *__restrict__ rec)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= 6 * n_corner) return;
    const int64_t c = k / 6;
    const int q = int(k - 6 * c);
    const int32_t tc = v2t[c];
    const int64_t t = tc / 3;
    const int a = tc - 3 * int(t);
    const int64_t i = 6 * t + q;
    const double w = area[t] * q6_w[q] * 0.079577471545947667884;
    rec[3 * k] = make_float4(pts[i], pts[M + i], pts[2 * M + i], float(w * q6_bary[q][a]));
    rec[3 * k + 1] = make_float4(float(normal[3 * t]), float(normal[3 * t + 1]), float(normal[3 * t + 2]), float(w));
    rec[3 * k + 2] = make_float4(float(curl[9 * t + 3 * a]), float(curl[9 * t + 3 * a + 1]),
                                 float(curl[9 * t + 3 * a + 2]), 0.0f);
}

struct DenseDom {
    float k, k2pi, kim, sV, sW, k2re, k2im, pad;
};

struct Acc4 {
    float vr, vi, kr, ki, pr, pi, wr, wi;
};

// sums of one pass over the point pairs of a (test corner, trial corner) pair:
// V = sum G (w lambda)(w lambda)',  Cc = sum G w w'
struct Corner {
    float vr, vi, cr, ci;
};

// one point pair of one pass: K and K' into the vertex-pair sums, V and the
// curl-term sum into the corner-pair sums (weights without the 4 pi)
template <bool ATT, bool WRAP>
__device__ __forceinline__ void dense_pair(float r, float rinv, float ww, float ws, float tK, float tKp, float k,
                                           float k2pi, float kim, Acc4 &A, Corner &C)
{
    float ph = r * k2pi;
    if (WRAP) ph = ph - rintf(ph);   // else the hardware sine and cosine reduce |ph| < 256 revolutions
    float gr = __builtin_amdgcn_cosf(ph) * rinv, gi = __builtin_amdgcn_sinf(ph) * rinv;
    const float kr = r * k, rinv2 = rinv * rinv;
    float fr, fi;
    if (ATT) {
        const float damp = __expf(-kim * r);
        gr *= damp;
        gi *= damp;
        const float re1 = fmaf(kim, r, 1.0f);
        fr = fmaf(gr, re1, gi * kr) * rinv2;
        fi = fmaf(gi, re1, -gr * kr) * rinv2;
    } else {
        fr = fmaf(gi, kr, gr) * rinv2;
        fi = fmaf(-gr, kr, gi) * rinv2;
    }
    C.vr = fmaf(ww, gr, C.vr);
    C.vi = fmaf(ww, gi, C.vi);
    C.cr = fmaf(ws, gr, C.cr);
    C.ci = fmaf(ws, gi, C.ci);
    const float wk = ww * tK, wp = ww * tKp;
    A.kr = fmaf(wk, fr, A.kr);
    A.ki = fmaf(wk, fi, A.ki);
    A.pr = fmaf(-wp, fr, A.pr);
    A.pi = fmaf(-wp, fi, A.pi);
}

// the factors constant on a corner pair: V += Vc and
// W += (curl.curl') Cc - k^2 (n.n') Vc   (complex k^2)
__device__ __forceinline__ void corner_done(const Corner &C, float cc, float nn, float k2re, float k2im, Acc4 &A)
{
    A.vr += C.vr;
    A.vi += C.vi;
    const float ar = k2re * nn, ai = k2im * nn;
    A.wr = fmaf(cc, C.cr, A.wr) - fmaf(ar, C.vr, -ai * C.vi);
    A.wi = fmaf(cc, C.ci, A.wi) - fmaf(ar, C.vi, ai * C.vr);
}

// Entry sums of vertex pair (g, h): the test records of g (global memory,
// the six points of a test corner held in registers) against the trial
// records of h (`trial`, in LDS when staged), exterior pass and, on the same
// boundary, interior pass.  The records of a corner share its triangle's
// normal and curl, so the curl.curl' and n.n' factors of the W entry multiply
// sums over the corner pair's 36 point pairs.
template <bool ATT, bool WRAP>
__device__ __forceinline__ void vertex_pair_sums(const float4 *__restrict__ rec, int32_t q0, int32_t q1,
                                                 const float4 *trial, int cnt, const DenseDom &ext, const DenseDom &in,
                                                 bool same, Acc4 &E, Acc4 &I)
{
    // the constants of the loop in VGPRs (an SGPR operand halves the issue rate)
    const DenseDom e{in_vgpr(ext.k), in_vgpr(ext.k2pi), in_vgpr(ext.kim), 0.0f, 0.0f, in_vgpr(ext.k2re),
                     in_vgpr(ext.k2im), 0.0f};
    const DenseDom d{in_vgpr(in.k), in_vgpr(in.k2pi), in_vgpr(in.kim), 0.0f, 0.0f, in_vgpr(in.k2re), in_vgpr(in.k2im),
                     0.0f};
    for (int32_t c0 = q0; c0 < q1; c0 += 6) {
        const float4 Tn = rec[3 * c0 + 1], Tc = rec[3 * c0 + 2];   // test corner: normal, curl
        float4 T0[6];
        float tw[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            T0[q] = rec[3 * (c0 + q)];
            tw[q] = rec[3 * (c0 + q) + 1].w;
        }
        for (int p0 = 0; p0 < cnt; p0 += 6) {
            const float4 Sn = trial[3 * p0 + 1], Sc = trial[3 * p0 + 2];   // trial corner: normal, curl
            const float nn = fmaf(Tn.x, Sn.x, fmaf(Tn.y, Sn.y, Tn.z * Sn.z));
            const float cc = fmaf(Tc.x, Sc.x, fmaf(Tc.y, Sc.y, Tc.z * Sc.z));
            Corner ce{0, 0, 0, 0}, ci{0, 0, 0, 0};
            for (int p = 0; p < 6; ++p) {
                const float4 S0 = trial[3 * (p0 + p)];
                const float sw = trial[3 * (p0 + p) + 1].w;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const float dx = T0[q].x - S0.x, dy = T0[q].y - S0.y, dz = T0[q].z - S0.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    if (r2 > 0.0f) {   // else a point with itself: singular correction
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float r = r2 * rinv;
                        const float ww = T0[q].w * S0.w, ws = tw[q] * sw;
                        const float tK = fmaf(dx, Sn.x, fmaf(dy, Sn.y, dz * Sn.z));
                        const float tKp = fmaf(dx, Tn.x, fmaf(dy, Tn.y, dz * Tn.z));
                        dense_pair<ATT, WRAP>(r, rinv, ww, ws, tK, tKp, e.k, e.k2pi, e.kim, E, ce);
                        if (same) dense_pair<ATT, WRAP>(r, rinv, ww, ws, tK, tKp, d.k, d.k2pi, d.kim, I, ci);
                    }
                }
            }
            corner_done(ce, cc, nn, e.k2re, e.k2im, E);
            if (same) corner_done(ci, cc, nn, d.k2re, d.k2im, I);
        }
    }
    // the records carry 1/(4 pi) on both sides; the kernel has it once
    const float four_pi = 12.566370614359172954f;
    for (Acc4 *A : {&E, &I}) {
        A->vr *= four_pi; A->vi *= four_pi; A->kr *= four_pi; A->ki *= four_pi;
        A->pr *= four_pi; A->pi *= four_pi; A->wr *= four_pi; A->wi *= four_pi;
    }
}

constexpr int STAGE_MAX_DEGREE = 8;   // columns of higher degree: the tile reads global memory

// Trial records of the tile's 16 column vertices (hv[c], -1 past the end) to
// LDS, column c at float4 c * stride (stride = 18 D + 1 for the staged degree
// D: odd, so the 16 columns start in different banks).  Returns false,
// staging nothing, when a column has more than 6 D records; the tile then
// reads them from global memory.  Every thread of the workgroup takes part.
__device__ __forceinline__ bool stage_columns(const float4 *__restrict__ rec, const int32_t *__restrict__ v2t_ptr,
                                              const int64_t *hv, int stride, float4 *srec, int *cnt)
{
    const int tid = threadIdx.y * 16 + threadIdx.x;
    if (tid < 16) cnt[tid] = hv[tid] >= 0 ? 6 * (v2t_ptr[hv[tid] + 1] - v2t_ptr[hv[tid]]) : 0;
    __syncthreads();
    bool fits = true;
    for (int c = 0; c < 16; ++c) fits = fits && 3 * cnt[c] < stride;
    if (fits)
        for (int c = 0; c < 16; ++c) {
            if (hv[c] < 0) continue;
            const int64_t p0 = 6 * int64_t(v2t_ptr[hv[c]]);
            for (int e = tid; e < 3 * cnt[c]; e += 256) srec[c * stride + e] = rec[3 * p0 + e];
        }
    __syncthreads();
    return fits;
}

// Dense matrix, one 16 x 16 tile of vertex pairs per workgroup; the trial
// records of the tile's columns are read from LDS (every one is used by the 16
// rows of the tile) unless one has more than the staged degree.
template <bool ATT, bool WRAP>
__global__ __launch_bounds__(256) void k_assemble_dense(const float4 *__restrict__ rec, const int32_t *__restrict__ v2t_ptr,
                                                        const int32_t *__restrict__ vdom, const DenseDom *__restrict__ doms,
                                                        DenseDom ext, const int32_t *__restrict__ rowD,
                                                        const int32_t *__restrict__ rowN, int64_t NV, int64_t n,
                                                        float2 *__restrict__ A, int stride)
{
    extern __shared__ float4 srec[];
    __shared__ int cnt[16];
    __shared__ int64_t hv[16];
    const int64_t g = int64_t(blockIdx.y) * 16 + threadIdx.y;
    const int64_t h = int64_t(blockIdx.x) * 16 + threadIdx.x;
    const int tid = threadIdx.y * 16 + threadIdx.x;
    if (tid < 16) hv[tid] = int64_t(blockIdx.x) * 16 + tid < NV ? int64_t(blockIdx.x) * 16 + tid : -1;
    __syncthreads();
    const bool staged = stage_columns(rec, v2t_ptr, hv, stride, srec, cnt);
    if (g >= NV || h >= NV) return;
    const int dg = vdom[g];
    const bool same = dg == vdom[h];
    const DenseDom in = doms[dg];
    Acc4 E = {0, 0, 0, 0, 0, 0, 0, 0}, I = {0, 0, 0, 0, 0, 0, 0, 0};
    const int32_t q0 = 6 * v2t_ptr[g], q1 = 6 * v2t_ptr[g + 1];
    if (staged)
        vertex_pair_sums<ATT, WRAP>(rec, q0, q1, srec + threadIdx.x * stride, cnt[threadIdx.x], ext, in, same, E, I);
    else
        vertex_pair_sums<ATT, WRAP>(rec, q0, q1, rec + 3 * int64_t(6 * v2t_ptr[h]), 6 * (v2t_ptr[h + 1] - v2t_ptr[h]),
                                    ext, in, same, E, I);
    const float sV = same ? in.sV : 0.0f, sW = same ? in.sW : 0.0f, s1 = same ? 1.0f : 0.0f;
    const int64_t rD = rowD[g], rN = rowN[g], cD = rowD[h], cN = rowN[h];
    A[rD * n + cD] = make_float2(-(E.kr + s1 * I.kr), -(E.ki + s1 * I.ki));
    A[rD * n + cN] = make_float2(E.vr + sV * I.vr, E.vi + sV * I.vi);
    A[rN * n + cD] = make_float2(E.wr + sW * I.wr, E.wi + sW * I.wi);
    A[rN * n + cN] = make_float2(E.pr + s1 * I.pr, E.pi + s1 * I.pi);
}

// A += singular correction (one thread per CSR entry)
__global__ void k_dense_correction(const int32_t *__restrict__ cptr, const int32_t *__restrict__ ccol,
                                   const double2 *__restrict__ cval, const int32_t *__restrict__ rowD,
                                   const int32_t *__restrict__ rowN, int64_t NV, int64_t n, float2 *__restrict__ A)
{
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= NV) return;
    const int64_t rD = rowD[g], rN = rowN[g];
    for (int32_t e = cptr[g]; e < cptr[g + 1]; ++e) {
        const int32_t h = ccol[e];
        const int64_t cD = rowD[h], cN = rowN[h];
        const int64_t idx[4] = {rD * n + cD, rD * n + cN, rN * n + cD, rN * n + cN};
        for (int b = 0; b < 4; ++b) {
            const float2 a = A[idx[b]];
            const double2 c = cval[4 * e + b];
            A[idx[b]] = make_float2(float(double(a.x) + c.x), float(double(a.y) + c.y));
        }
    }
}

// Device inputs of the entry kernels: vertex records, domain of every vertex,
// per-domain constants and the exterior ones.
struct EntrySetup {
    float4 *rec = nullptr;
    int32_t *vdom = nullptr;
    DenseDom *doms = nullptr;
    DenseDom ext{};
    bool att = false;
    int stride = 0;          // float4 per staged column (18 D + 1 for the staged degree D)
    size_t lds_bytes = 0;    // 16 staged columns
    EntrySetup() = default;
    EntrySetup(const EntrySetup &) = delete;
    EntrySetup &operator=(const EntrySetup &) = delete;
    ~EntrySetup()
    {
        if (rec) dfree(rec);
        if (vdom) dfree(vdom);
        if (doms) dfree(doms);
    }
};

static void entry_setup(bem_problem &p, EntrySetup &E)
{
    const int64_t n_corner = 3 * p.NT;
    dmalloc(reinterpret_cast<void **>(&E.rec), size_t(18 * n_corner) * sizeof(float4));
    k_vertex_points<<<dim3(blocks_1d(6 * n_corner, 256)), dim3(256), 0, p.stream>>>(
        p.d_v2t, n_corner, p.d_area, p.d_normal, p.d_curl, p.d_pts, p.M, E.rec);
    BEM_HIP(hipGetLastError());
    std::vector<int32_t> vdom(p.NV);
    std::vector<DenseDom> doms;
    E.att = p.k0im != 0.0;
    for (size_t j = 0; j < p.doms.size(); ++j) {
        const auto &d = p.doms[j];
        for (int64_t i = 0; i < d.nv; ++i) vdom[d.v_off + i] = int32_t(j);
        doms.push_back(DenseDom{float(d.kre), float(d.kre / (2.0 * M_PI)), float(d.kim), float(d.rho / p.rho0),
                                float(p.rho0 / d.rho), float(d.kre * d.kre - d.kim * d.kim), float(2.0 * d.kre * d.kim),
                                0.0f});
        E.att = E.att || d.kim != 0.0;
    }
    E.ext = DenseDom{float(p.k0re), float(p.k0re / (2.0 * M_PI)), float(p.k0im), 1.0f, 1.0f,
                     float(p.k0re * p.k0re - p.k0im * p.k0im), float(2.0 * p.k0re * p.k0im), 0.0f};
    dmalloc(reinterpret_cast<void **>(&E.vdom), vdom.size() * sizeof(int32_t));
    dmalloc(reinterpret_cast<void **>(&E.doms), doms.size() * sizeof(DenseDom));
    BEM_HIP(hipMemcpyAsync(E.vdom, vdom.data(), vdom.size() * sizeof(int32_t), hipMemcpyHostToDevice, p.stream));
    BEM_HIP(hipMemcpyAsync(E.doms, doms.data(), doms.size() * sizeof(DenseDom), hipMemcpyHostToDevice, p.stream));
    // staged degree: the mesh's largest, at most STAGE_MAX_DEGREE (LDS per
    // workgroup 16 (18 D + 1) float4: 28 KB at D = 6)
    std::vector<int32_t> deg(p.NV, 0);
    for (int64_t i = 0; i < 3 * p.NT; ++i) deg[p.h_tris[i]]++;
    const int maxdeg = p.NV > 0 ? *std::max_element(deg.begin(), deg.end()) : 1;
    const int D = std::max(1, std::min(maxdeg, STAGE_MAX_DEGREE));
    E.stride = 18 * D + 1;
    E.lds_bytes = size_t(16) * E.stride * sizeof(float4);
    BEM_HIP(hipStreamSynchronize(p.stream));
}

void launch_assemble_dense(bem_problem &p)
{
    EntrySetup E;
    entry_setup(p, E);
    const dim3 grid(unsigned((p.NV + 15) / 16), unsigned((p.NV + 15) / 16)), block(16, 16);
#define ASSEMBLE(A, W)                                                                                             \
    k_assemble_dense<A, W><<<grid, block, E.lds_bytes, p.stream>>>(E.rec, p.d_v2t_ptr, E.vdom, E.doms, E.ext, p.d_rowD, \
                                                                   p.d_rowN, p.NV, p.N, p.d_A, E.stride)
    if (E.att) {
        if (p.wrap_phase) ASSEMBLE(true, true); else ASSEMBLE(true, false);
    } else {
        if (p.wrap_phase) ASSEMBLE(false, true); else ASSEMBLE(false, false);
    }
#undef ASSEMBLE
    BEM_HIP(hipGetLastError());
    k_dense_correction<<<dim3(blocks_1d(p.NV, 256)), dim3(256), 0, p.stream>>>(
        p.d_cptr, p.d_ccol, p.d_cval, p.d_rowD, p.d_rowN, p.NV, p.N, p.d_A);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(p.stream));
}

// Entries of hierarchical-matrix blocks: tile (block, 16 row vertices, 16
// column vertices) per workgroup; the 2 x 2 entries of a vertex pair (the same
// sums as k_assemble_dense) go to a (2 m) x (2 n) column-major complex64 block
// in interleaved (vertex, D/N) order: row 2 a + s, column 2 c + t.
template <bool ATT, bool WRAP>
__global__ __launch_bounds__(256) void k_hblock_entries(const float4 *__restrict__ rec,
                                                        const int32_t *__restrict__ v2t_ptr,
                                                        const int32_t *__restrict__ vdom,
                                                        const DenseDom *__restrict__ doms, DenseDom ext,
                                                        const int32_t *__restrict__ perm, const int4 *__restrict__ tiles,
                                                        const HBlock *__restrict__ blocks, float2 *const *__restrict__ out,
                                                        int stride)
{
    extern __shared__ float4 srec[];
    __shared__ int cnt[16];
    __shared__ int64_t hv[16];
    const int4 tl = tiles[blockIdx.x];
    const HBlock B = blocks[tl.x];
    const int m = B.r1 - B.r0, n = B.c1 - B.c0;
    const int a = tl.y * 16 + int(threadIdx.y), c = tl.z * 16 + int(threadIdx.x);
    const int tid = threadIdx.y * 16 + threadIdx.x;
    if (tid < 16) hv[tid] = tl.z * 16 + tid < n ? int64_t(perm[B.c0 + tl.z * 16 + tid]) : -1;
    __syncthreads();
    const bool staged = stage_columns(rec, v2t_ptr, hv, stride, srec, cnt);
    if (a >= m || c >= n) return;
    const int64_t g = perm[B.r0 + a], h = perm[B.c0 + c];
    const int dg = vdom[g];
    const bool same = dg == vdom[h];
    const DenseDom in = doms[dg];
    Acc4 E = {0, 0, 0, 0, 0, 0, 0, 0}, I = {0, 0, 0, 0, 0, 0, 0, 0};
    const int32_t q0 = 6 * v2t_ptr[g], q1 = 6 * v2t_ptr[g + 1];
    if (staged)
        vertex_pair_sums<ATT, WRAP>(rec, q0, q1, srec + threadIdx.x * stride, cnt[threadIdx.x], ext, in, same, E, I);
    else
        vertex_pair_sums<ATT, WRAP>(rec, q0, q1, rec + 3 * int64_t(6 * v2t_ptr[h]), 6 * (v2t_ptr[h + 1] - v2t_ptr[h]),
                                    ext, in, same, E, I);
    const float sV = same ? in.sV : 0.0f, sW = same ? in.sW : 0.0f, s1 = same ? 1.0f : 0.0f;
    float2 *D = out[tl.x];
    const int64_t ld = 2 * int64_t(m);
    D[(2 * int64_t(c)) * ld + 2 * a] = make_float2(-(E.kr + s1 * I.kr), -(E.ki + s1 * I.ki));        // DD
    D[(2 * int64_t(c) + 1) * ld + 2 * a] = make_float2(E.vr + sV * I.vr, E.vi + sV * I.vi);           // DN
    D[(2 * int64_t(c)) * ld + 2 * a + 1] = make_float2(E.wr + sW * I.wr, E.wi + sW * I.wi);           // ND
    D[(2 * int64_t(c) + 1) * ld + 2 * a + 1] = make_float2(E.pr + s1 * I.pr, E.pi + s1 * I.pi);       // NN
}

// Block += singular correction: one thread per (listed block, row vertex); the
// touching pairs of a row vertex whose column vertex lies in the block
__global__ void k_hblock_correction(const int2 *__restrict__ rows, int64_t n_rows, const HBlock *__restrict__ blocks,
                                    float2 *const *__restrict__ out, const int32_t *__restrict__ perm,
                                    const int32_t *__restrict__ iperm, const int32_t *__restrict__ cptr,
                                    const int32_t *__restrict__ ccol, const double2 *__restrict__ cval)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_rows) return;
    const int2 ra = rows[k];   // (block, local row vertex)
    const HBlock B = blocks[ra.x];
    const int64_t m = B.r1 - B.r0, ld = 2 * m;
    const int32_t g = perm[B.r0 + ra.y];
    float2 *D = out[ra.x];
    for (int32_t e = cptr[g]; e < cptr[g + 1]; ++e) {
        const int32_t hc = iperm[ccol[e]];
        if (hc < B.c0 || hc >= B.c1) continue;
        const int64_t c = hc - B.c0;
        const int64_t idx[4] = {(2 * c) * ld + 2 * ra.y, (2 * c + 1) * ld + 2 * ra.y, (2 * c) * ld + 2 * ra.y + 1,
                                (2 * c + 1) * ld + 2 * ra.y + 1};
        for (int b = 0; b < 4; ++b) {
            const float2 v = D[idx[b]];
            const double2 cv = cval[4 * e + b];
            D[idx[b]] = make_float2(float(double(v.x) + cv.x), float(double(v.y) + cv.y));
        }
    }
}

EntryCtx *entry_ctx_create(bem_problem &p)
{
    auto *E = new EntrySetup;
    try {
        entry_setup(p, *E);
    } catch (...) {
        delete E;
        throw;
    }
    return reinterpret_cast<EntryCtx *>(E);
}

void entry_ctx_free(EntryCtx *c) { delete reinterpret_cast<EntrySetup *>(c); }

void launch_hblock_entries(bem_problem &p, EntryCtx *ctx, const int32_t *perm, const int4 *tiles, int64_t n_tiles,
                           const HBlock *blocks, float2 *const *out)
{
    if (n_tiles == 0) return;
    const EntrySetup &E = *reinterpret_cast<EntrySetup *>(ctx);
    const dim3 block(16, 16);
    for (int64_t t0 = 0; t0 < n_tiles; t0 += (int64_t(1) << 30)) {
        const unsigned nt = unsigned(std::min<int64_t>(n_tiles - t0, int64_t(1) << 30));
#define ENTRIES(A, W)                                                                                              \
    k_hblock_entries<A, W><<<dim3(nt), block, E.lds_bytes, p.stream>>>(E.rec, p.d_v2t_ptr, E.vdom, E.doms, E.ext, perm, \
                                                                       tiles + t0, blocks, out, E.stride)
        if (E.att) {
            if (p.wrap_phase) ENTRIES(true, true); else ENTRIES(true, false);
        } else {
            if (p.wrap_phase) ENTRIES(false, true); else ENTRIES(false, false);
        }
#undef ENTRIES
        BEM_HIP(hipGetLastError());
    }
    BEM_HIP(hipStreamSynchronize(p.stream));
}

void launch_hblock_correction(bem_problem &p, const int2 *rows, int64_t n_rows, const HBlock *blocks,
                              float2 *const *out, const int32_t *perm, const int32_t *iperm)
{
    if (n_rows == 0) return;
    k_hblock_correction<<<dim3(blocks_1d(n_rows, 256)), dim3(256), 0, p.stream>>>(rows, n_rows, blocks, out, perm, iperm,
                                                                                 p.d_cptr, p.d_ccol, p.d_cval);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(p.stream));
}

// ---------------------------------------------------------------------------
// Low-rank blocks by adaptive cross approximation with partial pivoting
// ---------------------------------------------------------------------------
// The entries of a block are computed on demand, one residual row and one
// residual column per term (the vertex-pair sums above), so a block of m x n
// vertices and rank r costs r (m + n) vertex pairs instead of the m n of the
// complete-pivoting build.  One wave (a workgroup of 64 lanes) per block; lane
// l owns the vertices l, l + 64, ... of each side and the two interleaved rows
// (or columns) of each.
//
// Term k: the residual of row i is computed, its largest entry in an unused
// column j is the pivot, v_k = residual row / pivot and u_k = residual of
// column j; the next row is the largest entry of u_k in an unused row.  The
// Frobenius norm of S_k = sum u_l v_l is updated as
//   |S_k|^2 = |S_{k-1}|^2 + 2 Re sum_{l<k} <u_l, u_k> <v_k, v_l> + |u_k|^2 |v_k|^2,
// and the terms stop when |u_k| |v_k| <= eps |S_k|.  That test sees only the
// rows and columns pivoted so far, so it is confirmed on ACAP_CHECK_ROWS unused
// rows spread over the block (from a hash of the block and the rank), half of
// them D rows and half N rows: their residual, scaled to all unused rows, must
// be within eps |S_k|, else the worst of them is the next pivot row.  Both
// kinds are sampled because on coplanar clusters (the faces of a slab or a
// box) the double-layer entries vanish, the block splits into a D-row part
// (V) and an N-row part (W) with no row or column in common, and pivots taken
// from one part never reach the other.  Rank -1 when the cap comes first (the
// block is then stored dense).  Every decision is taken on wave-uniform values
// (shuffle reductions in a fixed order), so the result is deterministic.

constexpr int ACAP_CHECK_ROWS = 4;   // even: half D rows, half N rows

struct AcapIn {
    const float4 *rec;
    const int32_t *v2t_ptr, *vdom, *perm;
    const DenseDom *doms;
    DenseDom ext;
};

// entry (row 2 a + s, column 2 c + t) of a vertex pair, as k_hblock_entries
// stores it
__device__ __forceinline__ float2 acap_entry(const Acc4 &E, const Acc4 &I, const DenseDom &in, bool same, int s, int t)
{
    const float sV = same ? in.sV : 0.0f, sW = same ? in.sW : 0.0f, s1 = same ? 1.0f : 0.0f;
    if (s == 0)
        return t == 0 ? make_float2(-(E.kr + s1 * I.kr), -(E.ki + s1 * I.ki)) : make_float2(E.vr + sV * I.vr, E.vi + sV * I.vi);
    return t == 0 ? make_float2(E.wr + sW * I.wr, E.wi + sW * I.wi) : make_float2(E.pr + s1 * I.pr, E.pi + s1 * I.pi);
}

template <bool ATT, bool WRAP>
__device__ __forceinline__ void acap_pair(const AcapIn &a, int32_t g, int32_t h, Acc4 &E, Acc4 &I, DenseDom &in,
                                          bool &same)
{
    const int dg = a.vdom[g];
    same = dg == a.vdom[h];
    in = a.doms[dg];
    E = Acc4{0, 0, 0, 0, 0, 0, 0, 0};
    I = Acc4{0, 0, 0, 0, 0, 0, 0, 0};
    vertex_pair_sums<ATT, WRAP>(a.rec, 6 * a.v2t_ptr[g], 6 * a.v2t_ptr[g + 1], a.rec + 3 * int64_t(6 * a.v2t_ptr[h]),
                                6 * (a.v2t_ptr[h + 1] - a.v2t_ptr[h]), a.ext, in, same, E, I);
}

// e - x y (complex)
__device__ __forceinline__ float2 acap_msub(float2 e, float2 x, float2 y)
{
    return make_float2(e.x - fmaf(x.x, y.x, -x.y * y.y), e.y - fmaf(x.x, y.y, x.y * y.x));
}

__device__ __forceinline__ double acap_wsum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// largest v over the wave (ties: the smaller index), with its index and value
__device__ __forceinline__ void acap_argmax(float &v, int &idx, float2 &z)
{
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(idx, off);
        const float zx = __shfl_xor(z.x, off), zy = __shfl_xor(z.y, off);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
            z = make_float2(zx, zy);
        }
    }
}

// out[0 .. 2 n) = residual of block row i after k terms
template <bool ATT, bool WRAP>
__device__ void acap_row(const AcapIn &a, const HBlock &B, const float2 *U, const float2 *V, int64_t m2, int64_t n2,
                         int i, int k, float2 *out)
{
    const int32_t g = a.perm[B.r0 + (i >> 1)];
    const int s = i & 1, n = B.c1 - B.c0;
    for (int c = int(threadIdx.x); c < n; c += 64) {
        Acc4 E, I;
        DenseDom in;
        bool same;
        acap_pair<ATT, WRAP>(a, g, a.perm[B.c0 + c], E, I, in, same);
        float2 e0 = acap_entry(E, I, in, same, s, 0), e1 = acap_entry(E, I, in, same, s, 1);
#pragma unroll 8
        for (int l = 0; l < k; ++l) {
            const float2 ul = U[int64_t(l) * m2 + i];
            e0 = acap_msub(e0, ul, V[int64_t(l) * n2 + 2 * c]);
            e1 = acap_msub(e1, ul, V[int64_t(l) * n2 + 2 * c + 1]);
        }
        out[2 * c] = e0;
        out[2 * c + 1] = e1;
    }
}

// out[0 .. 2 m) = residual of block column j after k terms
template <bool ATT, bool WRAP>
__device__ void acap_col(const AcapIn &a, const HBlock &B, const float2 *U, const float2 *V, int64_t m2, int64_t n2,
                         int j, int k, float2 *out)
{
    const int32_t h = a.perm[B.c0 + (j >> 1)];
    const int t = j & 1, m = B.r1 - B.r0;
    for (int r = int(threadIdx.x); r < m; r += 64) {
        Acc4 E, I;
        DenseDom in;
        bool same;
        acap_pair<ATT, WRAP>(a, a.perm[B.r0 + r], h, E, I, in, same);
        float2 e0 = acap_entry(E, I, in, same, 0, t), e1 = acap_entry(E, I, in, same, 1, t);
#pragma unroll 8
        for (int l = 0; l < k; ++l) {
            const float2 vl = V[int64_t(l) * n2 + j];
            e0 = acap_msub(e0, U[int64_t(l) * m2 + 2 * r], vl);
            e1 = acap_msub(e1, U[int64_t(l) * m2 + 2 * r + 1], vl);
        }
        out[2 * r] = e0;
        out[2 * r + 1] = e1;
    }
}

template <bool ATT, bool WRAP>
__global__ __launch_bounds__(64) void k_aca_partial(const AcapIn a, const HBlock *__restrict__ blocks,
                                                    const int32_t *__restrict__ ids, float2 *const *__restrict__ Uo,
                                                    float2 *const *__restrict__ Vo, const int32_t *__restrict__ kmax,
                                                    float eps, int32_t *__restrict__ rank_out)
{
    extern __shared__ unsigned char used[];   // [2 m] rows, then [2 n] columns
    __shared__ int pick[ACAP_CHECK_ROWS];
    const int lane = threadIdx.x;
    const int32_t bid = ids[blockIdx.x];
    const HBlock B = blocks[bid];
    const int m = B.r1 - B.r0, n = B.c1 - B.c0, m2 = 2 * m, n2 = 2 * n;
    unsigned char *usedr = used, *usedc = used + m2;
    float2 *U = Uo[blockIdx.x], *V = Vo[blockIdx.x];
    const int K = kmax[blockIdx.x];
    for (int r = lane; r < m2 + n2; r += 64) used[r] = 0;
    __syncthreads();
    const double eps2 = double(eps) * double(eps);
    double S2 = 0.0;
    int k = 0, i = 0, skips = 0, rows_used = 0, result = -1;
    for (;;) {
        float2 *vk = V + int64_t(k) * n2;
        acap_row<ATT, WRAP>(a, B, U, V, m2, n2, i, k, vk);
        if (lane == 0) usedr[i] = 1;
        ++rows_used;
        __syncthreads();
        // pivot: the largest entry of the residual row in an unused column
        float best = -1.0f;
        int j = 0x7fffffff;
        float2 piv = make_float2(0.0f, 0.0f);
        for (int c = lane; c < n; c += 64)
            for (int t = 0; t < 2; ++t) {
                const int cc = 2 * c + t;
                if (usedc[cc]) continue;
                const float2 z = vk[cc];
                const float q = fmaf(z.x, z.x, z.y * z.y);
                if (q > best) {
                    best = q;
                    j = cc;
                    piv = z;
                }
            }
        acap_argmax(best, j, piv);
        if (!(best > 0.0f)) {
            // no usable pivot in this row: the next unused row
            if (lane == 0) {
                int nxt = -1;
                for (int q = 1; q <= m2 && nxt < 0; ++q)
                    if (!usedr[(i + q) % m2]) nxt = (i + q) % m2;
                pick[0] = nxt;
            }
            __syncthreads();
            const int nxt = pick[0];
            __syncthreads();
            if (nxt < 0 || ++skips > 8) {
                result = k;
                break;
            }
            i = nxt;
            continue;
        }
        const float pd = fmaf(piv.x, piv.x, piv.y * piv.y);
        const float2 inv = make_float2(piv.x / pd, -piv.y / pd);
        for (int c = lane; c < n; c += 64) {
            const float2 z0 = vk[2 * c], z1 = vk[2 * c + 1];
            vk[2 * c] = make_float2(fmaf(z0.x, inv.x, -z0.y * inv.y), fmaf(z0.x, inv.y, z0.y * inv.x));
            vk[2 * c + 1] = make_float2(fmaf(z1.x, inv.x, -z1.y * inv.y), fmaf(z1.x, inv.y, z1.y * inv.x));
        }
        float2 *uk = U + int64_t(k) * m2;
        acap_col<ATT, WRAP>(a, B, U, V, m2, n2, j, k, uk);
        if (lane == 0) usedc[j] = 1;
        // norms of the new term and its products with the earlier ones (own entries)
        double nu = 0.0, nv = 0.0;
        for (int r = lane; r < m2; r += 64) {
            const float2 z = uk[r];
            nu += double(z.x) * z.x + double(z.y) * z.y;
        }
        for (int c = lane; c < n2; c += 64) {
            const float2 z = vk[c];
            nv += double(z.x) * z.x + double(z.y) * z.y;
        }
        nu = acap_wsum(nu);
        nv = acap_wsum(nv);
        // four earlier terms at a time (independent loads and reductions)
        double cross = 0.0;
        for (int l0 = 0; l0 < k; l0 += 4) {
            double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0}, br[4] = {0, 0, 0, 0}, bi[4] = {0, 0, 0, 0};
            const int nl = min(4, k - l0);
            for (int r = lane; r < m2; r += 64) {   // <u_l, u_k>
                const float2 y = uk[r];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < nl) {
                        const float2 x = U[int64_t(l0 + q) * m2 + r];
                        ar[q] += double(x.x) * y.x + double(x.y) * y.y;
                        ai[q] += double(x.x) * y.y - double(x.y) * y.x;
                    }
            }
            for (int c = lane; c < n2; c += 64) {   // <v_k, v_l>
                const float2 x = vk[c];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < nl) {
                        const float2 y = V[int64_t(l0 + q) * n2 + c];
                        br[q] += double(x.x) * y.x + double(x.y) * y.y;
                        bi[q] += double(x.x) * y.y - double(x.y) * y.x;
                    }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ar[q] = acap_wsum(ar[q]);
                ai[q] = acap_wsum(ai[q]);
                br[q] = acap_wsum(br[q]);
                bi[q] = acap_wsum(bi[q]);
            }
            for (int q = 0; q < nl; ++q) cross += ar[q] * br[q] - ai[q] * bi[q];
        }
        S2 += 2.0 * cross + nu * nv;
        ++k;
        __syncthreads();   // the new term and the column flag, for every lane
        if (nu * nv <= eps2 * S2) {
            if (k >= K) {
                result = k;
                break;
            }
            // confirm on unused rows; the slot of term k is scratch
            if (lane == 0)
                for (int q = 0; q < ACAP_CHECK_ROWS; ++q) {
                    uint32_t h = uint32_t(bid) * 0x9E3779B1u ^ uint32_t(k) * 0x85EBCA77u ^ uint32_t(q + 1) * 0xC2B2AE3Du;
                    h ^= h >> 15;
                    h *= 0x2C1B3C6Du;
                    h ^= h >> 12;
                    int r = -1;
                    for (int o = 0; o < m && r < 0; ++o) {   // rows of parity q & 1
                        const int c = 2 * int((h + uint32_t(o)) % uint32_t(m)) + (q & 1);
                        bool dup = usedr[c] != 0;
                        for (int e = 0; e < q; ++e) dup = dup || pick[e] == c;
                        if (!dup) r = c;
                    }
                    pick[q] = r;
                }
            __syncthreads();
            int chk[ACAP_CHECK_ROWS];
            for (int q = 0; q < ACAP_CHECK_ROWS; ++q) chk[q] = pick[q];
            __syncthreads();
            double sum = 0.0, worst = -1.0;
            int wr = -1, nchk = 0;
            float2 *tmp = V + int64_t(k) * n2;
            for (int q = 0; q < ACAP_CHECK_ROWS; ++q) {
                if (chk[q] < 0) continue;
                acap_row<ATT, WRAP>(a, B, U, V, m2, n2, chk[q], k, tmp);
                double e = 0.0;
                for (int c = lane; c < n2; c += 64) {
                    const float2 z = tmp[c];
                    e += double(z.x) * z.x + double(z.y) * z.y;
                }
                e = acap_wsum(e);
                sum += e;
                ++nchk;
                if (e > worst) {
                    worst = e;
                    wr = chk[q];
                }
            }
            if (nchk == 0 || sum * double(m2 - rows_used) / double(nchk) <= eps2 * S2) {
                result = k;
                break;
            }
            i = wr;
            continue;
        }
        if (k >= K) {
            result = -1;
            break;
        }
        // next row: the largest entry of u_{k-1} in an unused row
        float bu = -1.0f;
        int ni = 0x7fffffff;
        float2 zu = make_float2(0.0f, 0.0f);
        for (int r = lane; r < m; r += 64)
            for (int s = 0; s < 2; ++s) {
                const int rr = 2 * r + s;
                if (usedr[rr]) continue;
                const float2 z = uk[rr];
                const float q = fmaf(z.x, z.x, z.y * z.y);
                if (q > bu) {
                    bu = q;
                    ni = rr;
                    zu = z;
                }
            }
        acap_argmax(bu, ni, zu);
        if (ni == 0x7fffffff) {   // every row used
            result = k;
            break;
        }
        i = ni;
    }
    if (lane == 0) rank_out[blockIdx.x] = result;
}

void launch_aca_partial(bem_problem &p, EntryCtx *ctx, const int32_t *perm, const HBlock *blocks, const int32_t *ids,
                        int n, float2 *const *U, float2 *const *V, const int32_t *kmax, float eps, int32_t *rank,
                        int max_side)
{
    if (n == 0) return;
    const EntrySetup &E = *reinterpret_cast<EntrySetup *>(ctx);
    const AcapIn a{E.rec, p.d_v2t_ptr, E.vdom, perm, E.doms, E.ext};
    const size_t lds = size_t(4) * size_t(max_side);   // row and column flags of the largest block
#define ACAP(A, W) k_aca_partial<A, W><<<dim3(unsigned(n)), dim3(64), lds, p.stream>>>(a, blocks, ids, U, V, kmax, eps, rank)
    if (E.att) {
        if (p.wrap_phase) ACAP(true, true); else ACAP(true, false);
    } else {
        if (p.wrap_phase) ACAP(false, true); else ACAP(false, false);
    }
#undef ACAP
    BEM_HIP(hipGetLastError());
}

// y = A x, complex64 matrix, FP64 vectors and FP64 accumulation.  One wave per
// GEMV_ROWS rows; lanes stride over the columns two entries at a time (16-byte
// loads of A), GEMV_UNROLL column strides loaded before they are used (16
// loads of A in flight per lane), partial sums reduced across the wave in a
// fixed order.  Eight rows per wave also halve the re-reads of x against four.
constexpr int GEMV_ROWS = 8;
constexpr int GEMV_UNROLL = 2;

__global__ __launch_bounds__(256) void k_gemv(const float2 *__restrict__ A, const double2 *__restrict__ x, int64_t n,
                                              double2 *__restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t r0 = wave * GEMV_ROWS;
    if (r0 >= n) return;
    double ar[GEMV_ROWS], ai[GEMV_ROWS];
    const float2 *row[GEMV_ROWS];
#pragma unroll
    for (int k = 0; k < GEMV_ROWS; ++k) {
        ar[k] = ai[k] = 0.0;
        row[k] = A + (r0 + k < n ? r0 + k : n - 1) * n;   // rows past n repeat the last (not stored)
    }
    const int64_t npair = n / 2;
    int64_t c2 = lane;
    for (; c2 + 64 * (GEMV_UNROLL - 1) < npair; c2 += 64 * GEMV_UNROLL) {
        float4 a[GEMV_UNROLL][GEMV_ROWS];
        double2 x0[GEMV_UNROLL], x1[GEMV_UNROLL];
#pragma unroll
        for (int u = 0; u < GEMV_UNROLL; ++u) {
#pragma unroll
            for (int k = 0; k < GEMV_ROWS; ++k) a[u][k] = load_streamed(row[k] + 2 * (c2 + 64 * u));
            x0[u] = x[2 * (c2 + 64 * u)];
            x1[u] = x[2 * (c2 + 64 * u) + 1];
        }
#pragma unroll
        for (int u = 0; u < GEMV_UNROLL; ++u)
#pragma unroll
            for (int k = 0; k < GEMV_ROWS; ++k) {
                const float4 v = a[u][k];
                ar[k] += double(v.x) * x0[u].x - double(v.y) * x0[u].y + double(v.z) * x1[u].x - double(v.w) * x1[u].y;
                ai[k] += double(v.x) * x0[u].y + double(v.y) * x0[u].x + double(v.z) * x1[u].y + double(v.w) * x1[u].x;
            }
    }
    for (; c2 < npair; c2 += 64) {
        const double2 x0 = x[2 * c2], x1 = x[2 * c2 + 1];
#pragma unroll
        for (int k = 0; k < GEMV_ROWS; ++k) {
            const float4 v = load_streamed(row[k] + 2 * c2);
            ar[k] += double(v.x) * x0.x - double(v.y) * x0.y + double(v.z) * x1.x - double(v.w) * x1.y;
            ai[k] += double(v.x) * x0.y + double(v.y) * x0.x + double(v.z) * x1.y + double(v.w) * x1.x;
        }
    }
    if ((n & 1) && lane == 0) {
        const double2 xl = x[n - 1];
#pragma unroll
        for (int k = 0; k < GEMV_ROWS; ++k) {
            const float2 v = row[k][n - 1];
            ar[k] += double(v.x) * xl.x - double(v.y) * xl.y;
            ai[k] += double(v.x) * xl.y + double(v.y) * xl.x;
        }
    }
#pragma unroll
    for (int k = 0; k < GEMV_ROWS; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            ar[k] += __shfl_xor(ar[k], off);
            ai[k] += __shfl_xor(ai[k], off);
        }
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < GEMV_ROWS; ++k)
            if (r0 + k < n) y[r0 + k] = make_double2(ar[k], ai[k]);
}

void launch_gemv(bem_problem &p, const double2 *x, double2 *y)
{
    const int64_t waves = (p.N + GEMV_ROWS - 1) / GEMV_ROWS;
    const int64_t threads = waves * 64;
    k_gemv<<<dim3(blocks_1d(threads, 256)), dim3(256), 0, p.stream>>>(p.d_A, x, p.N, y);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
