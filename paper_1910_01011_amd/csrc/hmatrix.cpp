// Hierarchical matrix of the PMCHWT operator (the compression the paper uses
// to go beyond dense storage, there with Bempp's H-matrices).
//
// Build:
//  * cluster tree: clusters over several boundaries are split between
//    boundaries; a cluster of one boundary is bisected recursively at the
//    median of the longest axis of its bounding box, down to `leaf` vertices;
//    the vertex order is permuted so that every cluster is a range;
//  * block tree: a pair of clusters (s, t) is admissible when
//    max(diam s, diam t) <= eta dist(s, t); admissible pairs become low-rank
//    blocks, pairs of leaves dense blocks, others are split.  A cluster's box
//    bounds the supports of its vertices' P1 functions (every triangle at each
//    vertex), not the vertices alone: two vertices whose functions meet on
//    touching triangles then lie in clusters at distance 0, which are never
//    admissible;
//  * low-rank blocks: adaptive cross approximation with partial pivoting to
//    the relative tolerance eps (Frobenius norm, confirmed on sampled rows),
//    the entries of each pivot row and column computed on demand on the GPU
//    (the far-field vertex-pair sums of the dense assembly), in batches; a
//    block whose rank would not halve its storage is kept dense;
//  * dense blocks: every vertex-pair entry, plus the FP64 singular correction.
//    The build counts the entries of the singular pattern that fall in
//    low-rank blocks and fails unless there are none.
// Apply: reorder x, one workgroup per block writes its products, each row sums
// its blocks' products in a fixed order (no atomics; deterministic).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <memory>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "bem_internal.h"

namespace bem {

void launch_aca(hipStream_t s, const HBlock *blocks, const int32_t *ids, int n, float2 *const *R, float2 *const *U,
                float2 *const *V, const int32_t *kmax, float eps, int32_t *rank);
void launch_copy_list(hipStream_t s, const float2 *const *src, float2 *const *dst, const int64_t *count, int n);
void launch_h_apply(hipStream_t s, const HBlock *blocks, int n_blocks, const int32_t *perm, const int32_t *rowD,
                    const int32_t *rowN, const int32_t *rowptr, const int32_t *rowz, int64_t NV, const double2 *x,
                    double2 *xp, double2 *z, double2 *y);

namespace {

constexpr int HK_CAP = 128;                       // largest rank kept (LDS of the apply kernel)
constexpr int HBLOCK_MAX_SIDE = 512;              // vertices on a side of a low-rank block
constexpr int64_t ACA_BATCH_BYTES = int64_t(4) << 30;   // dense scratch of one batch of far blocks
// U and V scratch of one batch of the partially pivoted build: large (up to
// 64 GB, at most half the free device memory), so that the long cross
// approximations of the largest blocks (one wave each) overlap the many short
// ones in a single launch
constexpr int64_t ACAP_BATCH_MAX = int64_t(64) << 30;
constexpr int64_t ACAP_BATCH_MIN = int64_t(4) << 30;

struct Cluster {
    int32_t b, e;          // range in the permuted order
    double lo[3], hi[3];   // bounding box of the supports of its vertices
    int32_t child[2];
};

// Cluster tree (vertex permutation and clusters) and block tree (blocks with
// their row and column ranges, and which of them are admissible).
struct HTree {
    std::vector<int32_t> perm;
    std::vector<Cluster> cl;
    std::vector<HBlock> blocks;
    std::vector<char> lowrank;
};

struct DevMem {
    void *p = nullptr;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem()
    {
        if (p) dfree(p);
    }
    template <typename T>
    T *alloc(size_t n)
    {
        dmalloc(reinterpret_cast<void **>(&p), std::max<size_t>(1, n) * sizeof(T));
        return static_cast<T *>(p);
    }
};

template <typename T>
T *upload(const std::vector<T> &h, DevMem &m, hipStream_t s)
{
    T *d = m.alloc<T>(h.size());
    if (!h.empty()) BEM_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

double diam(const Cluster &c)
{
    double s = 0;
    for (int d = 0; d < 3; ++d) s += (c.hi[d] - c.lo[d]) * (c.hi[d] - c.lo[d]);
    return std::sqrt(s);
}

double dist(const Cluster &a, const Cluster &b)
{
    double s = 0;
    for (int d = 0; d < 3; ++d) {
        const double g = std::max({0.0, a.lo[d] - b.hi[d], b.lo[d] - a.hi[d]});
        s += g * g;
    }
    return std::sqrt(s);
}

// Bounding box of the support of every vertex's P1 function: the vertices of
// all triangles at that vertex.  [NV][6] = (lo, hi).
std::vector<double> support_boxes(const bem_problem &p)
{
    std::vector<double> box(6 * size_t(p.NV));
    for (int64_t i = 0; i < p.NV; ++i)
        for (int d = 0; d < 3; ++d) box[6 * i + d] = box[6 * i + 3 + d] = p.h_verts[3 * size_t(i) + d];
    for (int64_t t = 0; t < p.NT; ++t)
        for (int a = 0; a < 3; ++a) {
            double *b = &box[6 * size_t(p.h_tris[3 * t + a])];
            for (int c = 0; c < 3; ++c) {
                const double *x = &p.h_verts[3 * size_t(p.h_tris[3 * t + c])];
                for (int d = 0; d < 3; ++d) {
                    b[d] = std::min(b[d], x[d]);
                    b[3 + d] = std::max(b[3 + d], x[d]);
                }
            }
        }
    return box;
}

HTree plan_tree(const bem_problem &p, int leaf, double eta, int max_side)
{
    const int64_t NV = p.NV;
    const std::vector<double> sbox = support_boxes(p);
    HTree T;
    std::vector<int32_t> &perm = T.perm;
    std::vector<Cluster> &cl = T.cl;
    perm.resize(NV);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<int32_t> stack;
    const auto make = [&](int32_t b, int32_t e) {
        Cluster c{};
        c.b = b;
        c.e = e;
        for (int d = 0; d < 3; ++d) {
            c.lo[d] = 1e300;
            c.hi[d] = -1e300;
        }
        for (int32_t i = b; i < e; ++i)
            for (int d = 0; d < 3; ++d) {
                c.lo[d] = std::min(c.lo[d], sbox[6 * size_t(perm[i]) + d]);
                c.hi[d] = std::max(c.hi[d], sbox[6 * size_t(perm[i]) + 3 + d]);
            }
        c.child[0] = c.child[1] = -1;
        cl.push_back(c);
        return int32_t(cl.size() - 1);
    };
    // first vertex of every boundary but the first (the vertices of a boundary
    // are a contiguous range of the original order)
    std::vector<int32_t> starts;
    for (size_t j = 1; j < p.doms.size(); ++j) starts.push_back(int32_t(p.doms[j].v_off));
    stack.push_back(make(0, int32_t(NV)));
    while (!stack.empty()) {
        const int32_t ci = stack.back();
        stack.pop_back();
        const Cluster c = cl[ci];
        // a cluster over several boundaries is split between two of them (the
        // boundary start nearest its middle), at any size: every block then
        // couples one boundary with one boundary, a single smooth kernel
        // sum that the partially pivoted cross approximation samples
        // uniformly.  Such clusters come from boundary splits alone, so the
        // permutation is still the identity on them.
        int32_t mid = -1;
        for (int32_t st : starts)
            if (st > c.b && st < c.e &&
                (mid < 0 || std::abs(2 * int64_t(st) - c.b - c.e) < std::abs(2 * int64_t(mid) - c.b - c.e)))
                mid = st;
        if (mid < 0) {
            if (c.e - c.b <= leaf) continue;
            int ax = 0;
            for (int d = 1; d < 3; ++d)
                if (c.hi[d] - c.lo[d] > c.hi[ax] - c.lo[ax]) ax = d;
            mid = c.b + (c.e - c.b) / 2;
            std::nth_element(perm.begin() + c.b, perm.begin() + mid, perm.begin() + c.e, [&](int32_t u, int32_t v) {
                const double xu = p.h_verts[3 * size_t(u) + ax], xv = p.h_verts[3 * size_t(v) + ax];
                return xu < xv || (xu == xv && u < v);
            });
        }
        const int32_t c0 = make(c.b, mid), c1 = make(mid, c.e);
        cl[ci].child[0] = c0;
        cl[ci].child[1] = c1;
        stack.push_back(c0);
        stack.push_back(c1);
    }
    std::vector<std::pair<int32_t, int32_t>> todo{{0, 0}};
    while (!todo.empty()) {
        const auto [a, b] = todo.back();
        todo.pop_back();
        const Cluster &A = cl[a], &B = cl[b];
        // admissible pairs larger than max_side vertices on a side are split
        // further: each block's cross approximation runs in one workgroup, so
        // bounded blocks keep the whole chip busy
        const bool adm = std::max(diam(A), diam(B)) <= eta * dist(A, B) && A.e - A.b <= max_side &&
                         B.e - B.b <= max_side;
        const bool la = A.child[0] < 0, lb = B.child[0] < 0;
        if (adm || (la && lb)) {
            HBlock hb{};
            hb.r0 = A.b;
            hb.r1 = A.e;
            hb.c0 = B.b;
            hb.c1 = B.e;
            hb.rank = -1;
            T.blocks.push_back(hb);
            T.lowrank.push_back(adm ? 1 : 0);
        } else if (la) {
            todo.push_back({a, B.child[0]});
            todo.push_back({a, B.child[1]});
        } else if (lb) {
            todo.push_back({A.child[0], b});
            todo.push_back({A.child[1], b});
        } else {
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) todo.push_back({A.child[i], B.child[j]});
        }
    }
    return T;
}

int64_t touching_in_lowrank(const HTree &T, int64_t NV, const std::vector<int32_t> &cptr,
                            const std::vector<int32_t> &ccol)
{
    std::vector<int32_t> iperm(NV);
    for (int64_t i = 0; i < NV; ++i) iperm[T.perm[i]] = int32_t(i);
    int64_t n = 0;
    for (size_t i = 0; i < T.blocks.size(); ++i) {
        if (!T.lowrank[i]) continue;
        const HBlock &hb = T.blocks[i];
        for (int32_t r = hb.r0; r < hb.r1; ++r) {
            const int32_t g = T.perm[r];
            for (int32_t k = cptr[g]; k < cptr[g + 1]; ++k) {
                const int32_t c = iperm[ccol[k]];
                n += (c >= hb.c0 && c < hb.c1) ? 1 : 0;
            }
        }
    }
    return n;
}

}  // namespace

struct HMatrix {
    std::vector<HBlock> blocks;
    std::vector<void *> pools;   // device storage of the blocks
    HBlock *d_blocks = nullptr;
    int32_t *d_perm = nullptr, *d_rowptr = nullptr, *d_rowz = nullptr;
    double2 *d_xp = nullptr, *d_z = nullptr;
    int64_t z_len = 0;
    bem_hmatrix_info info{};
    ~HMatrix()
    {
        for (void *q : pools)
            if (q) dfree(q);
        void *ptrs[] = {d_blocks, d_perm, d_rowptr, d_rowz, d_xp, d_z};
        for (void *q : ptrs)
            if (q) dfree(q);
    }
};

void hmatrix_free(HMatrix *h) { delete h; }

static HMatrix *build(bem_problem &p, double eps, int leaf, double eta, int max_side)
{
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t NV = p.NV;
    hipStream_t s = p.stream;
    HTree T = plan_tree(p, leaf, eta, max_side);
    std::vector<int32_t> &perm = T.perm;
    {
        // every entry of the singular pattern must lie in a dense block (that
        // is where the FP64 correction is added)
        std::vector<int32_t> cptr(NV + 1), ccol(std::max<int64_t>(1, p.nnz));
        BEM_HIP(hipMemcpyAsync(cptr.data(), p.d_cptr, cptr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (p.nnz > 0)
            BEM_HIP(hipMemcpyAsync(ccol.data(), p.d_ccol, size_t(p.nnz) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        const int64_t bad = touching_in_lowrank(T, NV, cptr, ccol);
        if (bad != 0)
            throw Error{BEM_ERR_DEVICE, "hierarchical matrix: " + std::to_string(bad) +
                                            " singular-pattern entries in low-rank blocks"};
    }
    std::vector<int32_t> iperm(NV);
    for (int64_t i = 0; i < NV; ++i) iperm[perm[i]] = int32_t(i);
    auto H = std::make_unique<HMatrix>();
    H->blocks = std::move(T.blocks);
    std::vector<char> lowrank = std::move(T.lowrank);
    const int nb = int(H->blocks.size());
    // product offsets and the per-row lists
    int64_t zl = 0;
    for (auto &hb : H->blocks) {
        hb.zoff = zl;
        zl += 2 * int64_t(hb.r1 - hb.r0);
    }
    if (zl >= (int64_t(1) << 31)) throw Error{BEM_ERR_UNSUPPORTED, "hierarchical matrix: too many block products"};
    H->z_len = zl;
    std::vector<int32_t> rowptr(2 * NV + 1, 0), rowz(zl);
    for (const auto &hb : H->blocks)
        for (int64_t r = 2 * int64_t(hb.r0); r < 2 * int64_t(hb.r1); ++r) rowptr[r + 1]++;
    for (int64_t r = 0; r < 2 * NV; ++r) rowptr[r + 1] += rowptr[r];
    {
        std::vector<int32_t> fill(rowptr.begin(), rowptr.end() - 1);
        for (const auto &hb : H->blocks)
            for (int64_t a = 0; a < 2 * int64_t(hb.r1 - hb.r0); ++a)
                rowz[fill[2 * int64_t(hb.r0) + a]++] = int32_t(hb.zoff + a);
    }
    // device copies that live with the matrix (owned by H)
    const auto own = [&](auto &dst, const auto &h) {
        using T = typename std::decay_t<decltype(h)>::value_type;
        dmalloc(reinterpret_cast<void **>(&dst), std::max<size_t>(1, h.size()) * sizeof(T));
        if (!h.empty()) BEM_HIP(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    };
    own(H->d_perm, perm);
    own(H->d_rowptr, rowptr);
    own(H->d_rowz, rowz);
    dmalloc(reinterpret_cast<void **>(&H->d_xp), size_t(2 * NV) * sizeof(double2));
    dmalloc(reinterpret_cast<void **>(&H->d_z), size_t(std::max<int64_t>(1, zl)) * sizeof(double2));
    DevMem m_iperm;
    int32_t *d_iperm = upload(iperm, m_iperm, s);

    // dense storage size and low-rank rank caps
    std::vector<int> far_ids, dense_ids;
    for (int i = 0; i < nb; ++i) (lowrank[i] ? far_ids : dense_ids).push_back(i);
    H->info.n_admissible = int64_t(far_ids.size());
    const auto mn = [&](int i) {
        const auto &hb = H->blocks[i];
        return std::make_pair(2 * int64_t(hb.r1 - hb.r0), 2 * int64_t(hb.c1 - hb.c0));
    };
    const auto kcap = [&](int i) {
        const auto [m2, n2] = mn(i);
        // a rank-k block stores k (m2 + n2) values: keep it only if below m2 n2 / 2
        return int(std::min<int64_t>(HK_CAP, std::max<int64_t>(1, m2 * n2 / (2 * (m2 + n2)))));
    };
    // far blocks: entries into scratch, ACA, compaction; batches by scratch size
    std::sort(far_ids.begin(), far_ids.end(), [&](int u, int v) {
        const auto a = mn(u), b = mn(v);
        return a.first * a.second > b.first * b.second || (a.first * a.second == b.first * b.second && u < v);
    });
    dmalloc(reinterpret_cast<void **>(&H->d_blocks), std::max<size_t>(1, size_t(nb)) * sizeof(HBlock));
    const auto push_blocks = [&]() {
        BEM_HIP(hipMemcpyAsync(H->d_blocks, H->blocks.data(), size_t(nb) * sizeof(HBlock), hipMemcpyHostToDevice, s));
        BEM_HIP(hipStreamSynchronize(s));
    };
    const auto tiles_of = [&](const std::vector<int> &ids, std::vector<int4> &tiles) {
        tiles.clear();
        for (int i : ids) {
            const auto &hb = H->blocks[i];
            const int tm = (hb.r1 - hb.r0 + 15) / 16, tn = (hb.c1 - hb.c0 + 15) / 16;
            for (int a = 0; a < tm; ++a)
                for (int c = 0; c < tn; ++c) tiles.push_back(make_int4(i, a, c, 0));
        }
    };
    std::vector<int> fallback;
    push_blocks();
    EntryCtx *ectx = entry_ctx_create(p);
    struct CtxGuard {
        EntryCtx *c;
        ~CtxGuard() { entry_ctx_free(c); }
    } ctx_guard{ectx};
    // ranks -> storage of the exact size; blocks without a rank become dense
    const auto compact = [&](const std::vector<int> &batch, const std::vector<int32_t> &rank,
                             const std::vector<float2 *> &Ub, const std::vector<float2 *> &Vb) {
        int64_t keep = 0;
        for (size_t j = 0; j < batch.size(); ++j)
            if (rank[j] >= 0) {
                const auto [m2, n2] = mn(batch[j]);
                keep += int64_t(rank[j]) * (m2 + n2);
            }
        float2 *pool = nullptr;
        dmalloc(reinterpret_cast<void **>(&pool), size_t(std::max<int64_t>(1, keep)) * sizeof(float2));
        H->pools.push_back(pool);
        std::vector<const float2 *> src;
        std::vector<float2 *> dst;
        std::vector<int64_t> cnt;
        int64_t po = 0;
        for (size_t j = 0; j < batch.size(); ++j) {
            HBlock &hb = H->blocks[batch[j]];
            if (rank[j] < 0) {
                fallback.push_back(batch[j]);
                continue;
            }
            const auto [m2, n2] = mn(batch[j]);
            hb.rank = rank[j];
            hb.U = pool + po;
            src.push_back(Ub[j]);
            dst.push_back(hb.U);
            cnt.push_back(int64_t(rank[j]) * m2);   // first rank columns (column-major)
            po += int64_t(rank[j]) * m2;
            hb.V = pool + po;
            src.push_back(Vb[j]);
            dst.push_back(hb.V);
            cnt.push_back(int64_t(rank[j]) * n2);   // first rank rows (row-major)
            po += int64_t(rank[j]) * n2;
            H->info.max_rank = std::max(H->info.max_rank, rank[j]);
            H->info.n_lowrank++;
            H->info.bytes += (int64_t(rank[j]) * (m2 + n2)) * int64_t(sizeof(float2));
        }
        DevMem m_src, m_dst, m_cnt;
        const float2 **d_src = upload(src, m_src, s);
        float2 **d_dst = upload(dst, m_dst, s);
        int64_t *d_cnt = upload(cnt, m_cnt, s);
        launch_copy_list(s, d_src, d_dst, d_cnt, int(src.size()));
        BEM_HIP(hipStreamSynchronize(s));
    };
    // low-rank blocks by cross approximation with partial pivoting (entries
    // on demand); BEM_HMATRIX_ACA=complete selects complete pivoting on the
    // computed blocks (for comparisons)
    const char *aca_env = std::getenv("BEM_HMATRIX_ACA");
    const bool complete = aca_env && std::string(aca_env) == "complete";
    int64_t acap_batch = ACAP_BATCH_MIN;
    {
        size_t free_b = 0, total_b = 0;
        BEM_HIP(hipMemGetInfo(&free_b, &total_b));
        acap_batch = std::max(ACAP_BATCH_MIN, std::min(ACAP_BATCH_MAX, int64_t(free_b / 2)));
    }
    size_t fi = 0;
    while (!complete && fi < far_ids.size()) {
        std::vector<int> batch;
        int64_t bytes = 0;
        int side = 1;
        while (fi < far_ids.size()) {
            const auto [m2, n2] = mn(far_ids[fi]);
            const int64_t need = int64_t(kcap(far_ids[fi])) * (m2 + n2) * int64_t(sizeof(float2));
            if (!batch.empty() && bytes + need > acap_batch) break;
            batch.push_back(far_ids[fi++]);
            bytes += need;
            side = int(std::max<int64_t>(side, std::max(m2, n2) / 2));
        }
        DevMem m_scr;
        float2 *scr = m_scr.alloc<float2>(size_t(bytes / int64_t(sizeof(float2))));
        std::vector<float2 *> Ub, Vb;
        std::vector<int32_t> kb, ids32;
        int64_t off = 0;
        for (int i : batch) {
            const auto [m2, n2] = mn(i);
            const int k = kcap(i);
            Ub.push_back(scr + off);
            off += int64_t(k) * m2;
            Vb.push_back(scr + off);
            off += int64_t(k) * n2;
            kb.push_back(k);
            ids32.push_back(i);
        }
        DevMem m_ids, m_U, m_V, m_k, m_rank;
        int32_t *d_ids = upload(ids32, m_ids, s);
        float2 **d_U = upload(Ub, m_U, s), **d_V = upload(Vb, m_V, s);
        int32_t *d_k = upload(kb, m_k, s);
        int32_t *d_rank = m_rank.alloc<int32_t>(batch.size());
        launch_aca_partial(p, ectx, H->d_perm, H->d_blocks, d_ids, int(batch.size()), d_U, d_V, d_k, float(eps), d_rank,
                           side);
        std::vector<int32_t> rank(batch.size());
        BEM_HIP(hipMemcpyAsync(rank.data(), d_rank, rank.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        compact(batch, rank, Ub, Vb);
    }
    while (complete && fi < far_ids.size()) {
        std::vector<int> batch;
        int64_t bytes = 0;
        while (fi < far_ids.size()) {
            const auto [m2, n2] = mn(far_ids[fi]);
            const int64_t need = (m2 * n2 + int64_t(kcap(far_ids[fi])) * (m2 + n2)) * int64_t(sizeof(float2));
            if (!batch.empty() && bytes + need > ACA_BATCH_BYTES) break;
            batch.push_back(far_ids[fi++]);
            bytes += need;
        }
        DevMem m_scr;
        float2 *scr = m_scr.alloc<float2>(size_t(bytes / int64_t(sizeof(float2))));
        std::vector<float2 *> Rp(nb, nullptr), Rb, Ub, Vb;
        std::vector<int32_t> kb, ids32;
        int64_t off = 0;
        for (int i : batch) {
            const auto [m2, n2] = mn(i);
            const int k = kcap(i);
            Rp[i] = scr + off;
            Rb.push_back(scr + off);
            off += m2 * n2;
            Ub.push_back(scr + off);
            off += int64_t(k) * m2;
            Vb.push_back(scr + off);
            off += int64_t(k) * n2;
            kb.push_back(k);
            ids32.push_back(i);
        }
        std::vector<int4> tiles;
        tiles_of(batch, tiles);
        DevMem m_rp, m_tiles, m_ids, m_R, m_U, m_V, m_k, m_rank;
        float2 **d_rp = upload(Rp, m_rp, s);
        int4 *d_tiles = upload(tiles, m_tiles, s);
        launch_hblock_entries(p, ectx, H->d_perm, d_tiles, int64_t(tiles.size()), H->d_blocks, d_rp);
        int32_t *d_ids = upload(ids32, m_ids, s);
        float2 **d_R = upload(Rb, m_R, s), **d_U = upload(Ub, m_U, s), **d_V = upload(Vb, m_V, s);
        int32_t *d_k = upload(kb, m_k, s);
        int32_t *d_rank = m_rank.alloc<int32_t>(batch.size());
        launch_aca(s, H->d_blocks, d_ids, int(batch.size()), d_R, d_U, d_V, d_k, float(eps), d_rank);
        std::vector<int32_t> rank(batch.size());
        BEM_HIP(hipMemcpyAsync(rank.data(), d_rank, rank.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        compact(batch, rank, Ub, Vb);
    }
    // dense blocks: near pairs of leaves, and far blocks the ACA did not compress
    dense_ids.insert(dense_ids.end(), fallback.begin(), fallback.end());
    int64_t dense_len = 0;
    for (int i : dense_ids) {
        const auto [m2, n2] = mn(i);
        dense_len += m2 * n2;
    }
    float2 *dpool = nullptr;
    dmalloc(reinterpret_cast<void **>(&dpool), size_t(std::max<int64_t>(1, dense_len)) * sizeof(float2));
    H->pools.push_back(dpool);
    std::vector<float2 *> Dp(nb, nullptr);
    {
        int64_t off = 0;
        for (int i : dense_ids) {
            const auto [m2, n2] = mn(i);
            HBlock &hb = H->blocks[i];
            hb.rank = -1;
            hb.D = dpool + off;
            Dp[i] = hb.D;
            off += m2 * n2;
            H->info.n_dense++;
        }
        H->info.bytes += dense_len * int64_t(sizeof(float2));
    }
    push_blocks();
    if (!dense_ids.empty()) {
        std::vector<int4> tiles;
        tiles_of(dense_ids, tiles);
        std::vector<int2> rows;
        for (int i : dense_ids) {
            const auto &hb = H->blocks[i];
            for (int a = 0; a < hb.r1 - hb.r0; ++a) rows.push_back(make_int2(i, a));
        }
        DevMem m_dp, m_tiles, m_rows;
        float2 **d_dp = upload(Dp, m_dp, s);
        int4 *d_tiles = upload(tiles, m_tiles, s);
        int2 *d_rows = upload(rows, m_rows, s);
        launch_hblock_entries(p, ectx, H->d_perm, d_tiles, int64_t(tiles.size()), H->d_blocks, d_dp);
        launch_hblock_correction(p, d_rows, int64_t(rows.size()), H->d_blocks, d_dp, H->d_perm, d_iperm);
    }
    BEM_HIP(hipStreamSynchronize(s));
    // the apply launches the blocks largest first (each carries its own
    // product offset, so the order changes no sum) to shorten the tail
    const auto stored = [&](const HBlock &hb) {
        const int64_t m2 = 2 * int64_t(hb.r1 - hb.r0), n2 = 2 * int64_t(hb.c1 - hb.c0);
        return hb.rank < 0 ? m2 * n2 : int64_t(hb.rank) * (m2 + n2);
    };
    std::sort(H->blocks.begin(), H->blocks.end(), [&](const HBlock &u, const HBlock &v) {
        const int64_t a = stored(u), b = stored(v);
        return a > b || (a == b && u.zoff < v.zoff);
    });
    push_blocks();
    H->info.n_blocks = nb;
    H->info.dense_bytes = 8 * int64_t(p.N) * int64_t(p.N);
    H->info.build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return H.release();
}

void hmatrix_apply(bem_problem &p, const double2 *x, double2 *y, int n_rhs, bool record)
{
    HMatrix &H = *p.hm;
    if (record) {
        BEM_HIP(hipEventRecord(p.ev[0], p.stream));
        BEM_HIP(hipEventRecord(p.ev[1], p.stream));
    }
    for (int r = 0; r < n_rhs; ++r)
        launch_h_apply(p.stream, H.d_blocks, int(H.blocks.size()), H.d_perm, p.d_rowD, p.d_rowN, H.d_rowptr, H.d_rowz,
                       p.NV, x + int64_t(r) * p.N, H.d_xp, H.d_z, y + int64_t(r) * p.N);
    if (record) {
        BEM_HIP(hipEventRecord(p.ev[2], p.stream));
        BEM_HIP(hipEventRecord(p.ev[3], p.stream));
        BEM_HIP(hipEventRecord(p.ev[4], p.stream));
        p.timed = true;
    }
}

HMatrix *hmatrix_build(bem_problem &p, double eps, int leaf, double eta, bem_hmatrix_info *info)
{
    int max_side = HBLOCK_MAX_SIDE;
    if (const char *e = std::getenv("BEM_HMATRIX_MAX_SIDE")) {   // for measurements of the split
        const int v = std::atoi(e);
        if (v >= leaf) max_side = v;
    }
    HMatrix *h = build(p, eps, leaf, eta, std::max(max_side, leaf));
    if (info) *info = h->info;
    return h;
}

void hmatrix_plan(const bem_problem &p, int leaf, double eta, int64_t out[4])
{
    const HTree T = plan_tree(p, leaf, eta, std::max(HBLOCK_MAX_SIDE, leaf));
    std::vector<SingularItem> items;
    touching_pairs(p, items);
    std::vector<int32_t> cptr, ccol, cp, ci;
    correction_pattern(p, items, cptr, ccol, cp, ci);
    int64_t n_adm = 0;
    for (char c : T.lowrank) n_adm += c;
    out[0] = int64_t(T.blocks.size());
    out[1] = n_adm;
    out[2] = int64_t(ccol.size());
    out[3] = touching_in_lowrank(T, p.NV, cptr, ccol);
}

}  // namespace bem
