// Single-layer operator alone: y = V_k0 x, the Galerkin P1 matrix of
// V phi(x) = int_Gamma G(x, y) phi(y) ds_y, G = exp(ikr)/(4 pi r) (paper,
// Appendix A, single-layer operator), on the union of all boundaries at the
// exterior wavenumber.  It is the one-channel form of the fused far-field path:
//   gather   - P1 coefficients -> psi w at the trial quadrature points
//   pairs    - every (test point, trial point) pair of the exterior pass, FP32,
//              one complex accumulator per test point (G times psi w)
//   reduce   - sum of the per-split partials (fixed order)
//   scatter  - test-side P1 projection + the FP64 Sauter-Schwab V correction of
//              touching pairs (pass 0 of the singular pass, V block only)
// Per pair: difference, r^2, 1/r, r, phase, sin, cos, G and one complex
// multiply-add: about 21 FLOP and 3 transcendentals, against 140 FLOP of the
// fused multitrace pair.  It shares the scratch buffers of the fused path; its
// launch shape is timed on first use when the problem was set up with
// autotuning, and is the fused kernel's otherwise.
#include <algorithm>

#include "bem_internal.h"
#include "rule6.h"

namespace bem {

constexpr int SL_BLOCK = 256;   // threads of the pair kernel = trial tile (same as the fused kernel)
constexpr double SL_INV4PI = 0.079577471545947667884;

// trial record of point i = 6 t + q: rec[i] = (y, Re psi w), im[i] = Im psi w,
// psi = sum_a lambda_a(q) x[vertex a], w = |T| w_q / (4 pi)
__global__ void k_gather_v(const double2 *__restrict__ x, const int32_t *__restrict__ tris,
                           const double *__restrict__ area, const float *__restrict__ pts, int64_t M,
                           float4 *__restrict__ rec, float *__restrict__ im)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t t = i / 6;
    const int q = int(i - 6 * t);
    double pr = 0, pi = 0;
    for (int a = 0; a < 3; ++a) {
        const double2 v = x[tris[3 * t + a]];
        pr += q6_bary[q][a] * v.x;
        pi += q6_bary[q][a] * v.y;
    }
    const double w = area[t] * q6_w[q] * SL_INV4PI;
    rec[i] = make_float4(pts[i], pts[M + i], pts[2 * M + i], float(pr * w));
    im[i] = float(pi * w);
}

// Workgroup b * n_split + s owns test block b (SL_BLOCK * TPL points of the
// exterior pass) and trial chunk s (consecutive workgroups take consecutive
// chunks, so each XCD's L2 holds one chunk); trial tiles of SL_BLOCK points go
// through LDS and are read by broadcast.  FP32 sums within a tile, FP64 across
// tiles.  The point paired with itself (r = 0) is skipped: the singular
// correction accounts for it.
template <int TPL, bool ATT, bool WRAP>
__global__ __launch_bounds__(SL_BLOCK) void k_pairs_v(const PassDev *__restrict__ pass0, const float *__restrict__ pts,
                                                      const float4 *__restrict__ rec, const float *__restrict__ rim,
                                                      double *__restrict__ part, int64_t M, int n_split)
{
    __shared__ float4 l0[SL_BLOCK];
    __shared__ float l1[SL_BLOCK];
    const int4 w = make_int4(0, int(blockIdx.x) / n_split, int(blockIdx.x) % n_split, 0);
    const PassDev P = *pass0;
    const int tid = threadIdx.x;
    float xx[TPL], xy[TPL], xz[TPL];
    long long ti[TPL];
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const long long i = P.test_begin + (long long)w.y * (SL_BLOCK * TPL) + u * SL_BLOCK + tid;
        ti[u] = i;
        const long long ii = i < P.test_end ? i : P.test_end - 1;
        xx[u] = pts[ii];
        xy[u] = pts[M + ii];
        xz[u] = pts[2 * M + ii];
    }
    const long long n_trial = P.trial_end - P.trial_begin;
    long long chunk = (n_trial + n_split - 1) / n_split;
    chunk = (chunk + SL_BLOCK - 1) / SL_BLOCK * SL_BLOCK;
    const long long j_begin = P.trial_begin + (long long)w.z * chunk;
    const long long j_end = j_begin + chunk < P.trial_end ? j_begin + chunk : P.trial_end;
    const float k2pi = in_vgpr(P.k_over_2pi), kim = in_vgpr(P.kim);
    double acc[TPL][2];
#pragma unroll
    for (int u = 0; u < TPL; ++u) acc[u][0] = acc[u][1] = 0.0;
    for (long long jt = j_begin; jt < j_end; jt += SL_BLOCK) {
        const int cnt = int(j_end - jt < SL_BLOCK ? j_end - jt : SL_BLOCK);
        __syncthreads();
        if (tid < cnt) {
            l0[tid] = rec[jt + tid];
            l1[tid] = rim[jt + tid];
        }
        __syncthreads();
        float ar[TPL], ai[TPL];
#pragma unroll
        for (int u = 0; u < TPL; ++u) ar[u] = ai[u] = 0.0f;
        for (int j = 0; j < cnt; ++j) {
            const float4 L = l0[j];
            const float wi = l1[j];
#pragma unroll
            for (int u = 0; u < TPL; ++u) {
                const float dx = xx[u] - L.x, dy = xy[u] - L.y, dz = xz[u] - L.z;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float rinv = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
                const float r = r2 * rinv;
                float ph = r * k2pi;   // phase in revolutions (v_sin / v_cos reduce |ph| < 256)
                if (WRAP) ph = ph - rintf(ph);
                float gr = __builtin_amdgcn_cosf(ph) * rinv, gi = __builtin_amdgcn_sinf(ph) * rinv;
                if (ATT) {
                    const float damp = __expf(-kim * r);
                    gr *= damp;
                    gi *= damp;
                }
                ar[u] = fmaf(gr, L.w, fmaf(-gi, wi, ar[u]));
                ai[u] = fmaf(gr, wi, fmaf(gi, L.w, ai[u]));
            }
        }
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
            acc[u][0] += ar[u];
            acc[u][1] += ai[u];
        }
    }
    double *out = part + size_t(w.z) * 2 * size_t(M);
#pragma unroll
    for (int u = 0; u < TPL; ++u)
        if (ti[u] < P.test_end) {
            out[ti[u]] = acc[u][0];
            out[M + ti[u]] = acc[u][1];
        }
}

// pot[i] = sum over splits of the partials, four interleaved sums in a fixed order
__global__ void k_reduce_v(const double *__restrict__ part, int64_t M, int n_split, double2 *__restrict__ pot)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double s[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int k = 0;
    for (; k + 4 <= n_split; k += 4)
        for (int c = 0; c < 2; ++c)
            for (int m = 0; m < 4; ++m) s[c][m] += part[(size_t(k + m) * 2 + c) * M + i];
    for (; k < n_split; ++k)
        for (int c = 0; c < 2; ++c) s[c][0] += part[(size_t(k) * 2 + c) * M + i];
    pot[i] = make_double2((s[0][0] + s[0][1]) + (s[0][2] + s[0][3]), (s[1][0] + s[1][1]) + (s[1][2] + s[1][3]));
}

// y[g] = sum_{(t,a) at g} sum_q |t| w_q lambda_a(q) pot(t, q) + sum_e Vc[e] x[col e]
// (Vc: block 1 of the 4-block correction values, the V block of pass 0)
__global__ void k_scatter_v(const double2 *__restrict__ pot, const int32_t *__restrict__ v2t_ptr,
                            const int32_t *__restrict__ v2t, const double *__restrict__ area,
                            const int32_t *__restrict__ cptr, const int32_t *__restrict__ ccol,
                            const double2 *__restrict__ cval, const double2 *__restrict__ x, double2 *__restrict__ y,
                            int64_t NV)
{
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= NV) return;
    double yr = 0, yi = 0;
    for (int32_t k = v2t_ptr[g]; k < v2t_ptr[g + 1]; ++k) {
        const int32_t tc = v2t[k];
        const int64_t t = tc / 3;
        const int a = tc - 3 * int(t);
        const double ar = area[t];
        for (int q = 0; q < 6; ++q) {
            const double2 P = pot[6 * t + q];
            const double wl = ar * q6_w[q] * q6_bary[q][a];
            yr += wl * P.x;
            yi += wl * P.y;
        }
    }
    for (int32_t e = cptr[g]; e < cptr[g + 1]; ++e) {
        const double2 v = cval[4 * e + 1], xv = x[ccol[e]];
        yr += v.x * xv.x - v.y * xv.y;
        yi += v.x * xv.y + v.y * xv.x;
    }
    y[g] = make_double2(yr, yi);
}

static void launch_pairs_v(bem_problem &p, int tpl, int n_split, const float4 *rec, const float *rim)
{
    const bool att = p.passes[0].kim != 0.0;
    const int64_t nblk = (p.passes[0].test_end - p.passes[0].test_begin + SL_BLOCK * tpl - 1) / (SL_BLOCK * tpl);
    const dim3 grid(blocks_1d(nblk * n_split * SL_BLOCK, SL_BLOCK)), block(SL_BLOCK);
#define SL_LAUNCH2(T, W)                                                                                              \
    if (att) k_pairs_v<T, true, W><<<grid, block, 0, p.stream>>>(p.d_pass, p.d_pts, rec, rim, p.d_part, p.M, n_split); \
    else k_pairs_v<T, false, W><<<grid, block, 0, p.stream>>>(p.d_pass, p.d_pts, rec, rim, p.d_part, p.M, n_split);
#define SL_LAUNCH(T)                                                                                                  \
    if (p.wrap_phase) {                                                                                               \
        SL_LAUNCH2(T, true)                                                                                           \
    } else {                                                                                                          \
        SL_LAUNCH2(T, false)                                                                                          \
    }
    if (tpl == 4) {
        SL_LAUNCH(4)
    } else if (tpl == 2) {
        SL_LAUNCH(2)
    } else {
        SL_LAUNCH(1)
    }
#undef SL_LAUNCH
#undef SL_LAUNCH2
    BEM_HIP(hipGetLastError());
}

// Launch shape of the single-layer pair kernel (test points per lane, trial
// chunks): a short timing sweep on first use.  The partial sums (2 M doubles
// per chunk) live in the fused path's buffer of 2 x n_split x 10 M doubles,
// which bounds the chunks at 10 n_split.
static void tune_single_layer(bem_problem &p, const float4 *rec, const float *rim)
{
    const int64_t cap = 10 * int64_t(p.n_split);
    const int64_t m0 = p.passes[0].test_end - p.passes[0].test_begin;
    hipEvent_t e0, e1;
    BEM_HIP(hipEventCreate(&e0));
    BEM_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int best_tpl = 1, best_split = int(std::min<int64_t>(cap, 8));
    bool warmed = false;
    for (int tpl : {1, 2, 4})
        for (int ns : {4, 8, 16, 32, 64}) {
            const int64_t wgs = (m0 + SL_BLOCK * tpl - 1) / (SL_BLOCK * tpl) * ns;
            if (ns > cap || wgs < 256 || int64_t(ns) * SL_BLOCK > m0) continue;
            if (!warmed) {
                for (int w = 0; w < 3; ++w) launch_pairs_v(p, tpl, ns, rec, rim);
                warmed = true;
            }
            float t = 1e30f;
            for (int r = 0; r < 2; ++r) {
                BEM_HIP(hipEventRecord(e0, p.stream));
                launch_pairs_v(p, tpl, ns, rec, rim);
                BEM_HIP(hipEventRecord(e1, p.stream));
                BEM_HIP(hipEventSynchronize(e1));
                float ms = 0;
                BEM_HIP(hipEventElapsedTime(&ms, e0, e1));
                t = std::min(t, ms);
            }
            if (t < best) {
                best = t;
                best_tpl = tpl;
                best_split = ns;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p.sl_tpl = best_tpl;
    p.sl_split = best_split;
}

void launch_single_layer(bem_problem &p, const double2 *x, double2 *y, bool record)
{
    const int B = 256;
    // the single-layer records reuse the fused apply's buffers: M float4 of
    // records and M floats of imaginary parts (M + M/4 float4) in the trial
    // buffer of 2 M + 3 NT float4; potentials (M complex) in the 10 M doubles
    if (p.M + (p.M + 3) / 4 > 2 * p.M + 3 * p.NT)
        throw Error{BEM_ERR_DEVICE, "single-layer records do not fit the trial buffer"};
    float4 *rec = p.d_trial;
    float *rim = reinterpret_cast<float *>(p.d_trial + p.M);
    double2 *pot = reinterpret_cast<double2 *>(p.d_pot);
    if (record) BEM_HIP(hipEventRecord(p.ev[0], p.stream));
    k_gather_v<<<dim3(blocks_1d(p.M, B)), dim3(B), 0, p.stream>>>(x, p.d_tris, p.d_area, p.d_pts, p.M, rec, rim);
    BEM_HIP(hipGetLastError());
    if (p.sl_tpl == 0) {
        if (p.flags & BEM_AUTOTUNE) {
            tune_single_layer(p, rec, rim);
        } else {
            // without tuning: the fused kernel's shape, bounded by the partial buffer
            p.sl_tpl = std::min(p.tpl, 4);
            p.sl_split = p.n_split;
        }
    }
    if (record) BEM_HIP(hipEventRecord(p.ev[1], p.stream));
    launch_pairs_v(p, p.sl_tpl, p.sl_split, rec, rim);
    if (record) BEM_HIP(hipEventRecord(p.ev[2], p.stream));
    k_reduce_v<<<dim3(blocks_1d(p.M, B)), dim3(B), 0, p.stream>>>(p.d_part, p.M, p.sl_split, pot);
    BEM_HIP(hipGetLastError());
    if (record) BEM_HIP(hipEventRecord(p.ev[3], p.stream));
    k_scatter_v<<<dim3(blocks_1d(p.NV, B)), dim3(B), 0, p.stream>>>(pot, p.d_v2t_ptr, p.d_v2t, p.d_area, p.d_sl_cptr,
                                                                    p.d_sl_ccol, p.d_sl_cval, x, y, p.NV);
    BEM_HIP(hipGetLastError());
    if (record) {
        BEM_HIP(hipEventRecord(p.ev[4], p.stream));
        p.timed = true;
    }
}

}  // namespace bem
