// Far-field path of the Galerkin apply y = A x:
//   geometry  - per-triangle area, unit normal, P1 surface curls, quadrature points
//   gather    - P1 coefficients -> weighted densities at trial quadrature points
//   pairs     - all (test point, trial point) pairs of one wavenumber pass, FP32,
//               trial tiles staged in LDS, FP64 accumulation per tile
//   reduce    - sum of the per-split partial potentials (fixed order)
//   scatter   - test-side P1 projection per vertex + FP64 singular correction
//
// Operators (paper, Appendix A) with G = exp(ikr)/(4 pi r), d = x - y and
// F = G (1 - ikr)/r^2:  V: G;  K: F (d.n_y);  K': -F (d.n_x);
// W (integrated by parts): G [curl phi_b . curl phi_a - k^2 (n_x.n_y) phi_a phi_b].
// The PMCHWT rows of one domain (eq. Form2_calderon_sys_simp3) are
//   Dirichlet row:  -K u_D + sV V u_N,   Neumann row:  sW W u_D + K' u_N,
// with sV = sW = 1 for the exterior pass and sV = rho_j/rho_0, sW = rho_0/rho_j
// for the interior pass of domain j (eq. Form1_calderon_sys_int_ptot).
#include "bem_internal.h"
#include "rule6.h"

namespace bem {

constexpr int PAIR_BLOCK = 256;   // threads (test points per TPL) of a pair-kernel workgroup
constexpr double INV4PI = 0.079577471545947667884;

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

__global__ void k_geometry(const double *__restrict__ verts, const int32_t *__restrict__ tris, int64_t nt, int64_t M,
                           double *__restrict__ area, double *__restrict__ normal, double *__restrict__ curl,
                           float *__restrict__ pts, float *__restrict__ tnrm)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) P[a][d] = verts[3 * int64_t(tris[3 * t + a]) + d];
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) { e1[d] = P[1][d] - P[0][d]; e2[d] = P[2][d] - P[0][d]; }
    const double c0 = e1[1] * e2[2] - e1[2] * e2[1];
    const double c1 = e1[2] * e2[0] - e1[0] * e2[2];
    const double c2 = e1[0] * e2[1] - e1[1] * e2[0];
    const double twice = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    area[t] = 0.5 * twice;
    const double n[3] = {c0 / twice, c1 / twice, c2 / twice};
    for (int d = 0; d < 3; ++d) {
        normal[3 * t + d] = n[d];
        tnrm[d * nt + t] = float(n[d]);
    }
    // surface curl of the barycentric function lambda_a: -(P_{a+2} - P_{a+1}) / (2|T|)
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) curl[9 * t + 3 * a + d] = -(P[(a + 2) % 3][d] - P[(a + 1) % 3][d]) / twice;
    for (int q = 0; q < 6; ++q)
        for (int d = 0; d < 3; ++d) {
            const double x = q6_bary[q][0] * P[0][d] + q6_bary[q][1] * P[1][d] + q6_bary[q][2] * P[2][d];
            pts[d * M + 6 * t + q] = float(x);
        }
}

void launch_geometry(bem_problem &p)
{
    const int B = 256;
    k_geometry<<<dim3(blocks_1d(p.NT, B)), dim3(B), 0, p.stream>>>(
        p.d_verts, p.d_tris, p.NT, p.M, p.d_area, p.d_normal, p.d_curl, p.d_pts, p.d_tnrm);
    BEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// gather: trial records, grouped by triangle (float4)
//   point i = 6 t + q, at 2 i:       P0 = (y, 0)   P1 = (u_D w, u_N w)
//   triangle t, at 2 M + 3 t:        T0 = (n_y, 0)
//                                    T1 = (curl(u_D).x, curl(u_D).y) |T| / (4 pi)
//                                    T2 = (curl(u_D).z |T| / (4 pi), 0, 0)
// with w = |T| w_q / (4 pi): the normal and the surface curl of u_D are
// constant on a triangle, and the curl density of point q is w_q times T1, T2.
// ---------------------------------------------------------------------------

__global__ void k_gather(const double2 *__restrict__ x, const int32_t *__restrict__ tris,
                         const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN,
                         const double *__restrict__ area, const double *__restrict__ curl,
                         const float *__restrict__ pts, const float *__restrict__ tnrm, int64_t nt, int64_t M,
                         float4 *__restrict__ trial)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t t = i / 6;
    const int q = int(i - 6 * t);
    double uDr = 0, uDi = 0, uNr = 0, uNi = 0, cr[3] = {0, 0, 0}, ci[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        const int32_t g = tris[3 * t + a];
        const double2 xd = x[rowD[g]];
        const double2 xn = x[rowN[g]];
        const double l = q6_bary[q][a];
        uDr += l * xd.x; uDi += l * xd.y;
        uNr += l * xn.x; uNi += l * xn.y;
        if (q == 0)
            for (int d = 0; d < 3; ++d) {
                const double c = curl[9 * t + 3 * a + d];
                cr[d] += c * xd.x;
                ci[d] += c * xd.y;
            }
    }
    const double A = area[t] * INV4PI, w = A * q6_w[q];
    trial[2 * i] = make_float4(pts[i], pts[M + i], pts[2 * M + i], 0.0f);
    trial[2 * i + 1] = make_float4(float(uDr * w), float(uDi * w), float(uNr * w), float(uNi * w));
    if (q == 0) {
        float4 *r = trial + 2 * M + 3 * t;
        r[0] = make_float4(tnrm[t], tnrm[nt + t], tnrm[2 * nt + t], 0.0f);
        r[1] = make_float4(float(cr[0] * A), float(ci[0] * A), float(cr[1] * A), float(ci[1] * A));
        r[2] = make_float4(float(cr[2] * A), float(ci[2] * A), 0.0f, 0.0f);
    }
}

void launch_gather(bem_problem &p, const double2 *x)
{
    const int B = 256;
    k_gather<<<dim3(blocks_1d(p.M, B)), dim3(B), 0, p.stream>>>(
        x, p.d_tris, p.d_rowD, p.d_rowN, p.d_area, p.d_curl, p.d_pts, p.d_tnrm, p.NT, p.M, p.d_trial);
    BEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// pair kernel
// ---------------------------------------------------------------------------
//
// Work item (pass, test block, split): a workgroup of 256 lanes owns
// 256 * TPL consecutive test points of the pass and one contiguous chunk of
// its trial triangles (split s of n_split).  Trial records go through LDS in
// tiles of 42 triangles (252 points); every lane reads each entry by
// broadcast.  Per test point x (normal n_x) the kernel forms, in FP32 within a
// tile and in FP64 across tiles,
//   A1 = sum G u_N w              A2 = sum F (d.n_y) u_D w
//   B1 = sum_T (n_x.n_y) sum_q G u_D w          B2 = sum F (d.n_x) u_N w
//   Cc = sum_T curl_T(u_D) |T|/(4 pi) sum_q w_q G
// over the trial points (d = x - y, F = G (1 - ikr)/r^2) and returns
//   D = sV A1 - A2 (Dirichlet row),  N = -k^2 sW B1 - B2 and C = sW Cc
// (Neumann row, scalar and curl parts).  The factors that are constant on a
// trial triangle (n_x.n_y and the curl) multiply sums over its six points
// once per triangle rather than once per pair.

constexpr int TILE_TRI = 42;               // trial triangles per LDS tile
constexpr int TILE_PTS = 6 * TILE_TRI;     // their 252 quadrature points

struct Acc {
    float a1r, a1i, a2r, a2i, b1r, b1i, b2r, b2i, xr, xi, yr, yi, zr, zi;
};

// per-triangle sums of one test point: T = sum G u_D w, S = sum w_q G
struct TriSum {
    float tr, ti, sr, si;
};

// one (test point, trial point) pair
template <bool ATT, bool WRAP>
__device__ __forceinline__ void pair_step(const float xx, const float xy, const float xz, const float nx,
                                          const float ny, const float nz, const float4 P0, const float4 P1,
                                          const float4 T0, const float cq, const float k, const float k2pi,
                                          const float kim, Acc &a, TriSum &s)
{
    const float dx = xx - P0.x, dy = xy - P0.y, dz = xz - P0.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    // r2 == 0 only for a point paired with itself (coincident triangle, same
    // quadrature point); that term belongs to the singular correction.
    const float rinv = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
    const float r = r2 * rinv;
    float ph = r * k2pi;                       // phase in revolutions
    // v_sin / v_cos take revolutions and reduce |ph| < 256 themselves; the
    // explicit reduction is kept only when a pass's phases can exceed that
    if (WRAP) ph = ph - rintf(ph);
    const float sn = __builtin_amdgcn_sinf(ph);  // sin(2 pi ph)
    const float cs = __builtin_amdgcn_cosf(ph);
    float gr = cs * rinv, gi = sn * rinv;
    float fr, fi;
    const float kr = r * k;
    const float rinv2 = rinv * rinv;
    if (ATT) {
        const float damp = __expf(-kim * r);
        gr *= damp;
        gi *= damp;
        // (1 - i k r) with complex k = (1 + kim r) - i kr
        const float re1 = fmaf(kim, r, 1.0f);
        fr = fmaf(gr, re1, gi * kr) * rinv2;
        fi = fmaf(gi, re1, -gr * kr) * rinv2;
    } else {
        fr = fmaf(gi, kr, gr) * rinv2;
        fi = fmaf(-gr, kr, gi) * rinv2;
    }
    const float tK = fmaf(dx, T0.x, fmaf(dy, T0.y, dz * T0.z));    // d . n_y
    const float tKp = fmaf(dx, nx, fmaf(dy, ny, dz * nz));         // d . n_x
    const float eKr = fr * tK, eKi = fi * tK;
    const float ePr = fr * tKp, ePi = fi * tKp;
    // A1 += G u_N w, A2 += eK u_D w, B2 += eP u_N w
    a.a1r = fmaf(gr, P1.z, fmaf(-gi, P1.w, a.a1r));
    a.a1i = fmaf(gr, P1.w, fmaf(gi, P1.z, a.a1i));
    a.a2r = fmaf(eKr, P1.x, fmaf(-eKi, P1.y, a.a2r));
    a.a2i = fmaf(eKr, P1.y, fmaf(eKi, P1.x, a.a2i));
    a.b2r = fmaf(ePr, P1.z, fmaf(-ePi, P1.w, a.b2r));
    a.b2i = fmaf(ePr, P1.w, fmaf(ePi, P1.z, a.b2i));
    // T += G u_D w, S += w_q G
    s.tr = fmaf(gr, P1.x, fmaf(-gi, P1.y, s.tr));
    s.ti = fmaf(gr, P1.y, fmaf(gi, P1.x, s.ti));
    s.sr = fmaf(cq, gr, s.sr);
    s.si = fmaf(cq, gi, s.si);
}

// the per-triangle factors: B1 += (n_x.n_y) T, Cc += curl S
__device__ __forceinline__ void triangle_step(const float nx, const float ny, const float nz, const float4 T0,
                                              const float4 T1, const float4 T2, const TriSum &s, Acc &a)
{
    const float tW = fmaf(nx, T0.x, fmaf(ny, T0.y, nz * T0.z));    // n_x . n_y
    a.b1r = fmaf(tW, s.tr, a.b1r);
    a.b1i = fmaf(tW, s.ti, a.b1i);
    a.xr = fmaf(s.sr, T1.x, fmaf(-s.si, T1.y, a.xr));
    a.xi = fmaf(s.sr, T1.y, fmaf(s.si, T1.x, a.xi));
    a.yr = fmaf(s.sr, T1.z, fmaf(-s.si, T1.w, a.yr));
    a.yi = fmaf(s.sr, T1.w, fmaf(s.si, T1.z, a.yi));
    a.zr = fmaf(s.sr, T2.x, fmaf(-s.si, T2.y, a.zr));
    a.zi = fmaf(s.sr, T2.y, fmaf(s.si, T2.x, a.zi));
}

// Five waves per SIMD (one test point per lane): left to itself the compiler
// hoists all twelve LDS reads of a triangle and needs 129 VGPRs (three
// waves); bounded, it fits 93 without spills and runs 8 % faster.
template <int TPL, bool ATT, bool WRAP>
__device__ __forceinline__ void pairs_body(const int4 w, const PassDev *__restrict__ passes,
                                           const float *__restrict__ pts, const float *__restrict__ tnrm,
                                           const float4 *__restrict__ trial, double *__restrict__ part, int64_t M,
                                           int64_t nt, int n_split)
{
    __shared__ float4 lp[2][TILE_PTS];
    __shared__ float4 lt[3][TILE_TRI];
    const PassDev P = passes[w.x];
    const int tid = threadIdx.x;
    const float kv = in_vgpr(P.k), k2piv = in_vgpr(P.k_over_2pi), kimv = in_vgpr(P.kim);
    // the two weights of the 6-point rule (points 0-2 and 3-5)
    const float wqa = in_vgpr(float(q6_w[0])), wqb = in_vgpr(float(q6_w[3]));
    // pass constants of the per-tile combination: sV, sW and -k^2 sW
    const double sV = P.sV, sW = P.sW, cNr = -double(P.sW) * P.k2re, cNi = -double(P.sW) * P.k2im;

    // test points of this lane
    float xx[TPL], xy[TPL], xz[TPL], nx[TPL], ny[TPL], nz[TPL];
    long long ti[TPL];
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const long long i = P.test_begin + (long long)w.y * (PAIR_BLOCK * TPL) + u * PAIR_BLOCK + tid;
        ti[u] = i;
        const long long ii = i < P.test_end ? i : P.test_end - 1;
        const long long t = ii / 6;
        xx[u] = pts[ii];
        xy[u] = pts[M + ii];
        xz[u] = pts[2 * M + ii];
        nx[u] = tnrm[t];
        ny[u] = tnrm[nt + t];
        nz[u] = tnrm[2 * nt + t];
    }

    // trial chunk of this split: whole tiles (the pass ranges hold whole
    // triangles, so every chunk and tile does too)
    const long long n_trial = P.trial_end - P.trial_begin;
    long long chunk = (n_trial + n_split - 1) / n_split;
    chunk = (chunk + TILE_PTS - 1) / TILE_PTS * TILE_PTS;
    const long long j_begin = P.trial_begin + (long long)w.z * chunk;
    const long long j_end = j_begin + chunk < P.trial_end ? j_begin + chunk : P.trial_end;
    const float4 *tri_rec = trial + 2 * M;

    double acc[TPL][10];
#pragma unroll
    for (int u = 0; u < TPL; ++u)
#pragma unroll
        for (int c = 0; c < 10; ++c) acc[u][c] = 0.0;

    for (long long jt = j_begin; jt < j_end; jt += TILE_PTS) {
        const int cnt = int(j_end - jt < TILE_PTS ? j_end - jt : TILE_PTS);
        const int ntri = cnt / 6;
        __syncthreads();
        if (tid < cnt) {
            lp[0][tid] = trial[2 * (jt + tid)];
            lp[1][tid] = trial[2 * (jt + tid) + 1];
        }
        if (tid < ntri) {
            const float4 *r = tri_rec + 3 * (jt / 6 + tid);
            lt[0][tid] = r[0];
            lt[1][tid] = r[1];
            lt[2][tid] = r[2];
        }
        __syncthreads();
        Acc a[TPL];
#pragma unroll
        for (int u = 0; u < TPL; ++u) a[u] = Acc{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int tr = 0; tr < ntri; ++tr) {
            const float4 T0 = lt[0][tr];
            TriSum s[TPL];
#pragma unroll
            for (int u = 0; u < TPL; ++u) s[u] = TriSum{0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float4 P0 = lp[0][6 * tr + q], P1 = lp[1][6 * tr + q];
#pragma unroll
                for (int u = 0; u < TPL; ++u)
                    pair_step<ATT, WRAP>(xx[u], xy[u], xz[u], nx[u], ny[u], nz[u], P0, P1, T0, q < 3 ? wqa : wqb, kv,
                                         k2piv, kimv, a[u], s[u]);
            }
            const float4 T1 = lt[1][tr], T2 = lt[2][tr];
#pragma unroll
            for (int u = 0; u < TPL; ++u) triangle_step(nx[u], ny[u], nz[u], T0, T1, T2, s[u], a[u]);
        }
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
            const Acc &q = a[u];
            acc[u][0] += sV * double(q.a1r) - double(q.a2r);
            acc[u][1] += sV * double(q.a1i) - double(q.a2i);
            acc[u][2] += cNr * double(q.b1r) - cNi * double(q.b1i) - double(q.b2r);
            acc[u][3] += cNr * double(q.b1i) + cNi * double(q.b1r) - double(q.b2i);
            acc[u][4] += sW * double(q.xr);
            acc[u][5] += sW * double(q.xi);
            acc[u][6] += sW * double(q.yr);
            acc[u][7] += sW * double(q.yi);
            acc[u][8] += sW * double(q.zr);
            acc[u][9] += sW * double(q.zi);
        }
    }
    double *out = part + (size_t(P.slot) * n_split + w.z) * 10 * size_t(M);
#pragma unroll
    for (int u = 0; u < TPL; ++u)
        if (ti[u] < P.test_end)
#pragma unroll
            for (int c = 0; c < 10; ++c) out[size_t(c) * M + ti[u]] = acc[u][c];
}

template <int TPL, bool ATT, bool WRAP>
__global__ __launch_bounds__(PAIR_BLOCK) __attribute__((amdgpu_waves_per_eu(TPL == 1 ? 5 : 3))) void k_pairs(
    const int4 *__restrict__ work, const PassDev *__restrict__ passes, const float *__restrict__ pts,
    const float *__restrict__ tnrm, const float4 *__restrict__ trial, double *__restrict__ part, int64_t M,
    int64_t nt, int n_split)
{
    pairs_body<TPL, ATT, WRAP>(work[blockIdx.x], passes, pts, tnrm, trial, part, M, nt, n_split);
}

// Grouped launch: the work lists of several problems (their own records,
// partials and launch shapes) in one grid; workgroup b runs item
// b - start[m] of member m.  The member table travels in the kernel arguments.
template <int TPL, bool ATT, bool WRAP>
__global__ __launch_bounds__(PAIR_BLOCK) __attribute__((amdgpu_waves_per_eu(TPL == 1 ? 5 : 3))) void k_pairs_group(
    const PairGroup g)
{
    int m = 0;
    while (m + 1 < g.n && int(blockIdx.x) >= g.start[m + 1]) ++m;
    const PairMember &q = g.m[m];
    pairs_body<TPL, ATT, WRAP>(q.work[int(blockIdx.x) - g.start[m]], q.passes, q.pts, q.tnrm, q.trial, q.part, q.M,
                               q.nt, q.n_split);
}

void launch_pairs(bem_problem &p)
{
    bool att = false;
    for (int i = 0; i < p.n_pass; ++i)
        if (p.passes[i].kim != 0.0) att = true;
    const dim3 grid(unsigned(p.n_work)), block(PAIR_BLOCK);
#define PAIRS(T, A, W)                                                                                             \
    k_pairs<T, A, W><<<grid, block, 0, p.stream>>>(p.d_work, p.d_pass, p.d_pts, p.d_tnrm, p.d_trial, p.d_part, p.M, \
                                                   p.NT, p.n_split)
    const bool w = p.wrap_phase;
    if (p.tpl == 2) {
        if (att) {
            if (w) PAIRS(2, true, true); else PAIRS(2, true, false);
        } else {
            if (w) PAIRS(2, false, true); else PAIRS(2, false, false);
        }
    } else {
        if (att) {
            if (w) PAIRS(1, true, true); else PAIRS(1, true, false);
        } else {
            if (w) PAIRS(1, false, true); else PAIRS(1, false, false);
        }
    }
#undef PAIRS
    BEM_HIP(hipGetLastError());
}

// The pair-kernel variant of a problem: test points per lane, complex
// wavenumbers in some pass, explicit phase reduction.
int pair_variant(const bem_problem &p)
{
    bool att = false;
    for (int i = 0; i < p.n_pass; ++i)
        if (p.passes[i].kim != 0.0) att = true;
    return (p.tpl == 2 ? 4 : 0) + (att ? 2 : 0) + (p.wrap_phase ? 1 : 0);
}

void launch_pairs_group(hipStream_t s, const std::vector<bem_problem *> &ps)
{
    if (ps.empty()) return;
    if (int(ps.size()) > PAIR_GROUP_MAX) throw Error{BEM_ERR_INVALID_ARG, "grouped pair launch: too many problems"};
    const int v = pair_variant(*ps[0]);
    PairGroup g{};
    g.n = int(ps.size());
    int64_t total = 0;
    for (int i = 0; i < g.n; ++i) {
        const bem_problem &p = *ps[i];
        if (pair_variant(p) != v) throw Error{BEM_ERR_INVALID_ARG, "grouped pair launch: mixed kernel variants"};
        g.start[i] = int(total);
        g.m[i] = PairMember{p.d_work, p.d_pass, p.d_pts, p.d_tnrm, p.d_trial, p.d_part, p.M, p.NT, p.n_split, 0};
        total += p.n_work;
    }
    if (total >= (int64_t(1) << 31) / PAIR_BLOCK) throw Error{BEM_ERR_UNSUPPORTED, "grouped pair launch too large"};
    for (int i = g.n; i <= PAIR_GROUP_MAX; ++i) g.start[i] = int(total);
    const dim3 grid{unsigned(total), 1u, 1u}, block{unsigned(PAIR_BLOCK), 1u, 1u};
#define PAIRS_G(T, A, W) k_pairs_group<T, A, W><<<grid, block, 0, s>>>(g)
    switch (v) {
    case 0: PAIRS_G(1, false, false); break;
    case 1: PAIRS_G(1, false, true); break;
    case 2: PAIRS_G(1, true, false); break;
    case 3: PAIRS_G(1, true, true); break;
    case 4: PAIRS_G(2, false, false); break;
    case 5: PAIRS_G(2, false, true); break;
    case 6: PAIRS_G(2, true, false); break;
    default: PAIRS_G(2, true, true); break;
    }
#undef PAIRS_G
    BEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// reduce: pot[i][c] = sum over slots and splits of the partials (fixed order)
// ---------------------------------------------------------------------------

// One thread per (channel, point): 2 n_split coalesced loads, summed as four
// interleaved partial sums combined in a fixed order (deterministic).
__global__ void k_reduce(const double *__restrict__ part, int64_t M, int n_split, double *__restrict__ pot)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= 10 * M) return;
    const int64_t c = idx / M, i = idx - c * M;
    const size_t stride = size_t(10) * M;
    const double *q = part + idx;
    const int n = 2 * n_split;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 4 <= n; k += 4) {
        s0 += q[size_t(k) * stride];
        s1 += q[size_t(k + 1) * stride];
        s2 += q[size_t(k + 2) * stride];
        s3 += q[size_t(k + 3) * stride];
    }
    for (; k < n; ++k) s0 += q[size_t(k) * stride];
    pot[10 * i + c] = (s0 + s1) + (s2 + s3);
}

void launch_reduce(bem_problem &p)
{
    const int B = 256;
    k_reduce<<<dim3(blocks_1d(10 * p.M, B)), dim3(B), 0, p.stream>>>(p.d_part, p.M, p.n_split, p.d_pot);
    BEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// scatter: one thread per vertex g
//   y_D[g] = sum_{(t,a) at g} sum_q |t| w_q lambda_a(q) D(t,q)            + correction
//   y_N[g] = sum_{(t,a) at g} sum_q |t| w_q [lambda_a(q) N(t,q) + curl_a . C(t,q)] + correction
// correction: y_D += C_DD x_D + C_DN x_N,  y_N += C_ND x_D + C_NN x_N over the
// vertex-level CSR of touching pairs.
// ---------------------------------------------------------------------------

__global__ void k_scatter(const double *__restrict__ pot, const int32_t *__restrict__ v2t_ptr,
                          const int32_t *__restrict__ v2t, const double *__restrict__ area,
                          const double *__restrict__ curl, const int32_t *__restrict__ rowD,
                          const int32_t *__restrict__ rowN, const int32_t *__restrict__ cptr,
                          const int32_t *__restrict__ ccol, const double2 *__restrict__ cval,
                          const double2 *__restrict__ x, double2 *__restrict__ y, int64_t NV, int parts)
{
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= NV) return;
    double yDr = 0, yDi = 0, yNr = 0, yNi = 0;
    if (parts & 1) {
        for (int32_t k = v2t_ptr[g]; k < v2t_ptr[g + 1]; ++k) {
            const int32_t tc = v2t[k];
            const int64_t t = tc / 3;
            const int a = tc - 3 * int(t);
            const double ar = area[t];
            const double cx = curl[9 * t + 3 * a], cy = curl[9 * t + 3 * a + 1], cz = curl[9 * t + 3 * a + 2];
            for (int q = 0; q < 6; ++q) {
                const double *P = pot + 10 * (6 * t + q);
                const double w = ar * q6_w[q];
                const double wl = w * q6_bary[q][a];
                yDr += wl * P[0];
                yDi += wl * P[1];
                yNr += wl * P[2] + w * (cx * P[4] + cy * P[6] + cz * P[8]);
                yNi += wl * P[3] + w * (cx * P[5] + cy * P[7] + cz * P[9]);
            }
        }
    }
    if (parts & 2) {
        for (int32_t e = cptr[g]; e < cptr[g + 1]; ++e) {
            const int32_t h = ccol[e];
            const double2 xd = x[rowD[h]], xn = x[rowN[h]];
            const double2 DD = cval[4 * e], DN = cval[4 * e + 1], ND = cval[4 * e + 2], NN = cval[4 * e + 3];
            yDr += DD.x * xd.x - DD.y * xd.y + DN.x * xn.x - DN.y * xn.y;
            yDi += DD.x * xd.y + DD.y * xd.x + DN.x * xn.y + DN.y * xn.x;
            yNr += ND.x * xd.x - ND.y * xd.y + NN.x * xn.x - NN.y * xn.y;
            yNi += ND.x * xd.y + ND.y * xd.x + NN.x * xn.y + NN.y * xn.x;
        }
    }
    y[rowD[g]] = make_double2(yDr, yDi);
    y[rowN[g]] = make_double2(yNr, yNi);
}

void launch_scatter(bem_problem &p, const double2 *x, double2 *y, int parts)
{
    const int B = 256;
    k_scatter<<<dim3(blocks_1d(p.NV, B)), dim3(B), 0, p.stream>>>(
        p.d_pot, p.d_v2t_ptr, p.d_v2t, p.d_area, p.d_curl, p.d_rowD, p.d_rowN, p.d_cptr, p.d_ccol, p.d_cval, x, y,
        p.NV, parts);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
