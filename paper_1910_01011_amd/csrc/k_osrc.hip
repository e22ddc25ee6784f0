// OSRC block-diagonal preconditioner (paper, operator preconditioning section:
// eqs. OSRC_prec, OSRC_prec_blocks, OSRC_DtN_NtD_maps).
//
// For every domain the Galerkin residual rows are mapped to coefficients by the
// P1 mass matrix (z = M^-1 r) and then (the results land in the swapped
// positions, see k_osrc_out)
//   Dirichlet-equation row:  Lambda_DtN z = i k sqrt(1 + X) z
//   Neumann-equation row:    Lambda_NtD z = (i k)^-1 (M - S')^-1 M sqrt(1 + X) z
// with X = -M^-1 S', S' = S / k_eps^2, k_eps = k + 0.4 i k^(1/3) R_eps^(-2/3),
// k = k0, and the branch-rotated Pade form
//   sqrt(1 + X) z = C0 z - sum_l A_l (M - B_l S')^-1 S' z.
// The Neumann rows are evaluated as C0 w0 - sum_l A_l (w0 - z - B_l t_l)/(1 - B_l)
// with w0 = (M - S')^-1 M z and t_l the Pade solves (k_osrc_ntd): the same
// operator, so that w0 is solved in the same batch as the t_l.
// M and S are assembled on the union of all boundaries (block diagonal by
// domain).  The sparse solves of one application (two batches: the mass solve,
// then every Pade and w0 system) are done by a batched
// Jacobi-preconditioned COCG (conjugate orthogonal CG for complex symmetric
// matrices) in FP64, one workgroup per (system, domain) block.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "bem_internal.h"

namespace bem {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// mass and stiffness on the vertex adjacency pattern
// ---------------------------------------------------------------------------

// one thread per vertex row g: M_gh += |t| (1 + d_ab)/12, S_gh += e_a . e_b / (4 |t|)
__global__ void k_mass_stiff(const double *__restrict__ verts, const int32_t *__restrict__ tris,
                             const double *__restrict__ area, const int32_t *__restrict__ v2t_ptr,
                             const int32_t *__restrict__ v2t, const int32_t *__restrict__ aptr,
                             const int32_t *__restrict__ acol, int64_t NV, double *__restrict__ Mv,
                             double *__restrict__ Sv)
{
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= NV) return;
    for (int32_t e = aptr[g]; e < aptr[g + 1]; ++e) {
        Mv[e] = 0.0;
        Sv[e] = 0.0;
    }
    for (int32_t k = v2t_ptr[g]; k < v2t_ptr[g + 1]; ++k) {
        const int64_t t = v2t[k] / 3;
        const int a = v2t[k] - 3 * int(t);
        double P[3][3];
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) P[c][d] = verts[3 * int64_t(tris[3 * t + c]) + d];
        double ea[3];
        for (int d = 0; d < 3; ++d) ea[d] = P[(a + 2) % 3][d] - P[(a + 1) % 3][d];
        const double ar = area[t];
        for (int b = 0; b < 3; ++b) {
            double eb[3];
            for (int d = 0; d < 3; ++d) eb[d] = P[(b + 2) % 3][d] - P[(b + 1) % 3][d];
            const int32_t h = tris[3 * t + b];
            int32_t e = aptr[g];
            while (e < aptr[g + 1] - 1 && acol[e] != h) ++e;
            Mv[e] += ar * (a == b ? 2.0 : 1.0) / 12.0;
            Sv[e] += (ea[0] * eb[0] + ea[1] * eb[1] + ea[2] * eb[2]) / (4.0 * ar);
        }
    }
}

// ---------------------------------------------------------------------------
// preconditioner pieces
// ---------------------------------------------------------------------------

// residual rows (R vectors in unknown order) -> [2R][NV]: D rows then N rows
__global__ void k_osrc_split(const double2 *__restrict__ Y, const int32_t *__restrict__ rowD,
                             const int32_t *__restrict__ rowN, int64_t NV, int64_t N, int R, double2 *__restrict__ U)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= NV * R) return;
    const int64_t r = idx / NV, g = idx - r * NV;
    U[(2 * r) * NV + g] = Y[r * N + rowD[g]];
    U[(2 * r + 1) * NV + g] = Y[r * N + rowN[g]];
}

// out[(v * L + l)][i] = sum_e S[e] z_v[col] * s  for l < L   (S' z replicated per Pade term)
__global__ void k_osrc_sprime(const int32_t *__restrict__ aptr, const int32_t *__restrict__ acol,
                              const double *__restrict__ Sv, const double2 *__restrict__ Z, int64_t n, int V, int L,
                              double2 s, double2 *__restrict__ out)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * V) return;
    const int64_t v = idx / n, i = idx - v * n;
    double re = 0, im = 0;
    for (int32_t e = aptr[i]; e < aptr[i + 1]; ++e) {
        const double2 z = Z[v * n + acol[e]];
        re += Sv[e] * z.x;
        im += Sv[e] * z.y;
    }
    const double2 w = make_double2(re * s.x - im * s.y, re * s.y + im * s.x);
    for (int l = 0; l < L; ++l) out[(v * L + l) * n + i] = w;
}

// Dirichlet rows (v = 2 r): i k (C0 z_v - sum_l A_l t_(v,l)), the square-root
// Pade approximant applied to z
__global__ void k_osrc_combine(const double2 *__restrict__ Z, const double2 *__restrict__ T,
                               const double2 *__restrict__ Al, int L, double2 C0, double2 ik, int64_t n, int R,
                               double2 *__restrict__ rootD)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const int64_t r = idx / n, i = idx - r * n, v = 2 * r;
    const double2 z = Z[v * n + i];
    double re = C0.x * z.x - C0.y * z.y, im = C0.x * z.y + C0.y * z.x;
    for (int l = 0; l < L; ++l) {
        const double2 t = T[(v * L + l) * n + i], a = Al[l];
        re -= a.x * t.x - a.y * t.y;
        im -= a.x * t.y + a.y * t.x;
    }
    rootD[idx] = make_double2(ik.x * re - ik.y * im, ik.x * im + ik.y * re);
}

// w = M x for the Neumann-row vectors (v = 2 r + 1) of Z: right-hand sides of
// the (M - S')^-1 M z solves, appended after the Pade systems
__global__ void k_mass_nrows(const int32_t *__restrict__ aptr, const int32_t *__restrict__ acol,
                             const double *__restrict__ Mv, const double2 *__restrict__ Z, int64_t n, int R,
                             double2 *__restrict__ W)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const int64_t r = idx / n, i = idx - r * n;
    const double2 *z = Z + (2 * r + 1) * n;
    double re = 0, im = 0;
    for (int32_t e = aptr[i]; e < aptr[i + 1]; ++e) {
        const double2 x = z[acol[e]];
        re += Mv[e] * x.x;
        im += Mv[e] * x.y;
    }
    W[idx] = make_double2(re, im);
}

// Neumann rows: wN = (M - S')^-1 M root with root = C0 z - sum_l A_l t_l and
// t_l = (M - B_l S')^-1 S' z.  With T = M^-1 S' (all maps are functions of T),
// (I - T)^-1 (I - B T)^-1 T = [(I - T)^-1 - (I - B T)^-1] / (1 - B) and
// (I - B T)^-1 = I + B (I - B T)^-1 T, so
//   wN = C0 w0 - sum_l A_l (w0 - z - B_l t_l) / (1 - B_l),  w0 = (M - S')^-1 M z,
// the same discrete operator with w0 solved beside the t_l instead of after them.
// coef[l] = (A_l / (1 - B_l), B_l)
__global__ void k_osrc_ntd(const double2 *__restrict__ Z, const double2 *__restrict__ T,
                           const double2 *__restrict__ W0, const double2 *__restrict__ coef, int L, double2 C0,
                           int64_t n, int R, double2 *__restrict__ WN)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const int64_t r = idx / n, i = idx - r * n, v = 2 * r + 1;
    const double2 z = Z[v * n + i], w0 = W0[idx];
    double re = C0.x * w0.x - C0.y * w0.y, im = C0.x * w0.y + C0.y * w0.x;
    for (int l = 0; l < L; ++l) {
        const double2 t = T[(v * L + l) * n + i], a = coef[2 * l], b = coef[2 * l + 1];
        // d = w0 - z - B_l t
        const double dr = w0.x - z.x - (b.x * t.x - b.y * t.y), di = w0.y - z.y - (b.x * t.y + b.y * t.x);
        re -= a.x * dr - a.y * di;
        im -= a.x * di + a.y * dr;
    }
    WN[idx] = make_double2(re, im);
}

// out (unknown order), with the paper's permutation of the unknowns of every
// domain to [u_N; u_D] folded in (GMRES on C A Pi y = C b is GMRES on
// (Pi C) A u = Pi C b): u_N positions <- Lambda_DtN result of the Dirichlet
// rows (rootD), u_D positions <- Lambda_NtD result of the Neumann rows (s wN)
__global__ void k_osrc_out(const double2 *__restrict__ rootD, const double2 *__restrict__ wN, double2 s,
                           const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN, int64_t NV, int64_t N,
                           int R, double2 *__restrict__ Y)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= NV * R) return;
    const int64_t r = idx / NV, g = idx - r * NV;
    Y[r * N + rowN[g]] = rootD[idx];
    const double2 w = wN[idx];
    Y[r * N + rowD[g]] = make_double2(s.x * w.x - s.y * w.y, s.x * w.y + s.y * w.x);
}

static unsigned nb(int64_t n) { return blocks_1d(n, 256); }

// stream-ordered scratch on the stream of the current problem
thread_local hipStream_t t_osrc_stream = nullptr;

struct OsrcBuf {
    double2 *p = nullptr;
    hipStream_t s;
    explicit OsrcBuf(size_t n) : s(t_osrc_stream)
    {
        BEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&p), std::max<size_t>(1, n) * sizeof(double2), s));
    }
    ~OsrcBuf() { (void)hipFreeAsync(p, s); }
};

void osrc_setup(bem_problem &p)
{
    if (p.d_aptr) return;
    // vertex adjacency (vertices sharing a triangle), sorted, including the diagonal
    std::vector<std::vector<int32_t>> adj(p.NV);
    for (int64_t t = 0; t < p.NT; ++t)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) adj[p.h_tris[3 * t + a]].push_back(p.h_tris[3 * t + b]);
    std::vector<int32_t> ptr(p.NV + 1, 0), col;
    for (int64_t g = 0; g < p.NV; ++g) {
        auto &r = adj[g];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        ptr[g + 1] = ptr[g] + int32_t(r.size());
        col.insert(col.end(), r.begin(), r.end());
    }
    p.a_nnz = ptr[p.NV];
    std::vector<int32_t> dpos(p.NV);
    for (int64_t g = 0; g < p.NV; ++g)
        dpos[g] = int32_t(std::lower_bound(col.begin() + ptr[g], col.begin() + ptr[g + 1], int32_t(g)) - col.begin());
    std::vector<int2> rng;
    for (const auto &d : p.doms) rng.push_back(make_int2(int(d.v_off), int(d.v_off + d.nv)));
    BEM_HIP(hipMalloc(&p.d_adiag, dpos.size() * sizeof(int32_t)));
    BEM_HIP(hipMalloc(&p.d_drange, rng.size() * sizeof(int2)));
    BEM_HIP(hipMemcpyAsync(p.d_adiag, dpos.data(), dpos.size() * sizeof(int32_t), hipMemcpyHostToDevice, p.stream));
    BEM_HIP(hipMemcpyAsync(p.d_drange, rng.data(), rng.size() * sizeof(int2), hipMemcpyHostToDevice, p.stream));
    BEM_HIP(hipMalloc(&p.d_aptr, ptr.size() * sizeof(int32_t)));
    BEM_HIP(hipMalloc(&p.d_acol, col.size() * sizeof(int32_t)));
    BEM_HIP(hipMalloc(&p.d_Mv, col.size() * sizeof(double)));
    BEM_HIP(hipMalloc(&p.d_Sv, col.size() * sizeof(double)));
    BEM_HIP(hipMemcpyAsync(p.d_aptr, ptr.data(), ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, p.stream));
    BEM_HIP(hipMemcpyAsync(p.d_acol, col.data(), col.size() * sizeof(int32_t), hipMemcpyHostToDevice, p.stream));
    k_mass_stiff<<<dim3(nb(p.NV)), dim3(256), 0, p.stream>>>(p.d_verts, p.d_tris, p.d_area, p.d_v2t_ptr, p.d_v2t,
                                                            p.d_aptr, p.d_acol, p.NV, p.d_Mv, p.d_Sv);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(p.stream));
}

// Persistent COCG: one 1024-lane workgroup per (system, domain) block of
// (M - c_g S) x_g = b_g.  M and S couple only vertices of one boundary, so
// the block of every domain is an independent system; each converges on its
// own (||r_d|| <= tol ||b_d||) with a Jacobi preconditioner
// (diag(M - c_g S)), zero initial guess, maxit iterations at most.  Every loop
// decision uses block-reduced values, so all waves of a workgroup take the same
// path and the loop ends for all of them.
constexpr int CG_BLOCK = 1024;

__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *red)
{
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[3 * w] = a;
        red[3 * w + 1] = b;
        red[3 * w + 2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int k = 0; k < CG_BLOCK / 64; ++k) {
        a += red[3 * k];
        b += red[3 * k + 1];
        c += red[3 * k + 2];
    }
}

// z = r / d (complex)
__device__ __forceinline__ double2 cdiv(double2 r, double2 d)
{
    const double den = d.x * d.x + d.y * d.y;
    return make_double2((r.x * d.x + r.y * d.y) / den, (r.y * d.x - r.x * d.y) / den);
}

__global__ __launch_bounds__(CG_BLOCK) void k_cocg_persistent(const int32_t *__restrict__ aptr,
                                                              const int32_t *__restrict__ acol,
                                                              const int32_t *__restrict__ adiag,
                                                              const double *__restrict__ Mv,
                                                              const double *__restrict__ Sv,
                                                              const int2 *__restrict__ drange, int n_dom,
                                                              const double2 *__restrict__ c,
                                                              const double2 *__restrict__ B, double2 *__restrict__ X,
                                                              double2 *__restrict__ Rw, double2 *__restrict__ Pw,
                                                              double2 *__restrict__ Qw, int64_t n, double tol,
                                                              int maxit)
{
    __shared__ double red[3 * (CG_BLOCK / 64)];
    const int64_t g = blockIdx.x / n_dom;
    const int2 rng = drange[blockIdx.x - g * n_dom];
    const int tid = threadIdx.x;
    const double2 cg = c[g];
    const double2 *b = B + g * n;
    double2 *x = X + g * n, *r = Rw + g * n, *pv = Pw + g * n, *q = Qw + g * n;
    auto diag = [&](int64_t i) {
        const int32_t e = adiag[i];
        return make_double2(Mv[e] - cg.x * Sv[e], -cg.y * Sv[e]);
    };
    double bn2 = 0, rr_ = 0, ri_ = 0;
    for (int64_t i = rng.x + tid; i < rng.y; i += CG_BLOCK) {
        const double2 v = b[i];
        const double2 z = cdiv(v, diag(i));
        x[i] = make_double2(0.0, 0.0);
        r[i] = v;
        pv[i] = z;
        bn2 += v.x * v.x + v.y * v.y;
        rr_ += v.x * z.x - v.y * z.y;   // rho = r^T z (unconjugated)
        ri_ += v.x * z.y + v.y * z.x;
    }
    block_sum3(bn2, rr_, ri_, red);
    if (bn2 == 0.0) return;
    double rho_r = rr_, rho_i = ri_;
    for (int it = 0; it < maxit; ++it) {
        __syncthreads();   // p complete before the product
        double pqr = 0, pqi = 0, dummy = 0;
        for (int64_t i = rng.x + tid; i < rng.y; i += CG_BLOCK) {
            double mr = 0, mi = 0, sr = 0, si = 0;
            for (int32_t e = aptr[i]; e < aptr[i + 1]; ++e) {
                const double2 v = pv[acol[e]];
                mr += Mv[e] * v.x;
                mi += Mv[e] * v.y;
                sr += Sv[e] * v.x;
                si += Sv[e] * v.y;
            }
            const double qr = mr - (cg.x * sr - cg.y * si), qi = mi - (cg.x * si + cg.y * sr);
            q[i] = make_double2(qr, qi);
            const double2 pp = pv[i];
            pqr += pp.x * qr - pp.y * qi;
            pqi += pp.x * qi + pp.y * qr;
        }
        block_sum3(pqr, pqi, dummy, red);
        const double den = pqr * pqr + pqi * pqi;
        if (den == 0.0) break;
        const double ar = (rho_r * pqr + rho_i * pqi) / den, ai = (rho_i * pqr - rho_r * pqi) / den;
        double rn2 = 0, sr2 = 0, si2 = 0;
        for (int64_t i = rng.x + tid; i < rng.y; i += CG_BLOCK) {
            const double2 pp = pv[i], qq = q[i], xx = x[i], rv = r[i];
            x[i] = make_double2(xx.x + ar * pp.x - ai * pp.y, xx.y + ar * pp.y + ai * pp.x);
            const double2 nr = make_double2(rv.x - (ar * qq.x - ai * qq.y), rv.y - (ar * qq.y + ai * qq.x));
            r[i] = nr;
            const double2 z = cdiv(nr, diag(i));
            rn2 += nr.x * nr.x + nr.y * nr.y;
            sr2 += nr.x * z.x - nr.y * z.y;
            si2 += nr.x * z.y + nr.y * z.x;
        }
        block_sum3(rn2, sr2, si2, red);
        if (rn2 <= tol * tol * bn2) break;
        const double d2 = rho_r * rho_r + rho_i * rho_i;
        if (d2 == 0.0) break;
        const double br = (sr2 * rho_r + si2 * rho_i) / d2, bi = (si2 * rho_r - sr2 * rho_i) / d2;
        rho_r = sr2;
        rho_i = si2;
        for (int64_t i = rng.x + tid; i < rng.y; i += CG_BLOCK) {
            const double2 pp = pv[i], z = cdiv(r[i], diag(i));
            pv[i] = make_double2(z.x + br * pp.x - bi * pp.y, z.y + br * pp.y + bi * pp.x);
        }
    }
}

static void cocg_batch(bem_problem &p, int G, const std::vector<cd> &c, const double2 *B, double2 *X, double tol,
                       int maxit)
{
    t_osrc_stream = p.stream;
    const int64_t n = p.NV;
    hipStream_t s = p.stream;
    const size_t tot = size_t(G) * n;
    OsrcBuf R(tot), Pp(tot), Q(tot), cdev{size_t(G)};
    std::vector<double2> t(G);
    for (int g = 0; g < G; ++g) t[g] = make_double2(c[g].real(), c[g].imag());
    BEM_HIP(hipMemcpyAsync(cdev.p, t.data(), G * sizeof(double2), hipMemcpyHostToDevice, s));
    BEM_HIP(hipStreamSynchronize(s));
    const int n_dom = int(p.doms.size());
    const int64_t wgs = int64_t(G) * n_dom;
    if (wgs >= (int64_t(1) << 31)) throw Error{BEM_ERR_UNSUPPORTED, "OSRC: too many systems in one batch"};
    k_cocg_persistent<<<dim3(unsigned(wgs)), dim3(CG_BLOCK), 0, s>>>(p.d_aptr, p.d_acol, p.d_adiag, p.d_Mv, p.d_Sv,
                                                                    p.d_drange, n_dom, cdev.p, B, X, R.p, Pp.p, Q.p,
                                                                    n, tol, maxit);
    BEM_HIP(hipGetLastError());
}

void osrc_apply(bem_problem &p, const OsrcParams &o, const double2 *Y, double2 *Out, int R)
{
    osrc_setup(p);
    t_osrc_stream = p.stream;
    const int64_t n = p.NV;
    hipStream_t s = p.stream;
    const int L = o.n_pade;
    // coefficients
    const cd k(p.k0re, p.k0im);
    const cd ke = k + cd(0.0, 0.4 * std::cbrt(p.k0re) * std::pow(o.r_eps, -2.0 / 3.0));
    const cd ke2 = ke * ke;
    std::vector<cd> A(L), B(L);
    const cd e = std::exp(cd(0.0, -o.theta)), c = e - 1.0;
    cd C0 = 1.0;
    for (int l = 1; l <= L; ++l) {
        const double a = 2.0 / (2 * L + 1) * std::pow(std::sin(l * M_PI / (2 * L + 1)), 2);
        const double b = std::pow(std::cos(l * M_PI / (2 * L + 1)), 2);
        const cd D = 1.0 + b * c;
        C0 += a * c / D;
        A[l - 1] = std::exp(cd(0.0, -o.theta / 2.0)) * a / (D * D);
        B[l - 1] = e * b / D;
    }
    C0 *= std::exp(cd(0.0, o.theta / 2.0));
    const cd ik = cd(0.0, 1.0) * k;
    // z = M^-1 (D rows, N rows)
    OsrcBuf U(size_t(2 * R) * n), Z(size_t(2 * R) * n);
    k_osrc_split<<<dim3(nb(n * R)), dim3(256), 0, s>>>(Y, p.d_rowD, p.d_rowN, n, p.N, R, U.p);
    BEM_HIP(hipGetLastError());
    cocg_batch(p, 2 * R, std::vector<cd>(2 * R, cd(0.0)), U.p, Z.p, o.cg_tol, o.cg_maxit);
    // one batch: t_(v,l) = (M - B_l S')^-1 S' z_v for both rows of every vector,
    // and w0_r = (M - S')^-1 M z_(N rows) (see k_osrc_ntd)
    const int64_t nt = int64_t(2 * R) * L;   // Pade systems
    OsrcBuf Bt(size_t(nt + R) * n), T(size_t(nt + R) * n);
    const cd inv = 1.0 / ke2;
    if (L > 0) {
        k_osrc_sprime<<<dim3(nb(n * 2 * R)), dim3(256), 0, s>>>(p.d_aptr, p.d_acol, p.d_Sv, Z.p, n, 2 * R, L,
                                                                make_double2(inv.real(), inv.imag()), Bt.p);
        BEM_HIP(hipGetLastError());
    }
    k_mass_nrows<<<dim3(nb(n * R)), dim3(256), 0, s>>>(p.d_aptr, p.d_acol, p.d_Mv, Z.p, n, R, Bt.p + nt * n);
    BEM_HIP(hipGetLastError());
    std::vector<cd> shifts(size_t(nt + R));
    for (int v = 0; v < 2 * R; ++v)
        for (int l = 0; l < L; ++l) shifts[size_t(v) * L + l] = B[l] / ke2;
    for (int r = 0; r < R; ++r) shifts[size_t(nt) + r] = inv;
    cocg_batch(p, int(nt + R), shifts, Bt.p, T.p, o.cg_tol, o.cg_maxit);
    // D rows: i k root; N rows: wN from w0 and the t_l
    OsrcBuf Al(size_t(std::max(L, 1))), coef(size_t(2 * std::max(L, 1))), rootD(size_t(R) * n),
        WN(size_t(R) * n);
    {
        std::vector<double2> t(L), cf(2 * L);
        for (int l = 0; l < L; ++l) {
            t[l] = make_double2(A[l].real(), A[l].imag());
            const cd q = A[l] / (1.0 - B[l]);
            cf[2 * l] = make_double2(q.real(), q.imag());
            cf[2 * l + 1] = make_double2(B[l].real(), B[l].imag());
        }
        if (L > 0) {
            BEM_HIP(hipMemcpyAsync(Al.p, t.data(), L * sizeof(double2), hipMemcpyHostToDevice, s));
            BEM_HIP(hipMemcpyAsync(coef.p, cf.data(), 2 * L * sizeof(double2), hipMemcpyHostToDevice, s));
        }
        BEM_HIP(hipStreamSynchronize(s));
    }
    k_osrc_combine<<<dim3(nb(n * R)), dim3(256), 0, s>>>(Z.p, T.p, Al.p, L, make_double2(C0.real(), C0.imag()),
                                                         make_double2(ik.real(), ik.imag()), n, R, rootD.p);
    BEM_HIP(hipGetLastError());
    k_osrc_ntd<<<dim3(nb(n * R)), dim3(256), 0, s>>>(Z.p, T.p, T.p + nt * n, coef.p, L,
                                                     make_double2(C0.real(), C0.imag()), n, R, WN.p);
    BEM_HIP(hipGetLastError());
    const cd sN = 1.0 / ik;
    k_osrc_out<<<dim3(nb(n * R)), dim3(256), 0, s>>>(rootD.p, WN.p, make_double2(sN.real(), sN.imag()), p.d_rowD,
                                                     p.d_rowN, n, p.N, R, Out);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(s));
}

}  // namespace bem
