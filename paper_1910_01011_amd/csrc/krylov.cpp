// Batched restarted GMRES and flexible GMRES for a block of right-hand sides
// (the paper solves with GMRES, restart 100, relative tolerance 1e-5).
//
// All R systems share the operator; every Arnoldi step applies the operator to
// the block of active vectors in one call (one GEMM in the assembled modes).
// Arnoldi is classical Gram-Schmidt applied twice, in FP64 on the device; the
// small Hessenberg least-squares problems (Givens rotations) are solved on the
// host per right-hand side.  A system whose residual estimate reaches the
// tolerance stops updating its Hessenberg matrix (its vectors still ride along
// until the cycle ends); at every restart the still-active systems are packed
// into contiguous buffers, so converged ones cost nothing afterwards.
//
// Flexible variant: with a preconditioner M (here an inner GMRES solve on a
// lower-precision operator), z_j = M(v_j) is stored and x is updated from the
// z's (Saad's FGMRES), so M may change from one step to the next.
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <complex>
#include <functional>
#include <vector>

#include "bem_internal.h"

namespace bem {

namespace {

using cd = std::complex<double>;

// Stream-ordered scratch (no device-wide synchronisation, so the solves of
// several problems on their own streams overlap).
template <typename T>
struct DevBuf {
    T *p = nullptr;
    hipStream_t s;
    DevBuf(size_t n, hipStream_t st) : s(st)
    {
        BEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&p), std::max<size_t>(1, n) * sizeof(T), s));
    }
    ~DevBuf() { (void)hipFreeAsync(p, s); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

// Pinned host staging for the values an Arnoldi step reads back: copies to
// and from pageable memory would make the host wait for each of them.  One
// buffer per thread and nesting depth (a flexible solve runs its inner solves
// on the same thread while it holds its own), grown as needed and kept until
// the process ends (a few kilobytes per thread and depth; freeing it at thread
// exit could run after the HIP runtime has shut down).
struct StageSlot {
    double2 *p = nullptr;
    size_t cap = 0;
};
thread_local std::vector<StageSlot> t_stage;
thread_local int t_stage_depth = 0;

struct StageLease {
    double2 *p = nullptr;
    explicit StageLease(size_t n)
    {
        if (int(t_stage.size()) <= t_stage_depth) t_stage.resize(size_t(t_stage_depth) + 1);
        StageSlot &sl = t_stage[size_t(t_stage_depth)];
        if (sl.cap < n) {
            if (sl.p) (void)hipHostFree(sl.p);
            sl.p = nullptr;
            sl.cap = 0;
            BEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&sl.p), n * sizeof(double2), hipHostMallocPortable));
            sl.cap = n;
        }
        p = sl.p;
        ++t_stage_depth;
    }
    ~StageLease() { --t_stage_depth; }
    StageLease(const StageLease &) = delete;
    StageLease &operator=(const StageLease &) = delete;
};

}  // namespace

void gmres_batch(bem_problem &p, int64_t n, int R, const double2 *B, double2 *X, const KrylovOpts &o,
                 const ApplyFn &A, const ApplyFn *M, bem_solve_info *info)
{
    hipStream_t s = p.stream;
    const int m = std::max(1, o.restart);
    const int nblk = bdot_chunks(n);
    DevBuf<double2> V(size_t(m + 1) * R * n, s), Z(M ? size_t(m) * R * n : 1, s), Xa(size_t(R) * n, s),
        Ba(size_t(R) * n, s);
    DevBuf<double2> hdev(size_t(R) * (m + 2), s), part(size_t(R) * (m + 2) * nblk, s);
    // per step: the two Gram-Schmidt coefficient blocks, the norms, the scales
    const StageLease lease(size_t(2) * R * (m + 2) + size_t(2) * R);
    double2 *const stage = lease.p;
    const int64_t ld = int64_t(R) * n;   // stride between basis vectors (packed to the active count)

    auto host_dots = [&](const double2 *Vb, int64_t ldv, int nvec, const double2 *w, int Ra, std::vector<cd> &out) {
        bdot(s, Vb, ldv, nvec, w, n, Ra, part.p, nblk, hdev.p);
        std::vector<double2> t(size_t(Ra) * nvec);
        BEM_HIP(hipMemcpyAsync(t.data(), hdev.p, t.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        out.resize(t.size());
        for (size_t i = 0; i < t.size(); ++i) out[i] = cd(t[i].x, t[i].y);
    };
    auto to_dev = [&](const std::vector<cd> &v) {
        std::vector<double2> t(v.size());
        for (size_t i = 0; i < v.size(); ++i) t[i] = make_double2(v[i].real(), v[i].imag());
        BEM_HIP(hipMemcpyAsync(hdev.p, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, s));
        BEM_HIP(hipStreamSynchronize(s));   // t is pageable and goes out of scope
    };

    // norms of b
    std::vector<double> bnorm(R);
    {
        std::vector<cd> d;
        host_dots(B, 0, 1, B, R, d);
        for (int r = 0; r < R; ++r) bnorm[r] = std::sqrt(std::max(0.0, d[r].real()));
    }
    BEM_HIP(hipMemsetAsync(X, 0, size_t(R) * n * sizeof(double2), s));
    std::vector<int> its(R, 0);
    std::vector<char> conv(R, 0);
    std::vector<double> est(R, 1.0);
    for (int r = 0; r < R; ++r)
        if (bnorm[r] == 0.0) { conv[r] = 1; est[r] = 0.0; }
    bool first = true;
    long steps = 0;   // Arnoldi steps of this call (for progress lines)
    for (;;) {
        std::vector<int> act;
        for (int r = 0; r < R; ++r)
            if (!conv[r] && its[r] < o.max_iter) act.push_back(r);
        if (act.empty()) break;
        const int Ra = int(act.size());
        // pack the active systems
        for (int a = 0; a < Ra; ++a) {
            BEM_HIP(hipMemcpyAsync(Ba.p + int64_t(a) * n, B + int64_t(act[a]) * n, n * sizeof(double2),
                                   hipMemcpyDeviceToDevice, s));
            BEM_HIP(hipMemcpyAsync(Xa.p + int64_t(a) * n, X + int64_t(act[a]) * n, n * sizeof(double2),
                                   hipMemcpyDeviceToDevice, s));
        }
        // r = b - A x  into V_0
        if (first) {
            BEM_HIP(hipMemcpyAsync(V.p, Ba.p, size_t(Ra) * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
        } else {
            A(Xa.p, V.p, Ra);
            std::vector<cd> mone(Ra, cd(-1.0, 0.0));
            to_dev(mone);
            bscale(s, V.p, V.p, n, Ra, hdev.p);
            std::vector<cd> one(Ra, cd(1.0, 0.0));
            to_dev(one);
            baxpy(s, Ba.p, 0, 1, hdev.p, V.p, n, Ra, 1.0);
        }
        first = false;
        std::vector<double> beta(Ra);
        {
            std::vector<cd> d;
            host_dots(V.p, 0, 1, V.p, Ra, d);
            for (int a = 0; a < Ra; ++a) beta[a] = std::sqrt(std::max(0.0, d[a].real()));
        }
        std::vector<char> live(Ra, 1);
        int n_live = 0;
        for (int a = 0; a < Ra; ++a) {
            est[act[a]] = beta[a] / bnorm[act[a]];
            if (est[act[a]] <= o.tol || beta[a] == 0.0) {
                conv[act[a]] = 1;
                live[a] = 0;
            } else {
                ++n_live;
            }
        }
        if (n_live == 0) break;
        {
            std::vector<cd> sc(Ra);
            for (int a = 0; a < Ra; ++a) sc[a] = beta[a] > 0 ? cd(1.0 / beta[a], 0.0) : cd(0.0, 0.0);
            to_dev(sc);
            bscale(s, V.p, V.p, n, Ra, hdev.p);
        }
        std::vector<std::vector<cd>> H(Ra, std::vector<cd>(size_t(m + 1) * m, cd(0))), g(Ra, std::vector<cd>(m + 1, cd(0)));
        std::vector<std::vector<cd>> cs(Ra, std::vector<cd>(m)), sn(Ra, std::vector<cd>(m));
        std::vector<int> jused(Ra, 0);
        for (int a = 0; a < Ra; ++a) g[a][0] = beta[a];
        int j = 0;
        for (; j < m; ++j) {
            double2 *vj = V.p + int64_t(j) * ld, *vj1 = V.p + int64_t(j + 1) * ld;
            const double2 *zj = vj;
            if (M) {
                double2 *zz = Z.p + int64_t(j) * ld;
                (*M)(vj, zz, Ra);
                zj = zz;
            }
            A(zj, vj1, Ra);
            // both Gram-Schmidt passes and the norm without waiting: each pass's
            // coefficients are used on the device as computed and copied to the
            // host for the Hessenberg matrix; the host waits once per step
            const size_t nh = size_t(Ra) * (j + 1);
            for (int pass = 0; pass < 2; ++pass) {
                bdot(s, V.p, ld, j + 1, vj1, n, Ra, part.p, nblk, hdev.p);
                BEM_HIP(hipMemcpyAsync(stage + pass * nh, hdev.p, nh * sizeof(double2), hipMemcpyDeviceToHost, s));
                baxpy(s, V.p, ld, j + 1, hdev.p, vj1, n, Ra, -1.0);
            }
            bdot(s, vj1, 0, 1, vj1, n, Ra, part.p, nblk, hdev.p);
            BEM_HIP(hipMemcpyAsync(stage + 2 * nh, hdev.p, Ra * sizeof(double2), hipMemcpyDeviceToHost, s));
            BEM_HIP(hipStreamSynchronize(s));
            std::vector<cd> h1(nh), h2(nh), nn(Ra);
            for (size_t i = 0; i < nh; ++i) {
                h1[i] = cd(stage[i].x, stage[i].y);
                h2[i] = cd(stage[nh + i].x, stage[nh + i].y);
            }
            for (int a = 0; a < Ra; ++a) nn[a] = cd(stage[2 * nh + a].x, stage[2 * nh + a].y);
            std::vector<cd> sc(Ra);
            bool any = false;
            for (int a = 0; a < Ra; ++a) {
                const double hn = std::sqrt(std::max(0.0, nn[a].real()));
                sc[a] = hn > 0 ? cd(1.0 / hn, 0.0) : cd(0.0, 0.0);
                if (!live[a]) continue;
                std::vector<cd> &Hh = H[a];
                for (int i = 0; i <= j; ++i) Hh[size_t(i) * m + j] = h1[size_t(a) * (j + 1) + i] + h2[size_t(a) * (j + 1) + i];
                Hh[size_t(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const cd x0 = Hh[size_t(i) * m + j], x1 = Hh[size_t(i + 1) * m + j];
                    Hh[size_t(i) * m + j] = cs[a][i] * x0 + sn[a][i] * x1;
                    Hh[size_t(i + 1) * m + j] = -std::conj(sn[a][i]) * x0 + std::conj(cs[a][i]) * x1;
                }
                const cd x0 = Hh[size_t(j) * m + j], x1 = Hh[size_t(j + 1) * m + j];
                const double rho = std::sqrt(std::norm(x0) + std::norm(x1));
                cs[a][j] = rho > 0 ? std::conj(x0) / rho : cd(1.0);
                sn[a][j] = rho > 0 ? std::conj(x1) / rho : cd(0.0);
                Hh[size_t(j) * m + j] = rho;
                Hh[size_t(j + 1) * m + j] = 0.0;
                g[a][j + 1] = -std::conj(sn[a][j]) * g[a][j];
                g[a][j] = cs[a][j] * g[a][j];
                jused[a] = j + 1;
                its[act[a]] += 1;
                est[act[a]] = std::abs(g[a][j + 1]) / bnorm[act[a]];
                if (est[act[a]] <= o.tol || hn == 0.0 || its[act[a]] >= o.max_iter) {
                    live[a] = 0;
                    if (est[act[a]] <= o.tol || hn == 0.0) conv[act[a]] = 1;
                }
                any = any || live[a];
            }
            // the scales go up from the staging buffer without a wait: the host
            // writes it again only after the next step's wait
            double2 *up = stage + 2 * nh + Ra;
            for (int a = 0; a < Ra; ++a) up[a] = make_double2(sc[a].real(), sc[a].imag());
            BEM_HIP(hipMemcpyAsync(hdev.p, up, Ra * sizeof(double2), hipMemcpyHostToDevice, s));
            bscale(s, vj1, vj1, n, Ra, hdev.p);
            ++steps;
            if (o.progress > 0 && steps % o.progress == 0) {
                double worst = 0.0;
                int n_act = 0;
                for (int a = 0; a < Ra; ++a)
                    if (live[a]) { worst = std::max(worst, est[act[a]]); ++n_act; }
                std::fprintf(stderr, "[bem] %s step %ld: %d of %d systems active, worst residual estimate %.3e\n",
                             o.label, steps, n_act, R, worst);
                std::fflush(stderr);
            }
            if (!any) { ++j; break; }
        }
        // x_a += basis * y_a, y_a = H_a^{-1} g_a (upper triangular)
        const int jm = *std::max_element(jused.begin(), jused.end());
        if (jm > 0) {
            std::vector<cd> coef(size_t(Ra) * jm, cd(0));
            for (int a = 0; a < Ra; ++a) {
                const int ju = jused[a];
                std::vector<cd> y(ju);
                for (int i = ju - 1; i >= 0; --i) {
                    cd acc = g[a][i];
                    for (int k = i + 1; k < ju; ++k) acc -= H[a][size_t(i) * m + k] * y[k];
                    y[i] = acc / H[a][size_t(i) * m + i];
                }
                for (int i = 0; i < ju; ++i) coef[size_t(a) * jm + i] = y[i];
            }
            to_dev(coef);
            baxpy(s, M ? Z.p : V.p, ld, jm, hdev.p, Xa.p, n, Ra, 1.0);
        }
        for (int a = 0; a < Ra; ++a)
            BEM_HIP(hipMemcpyAsync(X + int64_t(act[a]) * n, Xa.p + int64_t(a) * n, n * sizeof(double2),
                                   hipMemcpyDeviceToDevice, s));
    }
    // true residuals of the returned iterates
    A(X, V.p, R);
    {
        std::vector<cd> mone(R, cd(-1.0, 0.0)), one(R, cd(1.0, 0.0));
        to_dev(mone);
        bscale(s, V.p, V.p, n, R, hdev.p);
        to_dev(one);
        baxpy(s, B, 0, 1, hdev.p, V.p, n, R, 1.0);
        std::vector<cd> d;
        host_dots(V.p, 0, 1, V.p, R, d);
        for (int r = 0; r < R; ++r) {
            info[r].iterations = its[r];
            info[r].converged = conv[r];
            info[r].rel_residual = bnorm[r] > 0 ? std::sqrt(std::max(0.0, d[r].real())) / bnorm[r] : 0.0;
        }
    }
}

}  // namespace bem
