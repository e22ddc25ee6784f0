// Host runtime of the C ABI declared in include/bem.h: problem set-up on the
// device, the operator apply, GMRES and the right-hand side / field entry points.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "bem_internal.h"

namespace {

thread_local std::string g_last_error;

bem_status fail(bem_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

template <typename F>
bem_status guarded(F &&f)
{
    try {
        return f();
    } catch (const bem::Error &e) {
        return fail(e.status, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(BEM_ERR_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(BEM_ERR_DEVICE, e.what());
    }
}

template <typename T>
void dev_alloc(T **p, size_t n)
{
    bem::dmalloc(reinterpret_cast<void **>(p), std::max<size_t>(1, n) * sizeof(T));
}

template <typename T>
T *dev_copy(const std::vector<T> &h, hipStream_t s)
{
    T *d = nullptr;
    dev_alloc(&d, h.size());
    if (!h.empty()) BEM_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

void free_problem(bem_problem *p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    bem::AllocScope alloc_scope(p->stream);
    void *ptrs[] = {p->d_verts, p->d_tris, p->d_rowD, p->d_rowN, p->d_area, p->d_normal, p->d_curl, p->d_pts,
                    p->d_tnrm, p->d_v2t_ptr, p->d_v2t, p->d_pass, p->d_work, p->d_trial, p->d_part, p->d_pot,
                    p->d_cptr, p->d_ccol, p->d_cval, p->d_x, p->d_y, p->d_A, p->d_Ahi, p->d_Alo,
                    p->d_gx, p->d_gc, p->d_aptr, p->d_acol, p->d_Mv, p->d_Sv, p->d_adiag, p->d_drange,
                    p->d_sl_cptr, p->d_sl_ccol, p->d_sl_cval, p->d_cg_chunks, p->d_ell_col, p->d_ell_mv,
                    p->d_ell_sv, p->d_mdiag};
    for (void *q : ptrs)
        if (q) bem::dfree(q);
    if (p->hm) bem::hmatrix_free(p->hm);
    if (p->osrc) bem::osrc_free(p->osrc, p->stream);
    if (p->batch) bem::batch_detach(*p);
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->batch_ready) (void)hipEventDestroy(p->batch_ready);
    if (p->batch_done) (void)hipEventDestroy(p->batch_done);
    delete p;
}

// Validated host copies of the domains' meshes and media (no device work).
void load_domains(bem_problem &p, const bem_domain *domains, int32_t n_domains)
{
    int64_t voff = 0, toff = 0;
    for (int j = 0; j < n_domains; ++j) {
        const bem_domain &d = domains[j];
        bem::validate_mesh(d.vertices, d.n_vertices, d.triangles, d.n_triangles, j);
        bem::DomInfo di{d.n_vertices, d.n_triangles, voff, toff, d.k.re, d.k.im, d.rho};
        p.doms.push_back(di);
        p.h_verts.insert(p.h_verts.end(), d.vertices, d.vertices + 3 * d.n_vertices);
        for (int64_t i = 0; i < 3 * d.n_triangles; ++i) p.h_tris.push_back(int32_t(d.triangles[i] + voff));
        voff += d.n_vertices;
        toff += d.n_triangles;
    }
    p.NV = voff;
    p.NT = toff;
    p.M = 6 * toff;
    p.N = 2 * voff;
    if (p.M >= (int64_t(1) << 31) / 10) throw bem::Error{BEM_ERR_INVALID_ARG, "problem too large for 32-bit indexing"};
    bem::validate_disjoint(p.doms, p.h_verts);
}

bool finite_c(const bem_complex &z) { return std::isfinite(z.re) && std::isfinite(z.im); }

void build_work(bem_problem &p);

// Far-field pass table and work list.
void build_passes(bem_problem &p)
{
    using bem::PassDesc;
    p.passes.clear();
    PassDesc ext{};
    ext.test_begin = 0;
    ext.test_end = p.M;
    ext.trial_begin = 0;
    ext.trial_end = p.M;
    ext.kre = p.k0re;
    ext.kim = p.k0im;
    ext.sV = 1.0;
    ext.sW = 1.0;
    ext.slot = 0;
    p.passes.push_back(ext);
    for (const auto &d : p.doms) {
        PassDesc q{};
        // whole triangles: the pair kernel's trial tiles and records are per triangle
        q.test_begin = 6 * d.t_off;
        q.test_end = 6 * (d.t_off + d.nt);
        q.trial_begin = q.test_begin;
        q.trial_end = q.test_end;
        q.kre = d.kre;
        q.kim = d.kim;
        q.sV = d.rho / p.rho0;
        q.sW = p.rho0 / d.rho;
        q.slot = 1;
        p.passes.push_back(q);
    }
    p.n_pass = int(p.passes.size());
    // largest phase of any pair: bounding-box diagonal of all vertices times
    // the largest real wavenumber, in revolutions (the hardware sine and
    // cosine reduce arguments below 256 revolutions themselves)
    {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = 0; i < p.NV; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], p.h_verts[3 * size_t(i) + d]);
                hi[d] = std::max(hi[d], p.h_verts[3 * size_t(i) + d]);
            }
        double diag = 0.0, kmax = 0.0;
        for (int d = 0; d < 3; ++d) diag += (hi[d] - lo[d]) * (hi[d] - lo[d]);
        for (const auto &q : p.passes) kmax = std::max(kmax, std::abs(q.kre));
        p.wrap_phase = !(std::sqrt(diag) * kmax / (2.0 * M_PI) < 128.0);
    }
    std::vector<bem::PassDev> dv;
    for (const auto &q : p.passes) {
        bem::PassDev d{};
        d.test_begin = q.test_begin;
        d.test_end = q.test_end;
        d.trial_begin = q.trial_begin;
        d.trial_end = q.trial_end;
        d.k = float(q.kre);
        d.k_over_2pi = float(q.kre / (2.0 * M_PI));
        d.kim = float(q.kim);
        d.sV = float(q.sV);
        d.sW = float(q.sW);
        d.k2re = float(q.kre * q.kre - q.kim * q.kim);
        d.k2im = float(2.0 * q.kre * q.kim);
        d.slot = q.slot;
        dv.push_back(d);
    }
    p.d_pass = dev_copy(dv, p.stream);
    build_work(p);
}

// Work list of the pair kernel for the current (tpl, n_split).
void build_work(bem_problem &p)
{
    if (p.d_work) {
        BEM_HIP(hipStreamSynchronize(p.stream));
        bem::dfree(p.d_work);
        p.d_work = nullptr;
    }
    // work items: consecutive workgroups take consecutive splits, so that the
    // round-robin placement of workgroups on the 8 XCDs keeps one trial chunk
    // per XCD (its L2 holds that chunk).
    const int tb = 256 * p.tpl;
    std::vector<int4> work;
    for (int ip = 0; ip < p.n_pass; ++ip) {
        const int64_t nblk = (p.passes[ip].test_end - p.passes[ip].test_begin + tb - 1) / tb;
        for (int64_t b = 0; b < nblk; ++b)
            for (int s = 0; s < p.n_split; ++s) work.push_back(make_int4(ip, int(b), s, 0));
    }
    p.n_work = int(work.size());
    p.d_work = dev_copy(work, p.stream);
}

void ensure_scratch(bem_problem &p, int64_t n_rhs)
{
    if (p.scratch_rhs >= n_rhs) return;
    if (p.d_x) bem::dfree(p.d_x);
    if (p.d_y) bem::dfree(p.d_y);
    p.d_x = p.d_y = nullptr;
    p.scratch_rhs = 0;
    dev_alloc(&p.d_x, size_t(n_rhs * p.N));
    dev_alloc(&p.d_y, size_t(n_rhs * p.N));
    p.scratch_rhs = n_rhs;
}

// y = A x for one right-hand side, all on the device.
void apply_one(bem_problem &p, const double2 *x, double2 *y, int parts, bool record)
{
    if (record) BEM_HIP(hipEventRecord(p.ev[0], p.stream));
    if (parts & 1) {
        bem::launch_gather(p, x);
        if (record) BEM_HIP(hipEventRecord(p.ev[1], p.stream));
        bem::launch_pairs(p);
        if (record) BEM_HIP(hipEventRecord(p.ev[2], p.stream));
        bem::launch_reduce(p);
    } else if (record) {
        BEM_HIP(hipEventRecord(p.ev[1], p.stream));
        BEM_HIP(hipEventRecord(p.ev[2], p.stream));
    }
    if (record) BEM_HIP(hipEventRecord(p.ev[3], p.stream));
    bem::launch_scatter(p, x, y, parts);
    if (record) {
        BEM_HIP(hipEventRecord(p.ev[4], p.stream));
        p.timed = true;
    }
}

// y = A x with the dense matrix (assembled modes); events as in apply_one.
void apply_dense_one(bem_problem &p, const double2 *x, double2 *y, bool record)
{
    if (record) {
        BEM_HIP(hipEventRecord(p.ev[0], p.stream));
        BEM_HIP(hipEventRecord(p.ev[1], p.stream));
    }
    bem::launch_gemv(p, x, y);
    if (record) {
        BEM_HIP(hipEventRecord(p.ev[2], p.stream));
        BEM_HIP(hipEventRecord(p.ev[3], p.stream));
        BEM_HIP(hipEventRecord(p.ev[4], p.stream));
        p.timed = true;
    }
}

// Y = A X for several right-hand sides in one GEMM (assembled modes).
void grow(void **ptr, size_t &have, size_t need)
{
    if (have >= need) return;
    if (*ptr) bem::dfree(*ptr);
    *ptr = nullptr;
    have = 0;
    bem::dmalloc(ptr, need);
    have = need;
}

// search: allow the K-slice search for an untuned bucket (the solvers pass
// false: they take a cached choice, else the heuristic, so that no timing runs
// inside a solve).
// force_shape >= 0: that split-BF16 tile shape with heuristic K slices (no tuning).
void apply_dense_multi(bem_problem &p, const double2 *X, double2 *Y, int n_rhs, bool bf16, bool search = true,
                       int force_shape = -1)
{
    int code = 0;   // 100 * tile shape + K slices (0: heuristic)
    if (force_shape >= 0) {
        code = 100 * force_shape;
    } else if ((p.flags & BEM_AUTOTUNE) && !search) {
        code = bem::cached_gemm_slices(p, n_rhs, bf16);
    } else if (p.flags & BEM_AUTOTUNE) {
        // scratch for every candidate (K-slice partials capped at 4 GB), then tune once per bucket
        size_t cmax = 0;
        for (int shape = 0; shape < 2; ++shape)
            for (int s : {1, 2, 4, 8, 16, 32, 64}) {
                const bem::GemmPlan c = bem::gemm_plan(p, n_rhs, bf16, s, shape);
                if (c.bytes_c <= (size_t(4) << 30)) cmax = std::max(cmax, c.bytes_c);
            }
        const bem::GemmPlan g0 = bem::gemm_plan(p, n_rhs, bf16, 1);
        BEM_HIP(hipStreamSynchronize(p.stream));
        grow(&p.d_gx, p.gx_bytes, g0.bytes_x);
        grow(reinterpret_cast<void **>(&p.d_gc), p.gc_bytes, cmax);
        code = bem::tune_gemm_slices(p, n_rhs, bf16, p.d_gx, p.d_gc, Y);
    }
    const bem::GemmPlan g = bem::gemm_plan(p, n_rhs, bf16, code % 100, code / 100);
    if (p.gx_bytes < g.bytes_x) {
        if (p.d_gx) bem::dfree(p.d_gx);
        p.d_gx = nullptr;
        p.gx_bytes = 0;
        bem::dmalloc(&p.d_gx, g.bytes_x);
        p.gx_bytes = g.bytes_x;
    }
    if (p.gc_bytes < g.bytes_c) {
        if (p.d_gc) bem::dfree(p.d_gc);
        p.d_gc = nullptr;
        p.gc_bytes = 0;
        bem::dmalloc(reinterpret_cast<void **>(&p.d_gc), g.bytes_c);
        p.gc_bytes = g.bytes_c;
    }
    BEM_HIP(hipEventRecord(p.ev[0], p.stream));
    p.timed_gemm = true;
    bem::launch_gemm(p, g, X, Y, p.d_gx, p.d_gc);
    BEM_HIP(hipEventRecord(p.ev[3], p.stream));
    BEM_HIP(hipEventRecord(p.ev[4], p.stream));
    p.timed = true;
}

void apply_device(bem_problem &p, const double2 *x, double2 *y, int n_rhs, int parts, bool search = true)
{
    if (p.mode != BEM_OTF && n_rhs > 1) {
        apply_dense_multi(p, x, y, n_rhs, p.mode == BEM_ASSEMBLED_SPLIT_BF16, search);
        return;
    }
    for (int r = 0; r < n_rhs; ++r) {
        if (p.mode != BEM_OTF)
            apply_dense_one(p, x + int64_t(r) * p.N, y + int64_t(r) * p.N, r == n_rhs - 1);
        else
            apply_one(p, x + int64_t(r) * p.N, y + int64_t(r) * p.N, parts, r == n_rhs - 1);
    }
}

// OSRC inner-solve tolerance inside a solve: the caller's osrc_tol, else ten
// times tighter than the tolerance of the GMRES it preconditions (tol for the
// plain forms; inner_tol for the flexible forms, whose inner solves only
// need to reach inner_tol: the outer iteration corrects the rest), within
// [1e-10, 1e-4].  On the rib-cage stack's flexible solve 1e-4 instead of 1e-6
// saves a fifth of the time at the same outer iterations; 1e-3 stalls the
// inner solves.
double osrc_inner_tol(const bem_solve_opts &o)
{
    if (o.osrc_tol > 0) return o.osrc_tol;
    const double inner = (o.precision == BEM_PREC_FP32 || o.precision == BEM_PREC_HMATRIX) ? o.tol : o.inner_tol;
    return std::min(1e-4, std::max(1e-10, 0.1 * inner));
}

bem_solve_opts default_solve_opts()
{
    bem_solve_opts o{};
    o.tol = 1e-5;
    o.restart = 100;
    o.max_iter = 1000;
    o.precond = BEM_PRECOND_NONE;
    o.n_pade = 4;
    o.r_eps = 0.1;
    o.theta = M_PI / 3.0;
    o.precision = BEM_PREC_FP32;
    o.inner_restart = 30;
    o.inner_max_iter = 300;
    o.inner_tol = 1e-3;
    return o;
}

// ||b_r - (Ax)_r|| / ||b_r|| for R vectors (Ax is overwritten)
std::vector<double> residual_norms(bem_problem &p, const double2 *B, double2 *AX, int R)
{
    const int64_t n = p.N;
    const int nblk = bem::bdot_chunks(n);
    double2 *part = nullptr, *h = nullptr;
    dev_alloc(&part, size_t(R) * nblk);
    dev_alloc(&h, size_t(R));
    std::vector<double2> ones(R, make_double2(1.0, 0.0)), out(R);
    BEM_HIP(hipMemcpyAsync(h, ones.data(), R * sizeof(double2), hipMemcpyHostToDevice, p.stream));
    bem::baxpy(p.stream, B, 0, 1, h, AX, n, R, -1.0);
    bem::bdot(p.stream, AX, 0, 1, AX, n, R, part, nblk, h);
    BEM_HIP(hipMemcpyAsync(out.data(), h, R * sizeof(double2), hipMemcpyDeviceToHost, p.stream));
    std::vector<double2> bb(R);
    bem::bdot(p.stream, B, 0, 1, B, n, R, part, nblk, h);
    BEM_HIP(hipMemcpyAsync(bb.data(), h, R * sizeof(double2), hipMemcpyDeviceToHost, p.stream));
    BEM_HIP(hipStreamSynchronize(p.stream));
    bem::dfree(part);
    bem::dfree(h);
    std::vector<double> r(R);
    for (int i = 0; i < R; ++i) r[i] = bb[i].x > 0 ? std::sqrt(std::max(0.0, out[i].x) / bb[i].x) : 0.0;
    return r;
}

}  // namespace

namespace bem {
void set_error(const std::string &msg) { g_last_error = msg; }

void apply_dense_multi_dispatch(bem_problem &p, const double2 *X, double2 *Y, int R, bool bf16)
{
    apply_dense_multi(p, X, Y, R, bf16, false);
}

hipStream_t &alloc_stream()
{
    thread_local hipStream_t s = nullptr;
    return s;
}

void dmalloc(void **p, size_t bytes)
{
    *p = nullptr;
    BEM_HIP(hipMallocAsync(p, std::max<size_t>(1, bytes), alloc_stream()));
}

void dfree(void *p)
{
    if (p) (void)hipFreeAsync(p, alloc_stream());
}
}  // namespace bem

extern "C" {

const char *bem_last_error(void) { return g_last_error.c_str(); }

bem_status bem_assemble(const bem_domain *domains, int32_t n_domains, bem_complex k0, double rho0,
                        const bem_assemble_opts *opts, bem_problem **out)
{
    if (!out) return fail(BEM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!domains || n_domains < 1) return fail(BEM_ERR_INVALID_ARG, "need at least one domain");
    if (!finite_c(k0) || k0.im < 0 || !(rho0 > 0) || !std::isfinite(rho0))
        return fail(BEM_ERR_INVALID_ARG, "k0 must be finite with Im k0 >= 0 and rho0 > 0");
    bem_assemble_opts o{};
    o.mode = BEM_OTF;
    o.far_points = 6;
    o.ss_order = 6;
    if (opts) o = *opts;
    if (o.far_points == 0) o.far_points = 6;
    if (o.ss_order == 0) o.ss_order = 6;
    if (o.far_points != 6) return fail(BEM_ERR_UNSUPPORTED, "only the 6-point far rule is implemented");
    if (o.ss_order < 1 || o.ss_order > 16) return fail(BEM_ERR_INVALID_ARG, "ss_order must be in 1..16");
    if (o.mode != BEM_OTF && o.mode != BEM_ASSEMBLED_FP32 && o.mode != BEM_ASSEMBLED_SPLIT_BF16)
        return fail(BEM_ERR_INVALID_ARG, "unknown operator mode");
    if (k0.re <= 0) return fail(BEM_ERR_INVALID_ARG, "Re k0 must be positive");
    for (int j = 0; j < n_domains; ++j) {
        const bem_domain &d = domains[j];
        if (!d.vertices || !d.triangles) return fail(BEM_ERR_INVALID_ARG, "domain " + std::to_string(j) + ": NULL mesh");
        if (!finite_c(d.k) || d.k.im < 0 || d.k.re <= 0)
            return fail(BEM_ERR_INVALID_ARG, "domain " + std::to_string(j) + ": k must be finite, Re k > 0, Im k >= 0");
        if (!(d.rho > 0) || !std::isfinite(d.rho))
            return fail(BEM_ERR_INVALID_ARG, "domain " + std::to_string(j) + ": rho must be positive");
    }
    bem_problem *p = new bem_problem;
    bem_status st = guarded([&]() -> bem_status {
        p->device = o.device;
        p->stream = static_cast<hipStream_t>(o.stream);
        p->flags = o.flags;
        p->mode = o.mode;
        p->ss_order = o.ss_order;
        p->k0re = k0.re;
        p->k0im = k0.im;
        p->rho0 = rho0;
        load_domains(*p, domains, n_domains);
        p->h_rowD.resize(p->NV);
        p->h_rowN.resize(p->NV);
        for (const auto &d : p->doms)
            for (int64_t i = 0; i < d.nv; ++i) {
                p->h_rowD[d.v_off + i] = int32_t(2 * d.v_off + i);
                p->h_rowN[d.v_off + i] = int32_t(2 * d.v_off + d.nv + i);
            }
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        for (auto &e : p->ev) BEM_HIP(hipEventCreate(&e));
        p->d_verts = dev_copy(p->h_verts, p->stream);
        p->d_tris = dev_copy(p->h_tris, p->stream);
        p->d_rowD = dev_copy(p->h_rowD, p->stream);
        p->d_rowN = dev_copy(p->h_rowN, p->stream);
        dev_alloc(&p->d_area, p->NT);
        dev_alloc(&p->d_normal, 3 * p->NT);
        dev_alloc(&p->d_curl, 9 * p->NT);
        dev_alloc(&p->d_pts, 3 * p->M);
        dev_alloc(&p->d_tnrm, 3 * p->NT);
        // vertex -> (triangle, corner)
        std::vector<int32_t> vptr(p->NV + 1, 0), vlst(3 * p->NT);
        for (int64_t i = 0; i < 3 * p->NT; ++i) vptr[p->h_tris[i] + 1]++;
        for (int64_t i = 0; i < p->NV; ++i) vptr[i + 1] += vptr[i];
        {
            std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
            for (int64_t t = 0; t < p->NT; ++t)
                for (int a = 0; a < 3; ++a) vlst[fill[p->h_tris[3 * t + a]]++] = int32_t(3 * t + a);
        }
        p->d_v2t_ptr = dev_copy(vptr, p->stream);
        p->d_v2t = dev_copy(vlst, p->stream);
        bem::launch_geometry(*p);
        // far-field work decomposition: at least ~8 workgroups per CU
        p->tpl = 1;
        const int64_t blocks = (p->M + 255) / 256;
        p->n_split = int(std::clamp<int64_t>((8 * 256 + blocks - 1) / std::max<int64_t>(1, blocks), 1, 64));
        if (p->n_split > 1) p->n_split = std::min(64, (p->n_split + 7) / 8 * 8);
        build_passes(*p);
        dev_alloc(&p->d_trial, size_t(2 * p->M + 3 * p->NT));   // point records, then triangle records
        dev_alloc(&p->d_pot, size_t(10) * p->M);
        if ((o.flags & BEM_AUTOTUNE) && o.mode == BEM_OTF) {
            // partial sums for the largest candidate (at most 2 GB), then the choice
            int max_split = 64;
            while (max_split > 1 && size_t(2) * max_split * 10 * p->M * sizeof(double) > (size_t(2) << 30)) max_split /= 2;
            dev_alloc(&p->d_part, size_t(2) * max_split * 10 * p->M);
            bem::tune_pairs(*p, &build_work, max_split);
            BEM_HIP(hipStreamSynchronize(p->stream));
            bem::dfree(p->d_part);
            p->d_part = nullptr;
        }
        dev_alloc(&p->d_part, size_t(2) * p->n_split * 10 * p->M);
        // every (slot, split, point) partial is written by one work item on each
        // apply; zero once anyway so a pass with an empty range cannot leave garbage
        BEM_HIP(hipMemsetAsync(p->d_part, 0, size_t(2) * p->n_split * 10 * p->M * sizeof(double), p->stream));
        // singular correction
        std::vector<bem::SingularItem> items;
        bem::touching_pairs(*p, items);
        bem::run_singular(*p, items, &p->d_cptr, &p->d_ccol, &p->d_cval, &p->nnz);
        if (p->mode != BEM_OTF) {
            dev_alloc(&p->d_A, size_t(p->N) * size_t(p->N));
            bem::launch_assemble_dense(*p);
            if (p->mode == BEM_ASSEMBLED_SPLIT_BF16) bem::split_matrix_bf16(*p);
        }
        BEM_HIP(hipStreamSynchronize(p->stream));
        return BEM_OK;
    });
    if (st != BEM_OK) {
        free_problem(p);
        return st;
    }
    *out = p;
    return BEM_OK;
}

void bem_destroy(bem_problem *p) { free_problem(p); }

int64_t bem_num_unknowns(const bem_problem *p) { return p ? p->N : -1; }

bem_status bem_apply_parts(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs, int parts)
{
    if (!p || !x || !y || n_rhs < 0) return fail(BEM_ERR_INVALID_ARG, "bem_apply: bad arguments");
    if (parts < 0 || parts > 3) return fail(BEM_ERR_INVALID_ARG, "bem_apply: parts must be 0..3");
    if (p->mode != BEM_OTF && parts != 3)
        return fail(BEM_ERR_UNSUPPORTED, "bem_apply: an assembled matrix holds both parts together");
    if (n_rhs == 0) return BEM_OK;
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        const size_t bytes = size_t(n_rhs) * p->N * sizeof(double2);
        if (p->flags & BEM_DEVICE_PTRS) {
            apply_device(*p, reinterpret_cast<const double2 *>(x), reinterpret_cast<double2 *>(y), n_rhs, parts);
        } else {
            for (int64_t i = 0; i < int64_t(n_rhs) * p->N; ++i)
                if (!finite_c(x[i])) return fail(BEM_ERR_INVALID_ARG, "bem_apply: non-finite input");
            ensure_scratch(*p, n_rhs);
            BEM_HIP(hipMemcpyAsync(p->d_x, x, bytes, hipMemcpyHostToDevice, p->stream));
            apply_device(*p, p->d_x, p->d_y, n_rhs, parts);
            BEM_HIP(hipMemcpyAsync(y, p->d_y, bytes, hipMemcpyDeviceToHost, p->stream));
            BEM_HIP(hipStreamSynchronize(p->stream));
        }
        return BEM_OK;
    });
}

bem_status bem_apply_single_layer(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs)
{
    if (!p || !x || !y || n_rhs < 0) return fail(BEM_ERR_INVALID_ARG, "bem_apply_single_layer: bad arguments");
    if (n_rhs == 0) return BEM_OK;
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        if (!p->sl_ready) {
            // V correction of the exterior pass: its touching pairs, V block only
            std::vector<bem::SingularItem> items, ext;
            bem::touching_pairs(*p, items);
            for (const auto &it : items)
                if (it.pass == 0) ext.push_back(it);
            bem::run_singular(*p, ext, &p->d_sl_cptr, &p->d_sl_ccol, &p->d_sl_cval, &p->sl_nnz);
            p->sl_ready = true;
        }
        const int64_t nv = p->NV;
        const size_t bytes = size_t(n_rhs) * nv * sizeof(double2);
        const double2 *dx = reinterpret_cast<const double2 *>(x);
        double2 *dy = reinterpret_cast<double2 *>(y);
        if (!(p->flags & BEM_DEVICE_PTRS)) {
            for (int64_t i = 0; i < int64_t(n_rhs) * nv; ++i)
                if (!finite_c(x[i])) return fail(BEM_ERR_INVALID_ARG, "bem_apply_single_layer: non-finite input");
            ensure_scratch(*p, n_rhs);   // N = 2 NV per right-hand side: room for NV
            BEM_HIP(hipMemcpyAsync(p->d_x, x, bytes, hipMemcpyHostToDevice, p->stream));
            dx = p->d_x;
            dy = p->d_y;
        }
        for (int r = 0; r < n_rhs; ++r)
            bem::launch_single_layer(*p, dx + int64_t(r) * nv, dy + int64_t(r) * nv, r == n_rhs - 1);
        if (!(p->flags & BEM_DEVICE_PTRS)) {
            BEM_HIP(hipMemcpyAsync(y, p->d_y, bytes, hipMemcpyDeviceToHost, p->stream));
            BEM_HIP(hipStreamSynchronize(p->stream));
        }
        return BEM_OK;
    });
}

bem_status bem_apply(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs)
{
    return bem_apply_parts(p, x, y, n_rhs, 3);
}

bem_status bem_apply_noalloc(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs)
{
    if (!p || !x || !y || n_rhs < 0) return fail(BEM_ERR_INVALID_ARG, "bem_apply_noalloc: bad arguments");
    if (p->mode != BEM_OTF) return fail(BEM_ERR_INVALID_ARG, "bem_apply_noalloc: on-the-fly problems only");
    if (!(p->flags & BEM_DEVICE_PTRS))
        return fail(BEM_ERR_INVALID_ARG, "bem_apply_noalloc: needs device vectors (assemble with BEM_DEVICE_PTRS)");
    // scratch layout: trial records, pair-kernel partial sums, point potentials
    const auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t trial_b = up(sizeof(float4) * size_t(2 * p->M + 3 * p->NT));
    const size_t part_b = up(sizeof(double) * size_t(2) * p->n_split * 10 * size_t(p->M));
    const size_t pot_b = up(sizeof(double) * size_t(10) * p->M);
    if (trial_b + part_b + pot_b > bem::NOALLOC_SCRATCH_BYTES)
        return fail(BEM_ERR_UNSUPPORTED, "bem_apply_noalloc: the problem needs " + std::to_string(trial_b + part_b + pot_b) +
                                             " bytes of scratch, more than the " +
                                             std::to_string(bem::NOALLOC_SCRATCH_BYTES) + " available");
    if (n_rhs == 0) return BEM_OK;
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        char *base = static_cast<char *>(bem::noalloc_scratch(p->device));
        float4 *trial = reinterpret_cast<float4 *>(base);
        double *part = reinterpret_cast<double *>(base + trial_b);
        double *pot = reinterpret_cast<double *>(base + trial_b + part_b);
        // the array keeps the previous call's contents: clear the partial sums
        bem::launch_zero_f64(p->stream, part, int64_t(2) * p->n_split * 10 * p->M);
        struct Swap {
            bem_problem &q;
            float4 *t;
            double *a, *b;
            ~Swap() { q.d_trial = t; q.d_part = a; q.d_pot = b; }
        } restore{*p, p->d_trial, p->d_part, p->d_pot};
        p->d_trial = trial;
        p->d_part = part;
        p->d_pot = pot;
        apply_device(*p, reinterpret_cast<const double2 *>(x), reinterpret_cast<double2 *>(y), n_rhs, 3, false);
        return BEM_OK;
    });
}

bem_status bem_apply_with(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs, int kernel)
{
    if (!p || !x || !y || n_rhs < 0) return fail(BEM_ERR_INVALID_ARG, "bem_apply_with: bad arguments");
    if (kernel < BEM_APPLY_DEFAULT || kernel > BEM_APPLY_HMATRIX)
        return fail(BEM_ERR_INVALID_ARG, "bem_apply_with: unknown kernel");
    if (kernel == BEM_APPLY_DEFAULT) return bem_apply_parts(p, x, y, n_rhs, 3);
    if (kernel == BEM_APPLY_HMATRIX) {
        if (!p->hm) return fail(BEM_ERR_INVALID_ARG, "bem_apply_with: no hierarchical matrix (bem_hmatrix_build)");
        if (n_rhs == 0) return BEM_OK;
        return guarded([&]() -> bem_status {
            BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
            const size_t bytes = size_t(n_rhs) * p->N * sizeof(double2);
            if (p->flags & BEM_DEVICE_PTRS) {
                bem::hmatrix_apply(*p, reinterpret_cast<const double2 *>(x), reinterpret_cast<double2 *>(y), n_rhs, true);
            } else {
                ensure_scratch(*p, n_rhs);
                BEM_HIP(hipMemcpyAsync(p->d_x, x, bytes, hipMemcpyHostToDevice, p->stream));
                bem::hmatrix_apply(*p, p->d_x, p->d_y, n_rhs, true);
                BEM_HIP(hipMemcpyAsync(y, p->d_y, bytes, hipMemcpyDeviceToHost, p->stream));
                BEM_HIP(hipStreamSynchronize(p->stream));
            }
            return BEM_OK;
        });
    }
    if (p->mode == BEM_OTF) return fail(BEM_ERR_INVALID_ARG, "bem_apply_with: on-the-fly problems have no dense kernels");
    const bool split = kernel >= BEM_APPLY_MFMA_SPLIT_BF16;
    if (split && p->mode != BEM_ASSEMBLED_SPLIT_BF16)
        return fail(BEM_ERR_INVALID_ARG, "bem_apply_with: no BF16 planes (assemble with BEM_ASSEMBLED_SPLIT_BF16)");
    if (n_rhs == 0) return BEM_OK;
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        const size_t bytes = size_t(n_rhs) * p->N * sizeof(double2);
        const double2 *dx = reinterpret_cast<const double2 *>(x);
        double2 *dy = reinterpret_cast<double2 *>(y);
        if (!(p->flags & BEM_DEVICE_PTRS)) {
            ensure_scratch(*p, n_rhs);
            BEM_HIP(hipMemcpyAsync(p->d_x, x, bytes, hipMemcpyHostToDevice, p->stream));
            dx = p->d_x;
            dy = p->d_y;
        }
        if (kernel == BEM_APPLY_GEMV) {
            for (int r = 0; r < n_rhs; ++r)
                apply_dense_one(*p, dx + int64_t(r) * p->N, dy + int64_t(r) * p->N, r == n_rhs - 1);
        } else {
            const int shape = kernel == BEM_APPLY_MFMA_SPLIT_BF16_W4 ? 0 : kernel == BEM_APPLY_MFMA_SPLIT_BF16_W8 ? 1 : -1;
            apply_dense_multi(*p, dx, dy, n_rhs, split, true, shape);
        }
        if (!(p->flags & BEM_DEVICE_PTRS)) {
            BEM_HIP(hipMemcpyAsync(y, p->d_y, bytes, hipMemcpyDeviceToHost, p->stream));
            BEM_HIP(hipStreamSynchronize(p->stream));
        }
        return BEM_OK;
    });
}

bem_status bem_hmatrix_build(bem_problem *p, double eps, int32_t leaf_vertices, double eta, bem_hmatrix_info *info)
{
    if (!p) return fail(BEM_ERR_INVALID_ARG, "bem_hmatrix_build: bad arguments");
    if (!(eps > 0 && eps <= 0.1) || leaf_vertices < 8 || leaf_vertices > 4096 || !(eta > 0) || !std::isfinite(eta))
        return fail(BEM_ERR_INVALID_ARG, "bem_hmatrix_build: need 0 < eps <= 0.1, 8 <= leaf_vertices <= 4096, eta > 0");
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        if (p->hm) {
            bem::hmatrix_free(p->hm);
            p->hm = nullptr;
        }
        p->hm = bem::hmatrix_build(*p, eps, leaf_vertices, eta, info);
        return BEM_OK;
    });
}

bem_status bem_hmatrix_plan(const bem_domain *domains, int32_t n_domains, int32_t leaf_vertices, double eta,
                            int64_t *out4)
{
    if (!domains || n_domains < 1 || !out4) return fail(BEM_ERR_INVALID_ARG, "bem_hmatrix_plan: bad arguments");
    if (leaf_vertices < 8 || leaf_vertices > 4096 || !(eta > 0) || !std::isfinite(eta))
        return fail(BEM_ERR_INVALID_ARG, "bem_hmatrix_plan: need 8 <= leaf_vertices <= 4096, eta > 0");
    for (int j = 0; j < n_domains; ++j)
        if (!domains[j].vertices || !domains[j].triangles)
            return fail(BEM_ERR_INVALID_ARG, "domain " + std::to_string(j) + ": NULL mesh");
    return guarded([&]() -> bem_status {
        bem_problem p;
        load_domains(p, domains, n_domains);
        bem::hmatrix_plan(p, leaf_vertices, eta, out4);
        return BEM_OK;
    });
}

bem_status bem_pair_launch_shape(const bem_problem *p, int32_t *out2)
{
    if (!p || !out2) return fail(BEM_ERR_INVALID_ARG, "bem_pair_launch_shape: bad arguments");
    out2[0] = p->tpl;
    out2[1] = p->n_split;
    return BEM_OK;
}

bem_status bem_last_timings(const bem_problem *p, double *ms4)
{
    if (!p || !ms4) return fail(BEM_ERR_INVALID_ARG, "bem_last_timings: bad arguments");
    if (!p->timed) return fail(BEM_ERR_INVALID_ARG, "bem_last_timings: no apply recorded yet");
    return guarded([&]() -> bem_status {
        BEM_HIP(hipEventSynchronize(p->ev[4]));
        float t[4];
        BEM_HIP(hipEventElapsedTime(&t[0], p->ev[0], p->ev[4]));
        BEM_HIP(hipEventElapsedTime(&t[1], p->ev[1], p->ev[2]));
        BEM_HIP(hipEventElapsedTime(&t[2], p->ev[3], p->ev[4]));
        BEM_HIP(hipEventElapsedTime(&t[3], p->ev[0], p->ev[1]));
        for (int i = 0; i < 4; ++i) ms4[i] = t[i];
        return BEM_OK;
    });
}

bem_status bem_rhs(bem_problem *p, const bem_incident *inc, bem_complex *b)
{
    if (!p || !inc || !b || !inc->params || inc->n_fields < 1)
        return fail(BEM_ERR_INVALID_ARG, "bem_rhs: bad arguments");
    if (inc->kind < BEM_PLANE_WAVE || inc->kind > BEM_PISTON_ARRAY)
        return fail(BEM_ERR_INVALID_ARG, "bem_rhs: unknown incident kind");
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        const size_t n = size_t(inc->n_fields) * p->N;
        if (p->flags & BEM_DEVICE_PTRS) {
            bem::launch_rhs(*p, *inc, reinterpret_cast<double2 *>(b));
        } else {
            double2 *d_b = nullptr;
            dev_alloc(&d_b, n);
            bem::launch_rhs(*p, *inc, d_b);
            BEM_HIP(hipMemcpy(b, d_b, n * sizeof(double2), hipMemcpyDeviceToHost));
            bem::dfree(d_b);
        }
        return BEM_OK;
    });
}

bem_status bem_solve_rhs(bem_problem *p, const bem_complex *b, int32_t n_rhs, const bem_solve_opts *opts,
                         bem_complex *u, bem_solve_info *info)
{
    if (!p || !b || !u || !info || n_rhs < 1) return fail(BEM_ERR_INVALID_ARG, "bem_solve: bad arguments");
    bem_solve_opts o = opts ? *opts : default_solve_opts();
    if (!(o.tol > 0) || o.restart < 1 || o.max_iter < 1) return fail(BEM_ERR_INVALID_ARG, "bem_solve: bad options");
    if (o.precond != BEM_PRECOND_NONE && o.precond != BEM_PRECOND_OSRC && o.precond != BEM_PRECOND_OSRC_LEFT)
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: unknown preconditioner");
    if (o.precond != BEM_PRECOND_NONE) {
        if (!(o.r_eps > 0) || !std::isfinite(o.r_eps) || o.n_pade < 0 || o.n_pade > 64 || !std::isfinite(o.theta))
            return fail(BEM_ERR_INVALID_ARG, "bem_solve: OSRC needs r_eps > 0, 0 <= n_pade <= 64, finite theta");
    }
    if (o.inner_restart == 0) o.inner_restart = 30;
    if (o.inner_max_iter == 0) o.inner_max_iter = 300;
    if (o.inner_restart < 1 || o.inner_max_iter < 1)
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: inner_restart and inner_max_iter must be positive (0: default)");
    if (o.precision != BEM_PREC_FP32 && o.precision != BEM_PREC_SPLIT_BF16_FGMRES &&
        o.precision != BEM_PREC_FP32_MFMA_FGMRES && o.precision != BEM_PREC_HMATRIX &&
        o.precision != BEM_PREC_HMATRIX_FGMRES)
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: unknown precision mode");
    if ((o.precision == BEM_PREC_HMATRIX || o.precision == BEM_PREC_HMATRIX_FGMRES) && !p->hm)
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: no hierarchical matrix (bem_hmatrix_build)");
    if (o.precision == BEM_PREC_FP32_MFMA_FGMRES && p->mode == BEM_OTF)
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: MFMA refinement needs an assembled problem");
    if (o.precision == BEM_PREC_SPLIT_BF16_FGMRES && p->mode != BEM_ASSEMBLED_SPLIT_BF16)
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: split-BF16 refinement needs a problem assembled in split-BF16 mode");
    const bool plain = o.precision == BEM_PREC_FP32 || o.precision == BEM_PREC_HMATRIX;
    if (!plain && !(o.inner_tol > 0 && o.inner_tol < 1))
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: inner_tol must be in (0, 1)");
    if (!(o.osrc_tol >= 0 && o.osrc_tol < 1))
        return fail(BEM_ERR_INVALID_ARG, "bem_solve: osrc_tol must be in [0, 1) (0: 1e-10)");
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        const size_t n = size_t(n_rhs) * p->N;
        const double2 *db;
        double2 *du;
        double2 *tb = nullptr, *tu = nullptr;
        if (p->flags & BEM_DEVICE_PTRS) {
            db = reinterpret_cast<const double2 *>(b);
            du = reinterpret_cast<double2 *>(u);
        } else {
            for (size_t i = 0; i < n; ++i)
                if (!finite_c(b[i])) return fail(BEM_ERR_INVALID_ARG, "bem_solve: non-finite right-hand side");
            dev_alloc(&tb, n);
            dev_alloc(&tu, n);
            BEM_HIP(hipMemcpyAsync(tb, b, n * sizeof(double2), hipMemcpyHostToDevice, p->stream));
            db = tb;
            du = tu;
        }
        bem_problem &P = *p;
        const char *pe = std::getenv("BEM_PROGRESS");
        const int progress = pe ? std::max(0, std::atoi(pe)) : 0;
        // FP32-accurate operator: on-the-fly kernel, or the FP32 dense matrix
        // (GEMV with FP64 accumulation for one vector, FP32 MFMA GEMM for a block)
        const bool hmat = o.precision == BEM_PREC_HMATRIX;
        // a problem attached to a batch hands its operator applies to the
        // batch (continuous batching across concurrent solves)
        struct InSolve {
            bem_batch *b;
            explicit InSolve(bem_batch *x) : b(x) { if (b) bem::batch_enter(*b); }
            ~InSolve() { if (b) bem::batch_leave(*b); }
        } in_solve(P.batch);
        const bem::ApplyFn fp32_apply = [&P, hmat](const double2 *X, double2 *Y, int R) {
            if (P.batch) {
                bem::batch_apply(P, hmat ? bem::BATCH_HMATRIX : P.mode == BEM_OTF ? bem::BATCH_OTF : bem::BATCH_GEMV, X,
                                 Y, R);
            } else if (hmat) {
                bem::hmatrix_apply(P, X, Y, R, false);
            } else if (P.mode == BEM_OTF) {
                apply_device(P, X, Y, R, 3, false);
            } else {
                for (int r = 0; r < R; ++r) apply_dense_one(P, X + int64_t(r) * P.N, Y + int64_t(r) * P.N, true);
            }
        };
        if (plain && o.precond == BEM_PRECOND_OSRC) {
            // right preconditioning: GMRES on A P y = b, u = P y, with the
            // preconditioned vectors kept (flexible form, so an inexact inner
            // solve is harmless); the Arnoldi residual is that of the
            // unpreconditioned weak-form system, which is what stops it
            const bem::OsrcParams op{o.n_pade, o.r_eps, o.theta, osrc_inner_tol(o), 3000};
            const bem::ApplyFn prec = [&P, op](const double2 *V, double2 *Z, int R) { bem::osrc_apply(P, op, V, Z, R); };
            bem::gmres_batch(P, P.N, n_rhs, db, du, bem::KrylovOpts{o.tol, o.restart, o.max_iter, progress, "osrc gmres"},
                             fp32_apply, &prec, info);
        } else if (plain && o.precond == BEM_PRECOND_OSRC_LEFT) {
            // left preconditioning (the paper's form): GMRES on P A u = P b,
            // stopping on the preconditioned residual; the unpreconditioned
            // weak-form residual is reported afterwards
            const bem::OsrcParams op{o.n_pade, o.r_eps, o.theta, osrc_inner_tol(o), 3000};
            double2 *PB = nullptr, *tmp = nullptr;
            dev_alloc(&PB, n);
            dev_alloc(&tmp, n);
            struct G2 {
                double2 *a, *b;
                ~G2() { bem::dfree(a); bem::dfree(b); }
            } g2{PB, tmp};
            bem::osrc_apply(P, op, db, PB, n_rhs);
            const bem::ApplyFn prec_apply = [&P, &fp32_apply, op, tmp](const double2 *X, double2 *Y, int R) {
                fp32_apply(X, tmp, R);
                bem::osrc_apply(P, op, tmp, Y, R);
            };
            bem::gmres_batch(P, P.N, n_rhs, PB, du, bem::KrylovOpts{o.tol, o.restart, o.max_iter, progress},
                             prec_apply, nullptr, info);
            fp32_apply(du, tmp, n_rhs);
            const std::vector<double> rr = residual_norms(P, db, tmp, n_rhs);
            for (int r = 0; r < n_rhs; ++r) info[r].rel_residual = rr[r];
        } else if (plain) {
            bem::gmres_batch(P, P.N, n_rhs, db, du, bem::KrylovOpts{o.tol, o.restart, o.max_iter, progress},
                             fp32_apply, nullptr, info);
        } else {
            // flexible GMRES: outer Arnoldi on the FP32 matrix with FP64
            // accumulation, inner GMRES on the 3-term split-BF16 GEMM
            // (for the hierarchical matrix: outer on the FP32 operator of the
            // problem's mode, on the fly or dense; inner on the compressed one)
            const bool hinner = o.precision == BEM_PREC_HMATRIX_FGMRES;
            const bem::ApplyFn outer = [&P, &fp32_apply, hinner](const double2 *X, double2 *Y, int R) {
                if (hinner) {
                    fp32_apply(X, Y, R);
                    return;
                }
                if (P.batch) {
                    bem::batch_apply(P, bem::BATCH_GEMV, X, Y, R);
                    return;
                }
                for (int r = 0; r < R; ++r) apply_dense_one(P, X + int64_t(r) * P.N, Y + int64_t(r) * P.N, true);
            };
            const bool bf16 = o.precision == BEM_PREC_SPLIT_BF16_FGMRES;
            const bem::ApplyFn inner_op = [&P, bf16, hinner](const double2 *X, double2 *Y, int R) {
                if (P.batch)
                    bem::batch_apply(P, hinner ? bem::BATCH_HMATRIX : bf16 ? bem::BATCH_GEMM_BF16 : bem::BATCH_GEMM_F32,
                                     X, Y, R);
                else if (hinner) bem::hmatrix_apply(P, X, Y, R, false);
                else apply_dense_multi(P, X, Y, R, bf16, false);
            };
            const bem::KrylovOpts io{o.inner_tol, o.inner_restart, o.inner_max_iter, progress, "inner gmres"};
            bem::ApplyFn prec;
            double2 *PV = nullptr, *tmp = nullptr;
            struct G2 {
                double2 *a = nullptr, *b = nullptr;
                ~G2() { bem::dfree(a); bem::dfree(b); }
            } g2;
            if (o.precond != BEM_PRECOND_NONE) {
                // inner GMRES on the left-preconditioned system P A z = P v
                const bem::OsrcParams op{o.n_pade, o.r_eps, o.theta, osrc_inner_tol(o), 3000};
                dev_alloc(&PV, n);
                dev_alloc(&tmp, n);
                g2.a = PV;
                g2.b = tmp;
                prec = [&P, &inner_op, io, op, PV, tmp](const double2 *V, double2 *Z, int R) {
                    bem::osrc_apply(P, op, V, PV, R);
                    const bem::ApplyFn pa = [&P, &inner_op, op, tmp](const double2 *X, double2 *Y, int Ri) {
                        inner_op(X, tmp, Ri);
                        bem::osrc_apply(P, op, tmp, Y, Ri);
                    };
                    std::vector<bem_solve_info> ii(R);
                    bem::gmres_batch(P, P.N, R, PV, Z, io, pa, nullptr, ii.data());
                };
            } else {
                prec = [&P, &inner_op, io](const double2 *V, double2 *Z, int R) {
                    std::vector<bem_solve_info> ii(R);
                    bem::gmres_batch(P, P.N, R, V, Z, io, inner_op, nullptr, ii.data());
                };
            }
            bem::gmres_batch(P, P.N, n_rhs, db, du,
                             bem::KrylovOpts{o.tol, o.restart, o.max_iter, progress, "outer fgmres"}, outer, &prec,
                             info);
        }
        bool all = true;
        for (int r = 0; r < n_rhs; ++r) all = all && info[r].converged;
        if (!(p->flags & BEM_DEVICE_PTRS)) {
            BEM_HIP(hipMemcpyAsync(u, du, n * sizeof(double2), hipMemcpyDeviceToHost, p->stream));
            BEM_HIP(hipStreamSynchronize(p->stream));
            bem::dfree(tb);
            bem::dfree(tu);
        }
        if (!all) return fail(BEM_WARN_NOT_CONVERGED, "bem_solve: GMRES reached max_iter for some right-hand side");
        return BEM_OK;
    });
}

bem_status bem_apply_preconditioner(bem_problem *p, const bem_solve_opts *opts, const bem_complex *y,
                                    bem_complex *out, int32_t n_rhs)
{
    if (!p || !opts || !y || !out || n_rhs < 0) return fail(BEM_ERR_INVALID_ARG, "bem_apply_preconditioner: bad arguments");
    if (opts->precond != BEM_PRECOND_OSRC && opts->precond != BEM_PRECOND_OSRC_LEFT)
        return fail(BEM_ERR_INVALID_ARG, "bem_apply_preconditioner: precond must be OSRC");
    if (!(opts->r_eps > 0) || opts->n_pade < 0 || opts->n_pade > 64 || !std::isfinite(opts->theta))
        return fail(BEM_ERR_INVALID_ARG, "bem_apply_preconditioner: need r_eps > 0, 0 <= n_pade <= 64");
    if (!(opts->osrc_tol >= 0 && opts->osrc_tol < 1))
        return fail(BEM_ERR_INVALID_ARG, "bem_apply_preconditioner: osrc_tol must be in [0, 1)");
    if (n_rhs == 0) return BEM_OK;
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        const bem::OsrcParams op{opts->n_pade, opts->r_eps, opts->theta, opts->osrc_tol > 0 ? opts->osrc_tol : 1e-10, 3000};
        const size_t n = size_t(n_rhs) * p->N;
        if (p->flags & BEM_DEVICE_PTRS) {
            bem::osrc_apply(*p, op, reinterpret_cast<const double2 *>(y), reinterpret_cast<double2 *>(out), n_rhs);
            BEM_HIP(hipStreamSynchronize(p->stream));
        } else {
            double2 *dy = nullptr, *dout = nullptr;
            dev_alloc(&dy, n);
            dev_alloc(&dout, n);
            BEM_HIP(hipMemcpy(dy, y, n * sizeof(double2), hipMemcpyHostToDevice));
            bem::osrc_apply(*p, op, dy, dout, n_rhs);
            BEM_HIP(hipStreamSynchronize(p->stream));
            BEM_HIP(hipMemcpy(out, dout, n * sizeof(double2), hipMemcpyDeviceToHost));
            bem::dfree(dy);
            bem::dfree(dout);
        }
        return BEM_OK;
    });
}

bem_status bem_solve(bem_problem *p, const bem_incident *inc, const bem_solve_opts *opts, bem_complex *u,
                     bem_solve_info *info)
{
    if (!p || !inc || !u || !info || inc->n_fields < 1) return fail(BEM_ERR_INVALID_ARG, "bem_solve: bad arguments");
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        const size_t n = size_t(inc->n_fields) * p->N;
        double2 *d_b = nullptr;
        dev_alloc(&d_b, n);
        bem::launch_rhs(*p, *inc, d_b);
        const uint32_t saved = p->flags;
        bem_status st;
        if (saved & BEM_DEVICE_PTRS) {
            st = bem_solve_rhs(p, reinterpret_cast<bem_complex *>(d_b), inc->n_fields, opts, u, info);
        } else {
            std::vector<bem_complex> hb(n);
            BEM_HIP(hipMemcpy(hb.data(), d_b, n * sizeof(double2), hipMemcpyDeviceToHost));
            st = bem_solve_rhs(p, hb.data(), inc->n_fields, opts, u, info);
        }
        bem::dfree(d_b);
        return st;
    });
}

bem_status bem_evaluate_field(bem_problem *p, const bem_complex *u, const bem_incident *inc, const double *points,
                              int64_t n_points, bem_complex *field, int32_t *region)
{
    if (!p || !u || !points || !field || !region || n_points < 0)
        return fail(BEM_ERR_INVALID_ARG, "bem_evaluate_field: bad arguments");
    const int n_fields = inc ? inc->n_fields : 1;
    return guarded([&]() -> bem_status {
        BEM_HIP(hipSetDevice(p->device));
        bem::AllocScope alloc_scope(p->stream);
        if (p->flags & BEM_DEVICE_PTRS) {
            bem::launch_field(*p, reinterpret_cast<const double2 *>(u), inc, n_fields, points, n_points,
                              reinterpret_cast<double2 *>(field), region);
        } else {
            double2 *du = nullptr, *df = nullptr;
            double *dp = nullptr;
            int32_t *dr = nullptr;
            dev_alloc(&du, size_t(n_fields) * p->N);
            dev_alloc(&df, size_t(n_fields) * n_points);
            dev_alloc(&dp, size_t(3 * n_points));
            dev_alloc(&dr, size_t(n_points));
            BEM_HIP(hipMemcpy(du, u, size_t(n_fields) * p->N * sizeof(double2), hipMemcpyHostToDevice));
            BEM_HIP(hipMemcpy(dp, points, size_t(3 * n_points) * sizeof(double), hipMemcpyHostToDevice));
            bem::launch_field(*p, du, inc, n_fields, dp, n_points, df, dr);
            BEM_HIP(hipMemcpy(field, df, size_t(n_fields) * n_points * sizeof(double2), hipMemcpyDeviceToHost));
            BEM_HIP(hipMemcpy(region, dr, size_t(n_points) * sizeof(int32_t), hipMemcpyDeviceToHost));
            bem::dfree(du); bem::dfree(df); bem::dfree(dp); bem::dfree(dr);
        }
        return BEM_OK;
    });
}

bem_status bem_footprint_bytes(const bem_domain *domains, int32_t n_domains, const bem_assemble_opts *opts,
                               int32_t n_rhs, int32_t restart, uint64_t *bytes)
{
    if (!domains || n_domains < 1 || !bytes || n_rhs < 0 || restart < 0)
        return fail(BEM_ERR_INVALID_ARG, "bem_footprint_bytes: bad arguments");
    uint64_t nv = 0, nt = 0;
    for (int j = 0; j < n_domains; ++j) {
        nv += uint64_t(domains[j].n_vertices);
        nt += uint64_t(domains[j].n_triangles);
    }
    const uint64_t M = 6 * nt, N = 2 * nv;
    const uint64_t n_split = 16;
    uint64_t b = 0;
    b += nv * 24 + nt * 12 + nv * 8;              // vertices, triangles, row maps
    b += nt * (8 + 24 + 72 + 12) + M * 12;        // geometry, points
    b += M * 32 + nt * 48 + 2 * n_split * 10 * M * 8 + M * 80;   // trial records, partials, potentials
    b += nv * 24 * (4 + 4 * 64);                  // correction CSR (about 24 entries per row)
    b += uint64_t(n_rhs) * N * 16 * 2;            // x, y
    b += uint64_t(restart + 1) * N * 16 * uint64_t(n_rhs > 0 ? n_rhs : 1);   // Krylov bases
    const int mode = opts ? opts->mode : BEM_OTF;
    if (mode != BEM_OTF) {
        b += 8 * N * N;                                               // complex64 matrix
        if (mode == BEM_ASSEMBLED_SPLIT_BF16) b += 8 * N * N;        // BF16 hi/lo planes
        const uint64_t Np = ((2 * uint64_t(n_rhs) + 127) / 128) * 128;
        b += Np * 2 * N * 4 + 16 * N * Np * 4;                        // packed X, K-slice partials
    }
    *bytes = b;
    return BEM_OK;
}

}  // extern "C"
