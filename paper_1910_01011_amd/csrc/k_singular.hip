// FP64 singular pass.  For every ordered pair of touching triangles (same
// boundary; coincident, edge- or vertex-adjacent) and every wavenumber pass that
// covers it, the element matrices of V, K, K' and W are integrated with the
// Sauter-Schwab rules, and the 6-point x 6-point regular rule that the FP32
// far-field kernel applies to the same pair is subtracted (in the coincident
// case without the point-with-itself terms, which that kernel skips).  The
// differences, combined into the PMCHWT blocks
//   DD = -K,  DN = sV V,  ND = sW W,  NN = K'
// are summed per vertex pair into a complex128 CSR in a fixed order.
#include <algorithm>

#include "bem_internal.h"
#include "rule6.h"

namespace bem {

struct SAcc {
    double vr[9], vi[9], kr[9], ki[9], pr[9], pi[9];
    double sgr, sgi;   // sum of w G (curl part of W)
};

// Accumulate one quadrature pair with weight w (sign included).
__device__ __forceinline__ void s_point(const double *x, const double *y, const double *lx, const double *ly,
                                        double w, const double *nt, const double *ns, double kre, double kim,
                                        SAcc &A)
{
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double sn, cs;
    sincos(kre * r, &sn, &cs);
    const double e = (kim != 0.0 ? exp(-kim * r) : 1.0) * 0.079577471545947667884 / r;
    const double gr = e * cs, gi = e * sn;
    // F = G (1 - i k r) / r^2,  1 - i k r = (1 + kim r) - i kre r
    const double a1 = 1.0 + kim * r, b1 = -kre * r, ir2 = 1.0 / (r * r);
    const double fr = (gr * a1 - gi * b1) * ir2, fi = (gr * b1 + gi * a1) * ir2;
    const double dny = dx * ns[0] + dy * ns[1] + dz * ns[2];
    const double dnx = dx * nt[0] + dy * nt[1] + dz * nt[2];
    const double kr_ = fr * dny, ki_ = fi * dny;
    const double pr_ = -fr * dnx, pi_ = -fi * dnx;
    A.sgr += w * gr;
    A.sgi += w * gi;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double wa = w * lx[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double ll = wa * ly[b];
            const int ab = 3 * a + b;
            A.vr[ab] += ll * gr;
            A.vi[ab] += ll * gi;
            A.kr[ab] += ll * kr_;
            A.ki[ab] += ll * ki_;
            A.pr[ab] += ll * pr_;
            A.pi[ab] += ll * pi_;
        }
    }
}

__global__ __launch_bounds__(64) void k_singular(const SingularItem *__restrict__ items, int64_t n_items,
                                                 const PassDesc *__restrict__ passes,
                                                 const double *__restrict__ rule_c, int n_c,
                                                 const double *__restrict__ rule_e, int n_e,
                                                 const double *__restrict__ rule_v, int n_v,
                                                 const double *__restrict__ verts, const int32_t *__restrict__ tris,
                                                 const double *__restrict__ area, const double *__restrict__ normal,
                                                 const double *__restrict__ curl, double2 *__restrict__ out)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n_items) return;
    const SingularItem it = items[idx];
    const PassDesc P = passes[it.pass];
    double Pt[3][3], Ps[3][3], Qt[3][3], Qs[3][3], nt[3], ns[3];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
            Pt[a][d] = verts[3 * int64_t(tris[3 * int64_t(it.t) + a]) + d];
            Ps[a][d] = verts[3 * int64_t(tris[3 * int64_t(it.s) + a]) + d];
            Qt[a][d] = verts[3 * int64_t(tris[3 * int64_t(it.t) + it.pt[a]]) + d];
            Qs[a][d] = verts[3 * int64_t(tris[3 * int64_t(it.s) + it.ps[a]]) + d];
        }
    // position in the permuted order of each original corner (inverse permutation)
    int ipt[3], ips[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ipt[a] = it.pt[0] == a ? 0 : (it.pt[1] == a ? 1 : 2);
        ips[a] = it.ps[0] == a ? 0 : (it.ps[1] == a ? 1 : 2);
    }
    for (int d = 0; d < 3; ++d) {
        nt[d] = normal[3 * int64_t(it.t) + d];
        ns[d] = normal[3 * int64_t(it.s) + d];
    }
    const double at = area[it.t], as = area[it.s];
    SAcc A;
    for (int k = 0; k < 9; ++k) A.vr[k] = A.vi[k] = A.kr[k] = A.ki[k] = A.pr[k] = A.pi[k] = 0.0;
    A.sgr = A.sgi = 0.0;

    // singular rule on T x T with x = Q0 + s1 (Q1 - Q0) + s2 (Q2 - Q1): barycentric
    // (1 - s1, s1 - s2, s2) in the permuted order; Jacobian 2|T| per triangle
    const double *rule = it.cls == COINCIDENT ? rule_c : (it.cls == EDGE ? rule_e : rule_v);
    const int nr = it.cls == COINCIDENT ? n_c : (it.cls == EDGE ? n_e : n_v);
    const double jac = 4.0 * at * as;
    for (int m = 0; m < nr; ++m) {
        const double s1 = rule[5 * m], s2 = rule[5 * m + 1], u1 = rule[5 * m + 2], u2 = rule[5 * m + 3];
        const double w = rule[5 * m + 4] * jac;
        const double bx[3] = {1.0 - s1, s1 - s2, s2}, by[3] = {1.0 - u1, u1 - u2, u2};
        double x[3], y[3], lx[3], ly[3];
        for (int d = 0; d < 3; ++d) {
            x[d] = bx[0] * Qt[0][d] + bx[1] * Qt[1][d] + bx[2] * Qt[2][d];
            y[d] = by[0] * Qs[0][d] + by[1] * Qs[1][d] + by[2] * Qs[2][d];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lx[a] = ipt[a] == 0 ? bx[0] : (ipt[a] == 1 ? bx[1] : bx[2]);
            ly[a] = ips[a] == 0 ? by[0] : (ips[a] == 1 ? by[1] : by[2]);
        }
        s_point(x, y, lx, ly, w, nt, ns, P.kre, P.kim, A);
    }
    // minus the regular 6 x 6 rule (original vertex order)
    for (int q = 0; q < 6; ++q) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = q6_bary[q][0] * Pt[0][d] + q6_bary[q][1] * Pt[1][d] + q6_bary[q][2] * Pt[2][d];
        for (int p = 0; p < 6; ++p) {
            if (it.cls == COINCIDENT && p == q) continue;
            double y[3];
            for (int d = 0; d < 3; ++d) y[d] = q6_bary[p][0] * Ps[0][d] + q6_bary[p][1] * Ps[1][d] + q6_bary[p][2] * Ps[2][d];
            s_point(x, y, q6_bary[q], q6_bary[p], -(at * q6_w[q]) * (as * q6_w[p]), nt, ns, P.kre, P.kim, A);
        }
    }
    // PMCHWT blocks; W = curl_a . curl_b sum(w G) - k^2 (n_t . n_s) V
    const double nn = nt[0] * ns[0] + nt[1] * ns[1] + nt[2] * ns[2];
    const double k2r = P.kre * P.kre - P.kim * P.kim, k2i = 2.0 * P.kre * P.kim;
    double2 *o = out + 36 * idx;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const int ab = 3 * a + b;
            const double cc = curl[9 * int64_t(it.t) + 3 * a] * curl[9 * int64_t(it.s) + 3 * b] +
                              curl[9 * int64_t(it.t) + 3 * a + 1] * curl[9 * int64_t(it.s) + 3 * b + 1] +
                              curl[9 * int64_t(it.t) + 3 * a + 2] * curl[9 * int64_t(it.s) + 3 * b + 2];
            const double wr = cc * A.sgr - nn * (k2r * A.vr[ab] - k2i * A.vi[ab]);
            const double wi = cc * A.sgi - nn * (k2r * A.vi[ab] + k2i * A.vr[ab]);
            o[ab] = make_double2(-A.kr[ab], -A.ki[ab]);
            o[9 + ab] = make_double2(P.sV * A.vr[ab], P.sV * A.vi[ab]);
            o[18 + ab] = make_double2(P.sW * wr, P.sW * wi);
            o[27 + ab] = make_double2(A.pr[ab], A.pi[ab]);
        }
}

// cval[e][blk] = sum over the contributions listed for slot e (in item order)
__global__ void k_correction_sum(const double2 *__restrict__ elem, const int32_t *__restrict__ cptr_,
                                 const int32_t *__restrict__ cidx, int64_t nnz, double2 *__restrict__ cval)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    double2 s[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int32_t k = cptr_[e]; k < cptr_[e + 1]; ++k) {
        const int32_t c = cidx[k];
        const int64_t item = c / 9;
        const int ab = c - 9 * int(item);
        for (int blk = 0; blk < 4; ++blk) {
            const double2 v = elem[36 * item + 9 * blk + ab];
            s[blk].x += v.x;
            s[blk].y += v.y;
        }
    }
    for (int blk = 0; blk < 4; ++blk) cval[4 * e + blk] = s[blk];
}

template <typename T>
static T *dev_upload(const std::vector<T> &h, hipStream_t s)
{
    T *d = nullptr;
    dmalloc(reinterpret_cast<void **>(&d), std::max<size_t>(1, h.size()) * sizeof(T));
    if (!h.empty()) BEM_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

void run_singular(bem_problem &p, const std::vector<SingularItem> &items, int32_t **d_cptr, int32_t **d_ccol,
                  double2 **d_cval, int64_t *nnz_out)
{
    std::vector<int32_t> cptr, ccol, contrib_ptr, contrib_idx;
    correction_pattern(p, items, cptr, ccol, contrib_ptr, contrib_idx);
    const int64_t nnz = cptr[p.NV];
    *nnz_out = nnz;
    *d_cptr = dev_upload(cptr, p.stream);
    *d_ccol = dev_upload(ccol, p.stream);
    dmalloc(reinterpret_cast<void **>(d_cval), std::max<int64_t>(1, 4 * nnz) * sizeof(double2));

    const std::vector<double> rc = singular_rule(COINCIDENT, p.ss_order);
    const std::vector<double> re = singular_rule(EDGE, p.ss_order);
    const std::vector<double> rv = singular_rule(VERTEX, p.ss_order);
    double *d_rc = dev_upload(rc, p.stream), *d_re = dev_upload(re, p.stream), *d_rv = dev_upload(rv, p.stream);
    SingularItem *d_items = dev_upload(items, p.stream);
    PassDesc *d_passes = dev_upload(p.passes, p.stream);
    int32_t *d_cp = dev_upload(contrib_ptr, p.stream), *d_ci = dev_upload(contrib_idx, p.stream);
    double2 *d_elem = nullptr;
    const int64_t n_items = int64_t(items.size());
    dmalloc(reinterpret_cast<void **>(&d_elem), std::max<int64_t>(1, 36 * n_items) * sizeof(double2));
    if (n_items > 0) {
        const int B = 64;
        k_singular<<<dim3(blocks_1d(n_items, B)), dim3(B), 0, p.stream>>>(
            d_items, n_items, d_passes, d_rc, int(rc.size() / 5), d_re, int(re.size() / 5), d_rv, int(rv.size() / 5),
            p.d_verts, p.d_tris, p.d_area, p.d_normal, p.d_curl, d_elem);
        BEM_HIP(hipGetLastError());
    }
    if (nnz > 0) {
        const int B = 256;
        k_correction_sum<<<dim3(blocks_1d(nnz, B)), dim3(B), 0, p.stream>>>(d_elem, d_cp, d_ci, nnz, *d_cval);
        BEM_HIP(hipGetLastError());
    }
    BEM_HIP(hipStreamSynchronize(p.stream));
    dfree(d_rc); dfree(d_re); dfree(d_rv); dfree(d_items); dfree(d_passes);
    dfree(d_cp); dfree(d_ci); dfree(d_elem);
}

}  // namespace bem
