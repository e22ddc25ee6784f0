// Incident fields, right-hand sides and the field off the surface.
//
// Right-hand side (eq. Galerkin_disc_rhs1): b_D[g] = <p_inc, phi_g>,
// b_N[g] = <dp_inc/dn, phi_g>, integrated with the 6-point rule per triangle.
// Incident kinds:
//   plane wave    p = A exp(i k0 d.x)
//   point sources p = sum_s a_s exp(i k0 |x - s|) / (4 pi |x - s|)
//   pistons       flat baffled discs, p(x) = (-i k0 / 2 pi) int_disc exp(i k0 r)/r dS
//                 (unit rho c u), each discretised by 3 Gauss-Legendre radii
//                 (weight r dr) times 8 equal angles, i.e. a sum of 24 monopoles.
// Field (eq. rep_formula_gen): exterior p = p_inc + sum_j [DL_k0 u_D - SL_k0 u_N],
// inside domain j p = SL_kj((rho_j/rho_0) u_N) - DL_kj u_D, 6-point rule on the
// sources; the region comes from the solid-angle winding number of each domain.
// Points closer than 2 h_j to boundary j (h_j its mean edge length) are flagged
// with region -1; their field is still computed, with the winding-number region.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "bem_internal.h"
#include "rule6.h"

namespace bem {

constexpr double PI_D = 3.14159265358979323846;

// Device form of an incident field: plane waves keep their parameters
// ([n_fields][5]: unit direction, amplitude); point sources and pistons become
// one list of monopoles ([n][5]: position, complex amplitude) sorted by field,
// fptr[f] .. fptr[f + 1] the monopoles of field f.
struct IncDev {
    int kind;
    int n_fields;
    const double *params;   // plane waves (device copy)
    const double *src;      // monopoles (device copy)
    const int32_t *fptr;
    double k0re, k0im;
};

// monopole exp(i k |x - s|) / (4 pi |x - s|) and its gradient . n, times amplitude a
__device__ __forceinline__ void monopole(const double *x, const double *nrm, const double *s, double ar, double ai,
                                         double kre, double kim, double &pr, double &pi, double &qr, double &qi)
{
    const double dx = x[0] - s[0], dy = x[1] - s[1], dz = x[2] - s[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double sn, cs;
    sincos(kre * r, &sn, &cs);
    const double e = exp(-kim * r) / (4.0 * PI_D * r);
    const double gr = e * cs, gi = e * sn;
    const double vr = gr * ar - gi * ai, vi = gr * ai + gi * ar;   // a G
    pr += vr;
    pi += vi;
    // grad G . n = G (i k r - 1) / r^2 (x - s) . n,  i k r = -kim r + i kre r
    const double dn = (dx * nrm[0] + dy * nrm[1] + dz * nrm[2]) / (r * r);
    const double cr = -kim * r - 1.0, ci = kre * r;
    qr += (vr * cr - vi * ci) * dn;
    qi += (vr * ci + vi * cr) * dn;
}

// p_inc and dp_inc/dn of field f at x (normal nrm)
__device__ void incident(const IncDev &I, int f, const double *x, const double *nrm, double &pr, double &pi,
                         double &qr, double &qi)
{
    pr = pi = qr = qi = 0.0;
    if (I.kind == BEM_PLANE_WAVE) {
        const double *P = I.params + 5 * int64_t(f);
        const double dx = P[0] * x[0] + P[1] * x[1] + P[2] * x[2];
        const double dn = P[0] * nrm[0] + P[1] * nrm[1] + P[2] * nrm[2];
        double sn, cs;
        sincos(I.k0re * dx, &sn, &cs);
        const double e = exp(-I.k0im * dx);
        const double er = e * cs, ei = e * sn;
        pr = P[3] * er - P[4] * ei;
        pi = P[3] * ei + P[4] * er;
        // i k0 (d.n) p
        const double kr = -I.k0im * dn, ki = I.k0re * dn;
        qr = kr * pr - ki * pi;
        qi = kr * pi + ki * pr;
    } else {
        for (int32_t s = I.fptr[f]; s < I.fptr[f + 1]; ++s) {
            const double *S = I.src + 5 * int64_t(s);
            monopole(x, nrm, S, S[3], S[4], I.k0re, I.k0im, pr, pi, qr, qi);
        }
    }
}

// p_inc and dp_inc/dn of every field of [f0, f0 + gridDim.y) at every
// quadrature point 6 t + q: PQ[(f - f0) M + i] = (p, dp/dn) as two double2
__global__ void k_inc_points(IncDev I, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                             const double *__restrict__ normal, int64_t M, int f0, double2 *__restrict__ PQ)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t t = i / 6;
    const int q = int(i - 6 * t);
    const int f = f0 + int(blockIdx.y);
    double x[3];
    for (int d = 0; d < 3; ++d)
        x[d] = q6_bary[q][0] * verts[3 * int64_t(tris[3 * t]) + d] + q6_bary[q][1] * verts[3 * int64_t(tris[3 * t + 1]) + d] +
               q6_bary[q][2] * verts[3 * int64_t(tris[3 * t + 2]) + d];
    double pr, pi, qr, qi;
    incident(I, f, x, normal + 3 * t, pr, pi, qr, qi);
    double2 *o = PQ + 2 * (int64_t(blockIdx.y) * M + i);
    o[0] = make_double2(pr, pi);
    o[1] = make_double2(qr, qi);
}

// b_D[g] = sum over the corners (t, a) at g and the points q of
// w_t,q lambda_a(q) p_inc, b_N likewise with dp_inc/dn: one thread per
// (vertex, field of the chunk), the point values from k_inc_points
__global__ void k_rhs_scatter(const double2 *__restrict__ PQ, int64_t M, int f0, const double *__restrict__ area,
                              const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                              const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN, int64_t NV, int64_t N,
                              double2 *__restrict__ b)
{
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= NV) return;
    const int64_t fl = blockIdx.y, f = f0 + fl;
    double bDr = 0, bDi = 0, bNr = 0, bNi = 0;
    for (int32_t k = v2t_ptr[g]; k < v2t_ptr[g + 1]; ++k) {
        const int64_t t = v2t[k] / 3;
        const int a = v2t[k] - 3 * int(t);
        for (int q = 0; q < 6; ++q) {
            const double2 *v = PQ + 2 * (fl * M + 6 * t + q);
            const double w = area[t] * q6_w[q] * q6_bary[q][a];
            bDr += w * v[0].x; bDi += w * v[0].y;
            bNr += w * v[1].x; bNi += w * v[1].y;
        }
    }
    b[f * N + rowD[g]] = make_double2(bDr, bDi);
    b[f * N + rowN[g]] = make_double2(bNr, bNi);
}

// device scratch of one call, freed on every exit path (hipFree waits for the device)
struct DevScratch {
    void *p = nullptr;
    DevScratch() = default;
    DevScratch(const DevScratch &) = delete;
    DevScratch &operator=(const DevScratch &) = delete;
    ~DevScratch()
    {
        if (p) dfree(p);
    }
};

// Plane waves: directions normalised.  Point sources and pistons: one list of
// monopoles sorted by field (stable: the order of the parameters within a
// field); a piston is 3 Gauss-Legendre radii (weight r dr) times 8 equal
// angles of its disc, amplitude (-i k0 / 2 pi) * 4 pi * w_r r dtheta * A (G
// carries 1/(4 pi)).  Sources whose field index is outside [0, n_fields)
// contribute to no field.  One device allocation (*d_params) holds it all.
static IncDev upload_incident(bem_problem &p, const bem_incident &inc, double **d_params)
{
    IncDev I{};
    I.kind = inc.kind;
    I.n_fields = inc.n_fields;
    I.k0re = p.k0re;
    I.k0im = p.k0im;
    if (inc.kind == BEM_PLANE_WAVE) {
        std::vector<double> h(inc.params, inc.params + int64_t(inc.n_fields) * 5);
        for (int64_t f = 0; f < inc.n_fields; ++f) {
            double *d = &h[5 * f];
            const double l = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int c = 0; c < 3; ++c) d[c] /= l;
        }
        dmalloc(reinterpret_cast<void **>(d_params), std::max<size_t>(1, h.size()) * sizeof(double));
        BEM_HIP(hipMemcpyAsync(*d_params, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, p.stream));
        BEM_HIP(hipStreamSynchronize(p.stream));   // h is pageable and goes out of scope
        I.params = *d_params;
        return I;
    }
    const int64_t cols = inc.kind == BEM_POINT_SOURCES ? 6 : 10;
    const int nf = inc.n_fields;
    std::vector<std::vector<double>> per(size_t(std::max(1, nf)));
    for (int64_t s = 0; s < inc.n_params; ++s) {
        const double *P = inc.params + s * cols;
        const double fd = P[cols - 1];
        if (!(fd >= 0.0) || int64_t(fd) >= nf) continue;
        std::vector<double> &o = per[size_t(int64_t(fd))];
        if (inc.kind == BEM_POINT_SOURCES) {
            o.insert(o.end(), {P[0], P[1], P[2], P[3], P[4]});
            continue;
        }
        double nv[3] = {P[3], P[4], P[5]};
        const double ln = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        for (int d = 0; d < 3; ++d) nv[d] /= ln;
        // orthonormal in-plane basis (e1, e2) of the disc
        double ax[3] = {0, 0, 0};
        const double anx = std::fabs(nv[0]), any = std::fabs(nv[1]), anz = std::fabs(nv[2]);
        ax[(anx <= any && anx <= anz) ? 0 : (any <= anz ? 1 : 2)] = 1.0;
        double e1[3] = {nv[1] * ax[2] - nv[2] * ax[1], nv[2] * ax[0] - nv[0] * ax[2], nv[0] * ax[1] - nv[1] * ax[0]};
        const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (int d = 0; d < 3; ++d) e1[d] /= l1;
        const double e2[3] = {nv[1] * e1[2] - nv[2] * e1[1], nv[2] * e1[0] - nv[0] * e1[2],
                              nv[0] * e1[1] - nv[1] * e1[0]};
        const double gx[3] = {0.11270166537925831148, 0.5, 0.88729833462074168852};
        const double gw[3] = {0.27777777777777777778, 0.44444444444444444444, 0.27777777777777777778};
        const double a = P[6], br = 2.0 * p.k0im, bi = -2.0 * p.k0re;   // -2 i k0
        for (int i = 0; i < 3; ++i) {
            const double rho = a * gx[i];
            const double wgt = a * gw[i] * rho * (2.0 * PI_D / 8.0);
            for (int j = 0; j < 8; ++j) {
                const double th = 2.0 * PI_D * j / 8.0;
                const double ct = std::cos(th), st = std::sin(th);
                o.insert(o.end(), {P[0] + rho * (ct * e1[0] + st * e2[0]), P[1] + rho * (ct * e1[1] + st * e2[1]),
                                   P[2] + rho * (ct * e1[2] + st * e2[2]), wgt * (br * P[7] - bi * P[8]),
                                   wgt * (br * P[8] + bi * P[7])});
            }
        }
    }
    std::vector<double> src;
    std::vector<int32_t> fptr(size_t(nf) + 1, 0);
    for (int f = 0; f < nf; ++f) {
        src.insert(src.end(), per[size_t(f)].begin(), per[size_t(f)].end());
        if (src.size() / 5 > size_t(INT32_MAX)) throw Error{BEM_ERR_UNSUPPORTED, "incident field: too many sources"};
        fptr[size_t(f) + 1] = int32_t(src.size() / 5);
    }
    const size_t nsrc = src.size();
    const size_t ptr_doubles = (fptr.size() * sizeof(int32_t) + sizeof(double) - 1) / sizeof(double);
    dmalloc(reinterpret_cast<void **>(d_params), std::max<size_t>(1, nsrc + ptr_doubles) * sizeof(double));
    if (nsrc) BEM_HIP(hipMemcpyAsync(*d_params, src.data(), nsrc * sizeof(double), hipMemcpyHostToDevice, p.stream));
    int32_t *dptr = reinterpret_cast<int32_t *>(*d_params + nsrc);
    BEM_HIP(hipMemcpyAsync(dptr, fptr.data(), fptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, p.stream));
    // the host vectors go out of scope: the copies must be done first
    BEM_HIP(hipStreamSynchronize(p.stream));
    I.src = *d_params;
    I.fptr = dptr;
    return I;
}

void launch_rhs(bem_problem &p, const bem_incident &inc, double2 *b)
{
    double *d_params = nullptr;
    DevScratch params_mem, pq_mem;
    IncDev I = upload_incident(p, inc, &d_params);
    params_mem.p = d_params;
    // point values of a chunk of fields (at most 1 GiB), then the scatter
    const int64_t per_field = 2 * p.M * int64_t(sizeof(double2));
    const int chunk = int(std::max<int64_t>(1, std::min<int64_t>(inc.n_fields, (int64_t(1) << 30) / per_field)));
    dmalloc(&pq_mem.p, size_t(chunk) * size_t(per_field));
    double2 *PQ = static_cast<double2 *>(pq_mem.p);
    for (int f0 = 0; f0 < inc.n_fields; f0 += chunk) {
        const int nf = std::min(chunk, inc.n_fields - f0);
        k_inc_points<<<dim3(blocks_1d(p.M, 128), unsigned(nf)), dim3(128), 0, p.stream>>>(I, p.d_verts, p.d_tris,
                                                                                         p.d_normal, p.M, f0, PQ);
        BEM_HIP(hipGetLastError());
        k_rhs_scatter<<<dim3(blocks_1d(p.NV, 128), unsigned(nf)), dim3(128), 0, p.stream>>>(
            PQ, p.M, f0, p.d_area, p.d_v2t_ptr, p.d_v2t, p.d_rowD, p.d_rowN, p.NV, p.N, b);
        BEM_HIP(hipGetLastError());
    }
    BEM_HIP(hipStreamSynchronize(p.stream));
}

constexpr int FIELD_DIRECT_MAX = 4;                   // more fields: rows + dense product
constexpr int64_t FIELD_ROWS_BYTES = int64_t(512) << 20;   // row buffer of one chunk of points
constexpr int64_t FIELD_TARGET_THREADS = int64_t(256) * 4 * 8 * 64;   // eight waves per SIMD
constexpr int FIELD_MAX_SPLIT = 64;

struct DomDev {
    long long v_off, t_off, nt, nv;
    double kre, kim, rho;
    double h;   // mean edge length of the boundary mesh
};

// squared distance from the origin to the triangle (a, b, c): the foot of the
// perpendicular if it falls inside (same side of all three edges as the
// normal), else the nearest point of the three edges
__device__ double seg_dist2(const double *p, const double *q)
{
    const double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double t = fmin(1.0, fmax(0.0, -(p[0] * d[0] + p[1] * d[1] + p[2] * d[2]) / dd));
    const double v[3] = {p[0] + t * d[0], p[1] + t * d[1], p[2] + t * d[2]};
    return v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
}

__device__ double tri_dist2(const double *a, const double *b, const double *c)
{
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    const double s = (n[0] * a[0] + n[1] * a[1] + n[2] * a[2]) / nn;
    const double f[3] = {s * n[0], s * n[1], s * n[2]};   // foot of the perpendicular
    const double *v[3] = {a, b, c};
    bool inside = true;
    for (int e = 0; e < 3; ++e) {
        const double *p = v[e], *q = v[(e + 1) % 3];
        const double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]}, w[3] = {f[0] - p[0], f[1] - p[1], f[2] - p[2]};
        const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        if (cr[0] * n[0] + cr[1] * n[1] + cr[2] * n[2] < 0.0) inside = false;
    }
    if (inside) return f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
    return fmin(seg_dist2(a, b), fmin(seg_dist2(b, c), seg_dist2(c, a)));
}

// one thread per point: region by winding numbers (wreg) and the reported
// region code (-1 within 2 h of a boundary)
// Split s of S of every domain's triangles for one point: the domain's partial
// solid-angle sum (rpart[(s n_dom + j) np + ip]) and whether the point is within
// 2 h of one of these triangles (npart[s np + ip]).
__global__ void k_region(const DomDev *__restrict__ doms, int n_dom, const double *__restrict__ verts,
                         const int32_t *__restrict__ tris, const double *__restrict__ pts, int64_t np,
                         double *__restrict__ rpart, int32_t *__restrict__ npart)
{
    const int64_t ip = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ip >= np) return;
    const int sp = blockIdx.y, S = gridDim.y;
    const double x[3] = {pts[3 * ip], pts[3 * ip + 1], pts[3 * ip + 2]};
    bool near = false;
    for (int j = 0; j < n_dom; ++j) {
        double s = 0.0;
        const double h2 = 2.0 * doms[j].h;
        const long long t0 = doms[j].t_off + doms[j].nt * sp / S, t1 = doms[j].t_off + doms[j].nt * (sp + 1) / S;
        for (long long t = t0; t < t1; ++t) {
            double a[3], b[3], c[3];
            for (int d = 0; d < 3; ++d) {
                a[d] = verts[3 * int64_t(tris[3 * t]) + d] - x[d];
                b[d] = verts[3 * int64_t(tris[3 * t + 1]) + d] - x[d];
                c[d] = verts[3 * int64_t(tris[3 * t + 2]) + d] - x[d];
            }
            const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            const double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
            const double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            const double num = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                               a[2] * (b[0] * c[1] - b[1] * c[0]);
            const double den = la * lb * lc + (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) * lc +
                               (a[0] * c[0] + a[1] * c[1] + a[2] * c[2]) * lb + (b[0] * c[0] + b[1] * c[1] + b[2] * c[2]) * la;
            s += 2.0 * atan2(num, den);
            // within 2 h: every point of the triangle is within its longest
            // edge of each vertex, so the exact distance is needed only when
            // the nearest vertex is closer than 2 h + that edge
            if (!near) {
                const double e0 = (b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]);
                const double e1 = (c[0] - b[0]) * (c[0] - b[0]) + (c[1] - b[1]) * (c[1] - b[1]) + (c[2] - b[2]) * (c[2] - b[2]);
                const double e2 = (a[0] - c[0]) * (a[0] - c[0]) + (a[1] - c[1]) * (a[1] - c[1]) + (a[2] - c[2]) * (a[2] - c[2]);
                if (fmin(la, fmin(lb, lc)) < h2 + sqrt(fmax(e0, fmax(e1, e2))) && tri_dist2(a, b, c) < h2 * h2)
                    near = true;
            }
        }
        rpart[(int64_t(sp) * n_dom + j) * np + ip] = s;
    }
    npart[int64_t(sp) * np + ip] = near ? 1 : 0;
}

// region code of every point from the S partial sums (added in split order):
// the winding region (0 outside, j + 1 inside boundary j) and the reported
// code (-1 within 2 h of a boundary)
__global__ void k_region_reduce(const double *__restrict__ rpart, const int32_t *__restrict__ npart, int n_dom,
                                int S, int64_t np, int32_t *__restrict__ wreg, int32_t *__restrict__ region)
{
    const int64_t ip = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ip >= np) return;
    int reg = 0;
    bool near = false;
    for (int j = 0; j < n_dom; ++j) {
        double s = 0.0;
        for (int sp = 0; sp < S; ++sp) s += rpart[(int64_t(sp) * n_dom + j) * np + ip];
        if (rint(s / (4.0 * PI_D)) == 1.0) reg = j + 1;
    }
    for (int sp = 0; sp < S; ++sp) near = near || npart[int64_t(sp) * np + ip] != 0;
    wreg[ip] = reg;
    region[ip] = near ? -1 : reg;
}

// Split s of S of the source triangles of one point's winding region: the
// potentials of all fields over those triangles (fpart[(s F + f) np + ip]).
__global__ void k_field(const DomDev *__restrict__ doms, int n_dom, double k0re, double k0im, double rho0,
                        const double *__restrict__ verts, const int32_t *__restrict__ tris,
                        const double *__restrict__ area, const double *__restrict__ normal,
                        const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN,
                        const double2 *__restrict__ u, int64_t N, int n_fields, const double *__restrict__ pts,
                        int64_t np, const int32_t *__restrict__ wreg, double2 *__restrict__ fpart)
{
    const int64_t ip = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ip >= np) return;
    const int sp = blockIdx.y, S = gridDim.y;
    const double x[3] = {pts[3 * ip], pts[3 * ip + 1], pts[3 * ip + 2]};
    const int reg = wreg[ip];
    const int j0 = reg == 0 ? 0 : reg - 1, j1 = reg == 0 ? n_dom : reg;
    const double kre = reg == 0 ? k0re : doms[reg - 1].kre, kim = reg == 0 ? k0im : doms[reg - 1].kim;
    const double sN = reg == 0 ? -1.0 : doms[reg - 1].rho / rho0;   // coefficient of SL u_N
    const double sD = reg == 0 ? 1.0 : -1.0;                         // coefficient of DL u_D
    // the region's triangles are one contiguous range (domains are numbered in order)
    const long long T0 = doms[j0].t_off, T1 = doms[j1 - 1].t_off + doms[j1 - 1].nt;
    const long long t0 = T0 + (T1 - T0) * sp / S, t1 = T0 + (T1 - T0) * (sp + 1) / S;
    for (int f = 0; f < n_fields; ++f) {
        double pr = 0.0, pim = 0.0;
        const double2 *uf = u + int64_t(f) * N;
        for (long long t = t0; t < t1; ++t) {
            double P[3][3];
            double2 uD[3], uN[3];
            for (int c = 0; c < 3; ++c) {
                const int32_t g = tris[3 * t + c];
                for (int d = 0; d < 3; ++d) P[c][d] = verts[3 * int64_t(g) + d];
                uD[c] = uf[rowD[g]];
                uN[c] = uf[rowN[g]];
            }
            const double *n = normal + 3 * t;
            for (int q = 0; q < 6; ++q) {
                double y[3];
                for (int d = 0; d < 3; ++d)
                    y[d] = q6_bary[q][0] * P[0][d] + q6_bary[q][1] * P[1][d] + q6_bary[q][2] * P[2][d];
                const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                double sn, cs;
                sincos(kre * r, &sn, &cs);
                // one reciprocal for 1/(4 pi r) and 1/r^2; the damping only
                // for a complex wavenumber
                const double rinv = 1.0 / r;
                const double e = (kim != 0.0 ? exp(-kim * r) : 1.0) * (rinv * (0.25 / PI_D));
                const double gr = e * cs, gi = e * sn;
                const double a1 = 1.0 + kim * r, b1 = -kre * r, ir2 = rinv * rinv;
                const double dn = (dx * n[0] + dy * n[1] + dz * n[2]) * ir2;
                const double fr = (gr * a1 - gi * b1) * dn, fi = (gr * b1 + gi * a1) * dn;   // dG/dn_y
                double dr = 0, di = 0, nr = 0, ni = 0;
                for (int c = 0; c < 3; ++c) {
                    dr += q6_bary[q][c] * uD[c].x; di += q6_bary[q][c] * uD[c].y;
                    nr += q6_bary[q][c] * uN[c].x; ni += q6_bary[q][c] * uN[c].y;
                }
                const double w = area[t] * q6_w[q];
                pr += w * (sD * (fr * dr - fi * di) + sN * (gr * nr - gi * ni));
                pim += w * (sD * (fr * di + fi * dr) + sN * (gr * ni + gi * nr));
            }
        }
        fpart[(int64_t(sp) * n_fields + f) * np + ip] = make_double2(pr, pim);
    }
}

// field[f][ip] = incident (outside) + the S partial potentials in split order
__global__ void k_field_reduce(IncDev I, int has_inc, const double2 *__restrict__ fpart, int S, int n_fields,
                               const double *__restrict__ pts, int64_t np, const int32_t *__restrict__ wreg,
                               double2 *__restrict__ field)
{
    const int64_t ip = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ip >= np) return;
    const double x[3] = {pts[3 * ip], pts[3 * ip + 1], pts[3 * ip + 2]};
    for (int f = 0; f < n_fields; ++f) {
        double pr = 0.0, pim = 0.0;
        if (wreg[ip] == 0 && has_inc) {
            const double nz[3] = {0, 0, 1};
            double qr, qi;
            incident(I, f, x, nz, pr, pim, qr, qi);
        }
        for (int sp = 0; sp < S; ++sp) {
            const double2 v = fpart[(int64_t(sp) * n_fields + f) * np + ip];
            pr += v.x;
            pim += v.y;
        }
        field[int64_t(f) * np + ip] = make_double2(pr, pim);
    }
}

// Many fields: the representation formula is linear in u, so for a chunk of
// points the field of every field f is one row of a dense product,
//   field[f][p] = sum_n R[p][n] u_f[n] (+ p_inc,f(x_p) outside),
// R[p][rowD g] = sD sum_{(t,a) at g} sum_q |t| w_q lambda_a(q) dG/dn_y(x_p, y_q),
// R[p][rowN g] = sN sum_{(t,a) at g} sum_q |t| w_q lambda_a(q) G(x_p, y_q),
// with the wavenumber and signs of the point's winding region (zero for the
// vertices of other domains when the point is inside a domain).  The kernel
// values are then evaluated once per (point, source point) instead of once per
// field.  One thread per (point, vertex).
__global__ void k_field_rows(const DomDev *__restrict__ doms, int n_dom, double k0re, double k0im, double rho0,
                             const double *__restrict__ verts, const int32_t *__restrict__ tris,
                             const double *__restrict__ area, const double *__restrict__ normal,
                             const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                             const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN, int64_t NV, int64_t N,
                             const double *__restrict__ pts, const int32_t *__restrict__ wreg, int64_t p0, int64_t npc,
                             double2 *__restrict__ R)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= npc * NV) return;
    const int64_t pl = idx / NV, g = idx - pl * NV, ip = p0 + pl;
    const int reg = wreg[ip];
    int dom = 0;
    for (int j = 0; j < n_dom; ++j)
        if (g >= doms[j].v_off && g < doms[j].v_off + doms[j].nv) dom = j;
    double2 *row = R + pl * N;
    if (reg != 0 && dom != reg - 1) {
        row[rowD[g]] = make_double2(0.0, 0.0);
        row[rowN[g]] = make_double2(0.0, 0.0);
        return;
    }
    const double kre = reg == 0 ? k0re : doms[reg - 1].kre, kim = reg == 0 ? k0im : doms[reg - 1].kim;
    const double sN = reg == 0 ? -1.0 : doms[reg - 1].rho / rho0;
    const double sD = reg == 0 ? 1.0 : -1.0;
    const double x[3] = {pts[3 * ip], pts[3 * ip + 1], pts[3 * ip + 2]};
    double dr = 0, di = 0, nr = 0, ni = 0;
    for (int32_t k = v2t_ptr[g]; k < v2t_ptr[g + 1]; ++k) {
        const int64_t t = v2t[k] / 3;
        const int a = v2t[k] - 3 * int(t);
        double P[3][3];
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) P[c][d] = verts[3 * int64_t(tris[3 * t + c]) + d];
        const double *n = normal + 3 * t;
        for (int q = 0; q < 6; ++q) {
            double y[3];
            for (int d = 0; d < 3; ++d) y[d] = q6_bary[q][0] * P[0][d] + q6_bary[q][1] * P[1][d] + q6_bary[q][2] * P[2][d];
            const double ex = x[0] - y[0], ey = x[1] - y[1], ez = x[2] - y[2];
            const double r = sqrt(ex * ex + ey * ey + ez * ez);
            double sn, cs;
            sincos(kre * r, &sn, &cs);
            const double rinv = 1.0 / r;
            const double e = (kim != 0.0 ? exp(-kim * r) : 1.0) * (rinv * (0.25 / PI_D));
            const double gr = e * cs, gi = e * sn;
            const double a1 = 1.0 + kim * r, b1 = -kre * r, ir2 = rinv * rinv;
            const double dn = (ex * n[0] + ey * n[1] + ez * n[2]) * ir2;
            const double fr = (gr * a1 - gi * b1) * dn, fi = (gr * b1 + gi * a1) * dn;   // dG/dn_y
            const double w = area[t] * q6_w[q] * q6_bary[q][a];
            dr += w * fr; di += w * fi;
            nr += w * gr; ni += w * gi;
        }
    }
    row[rowD[g]] = make_double2(sD * dr, sD * di);
    row[rowN[g]] = make_double2(sN * nr, sN * ni);
}

// field[f][p0 + pl] = sum_n u_f[n] R[pl][n] (+ incident outside): tiles of 16
// fields x 16 points, K chunks of 32 through LDS, FP64 complex
constexpr int FG_T = 16, FG_K = 32;
__global__ __launch_bounds__(256) void k_field_gemm(const double2 *__restrict__ U, int64_t N, int n_fields,
                                                    const double2 *__restrict__ R, int64_t p0, int64_t npc, int64_t np,
                                                    const double *__restrict__ pts, const int32_t *__restrict__ wreg,
                                                    IncDev I, int has_inc, double2 *__restrict__ field)
{
    __shared__ double2 sU[FG_T][FG_K + 1], sR[FG_T][FG_K + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t f0 = int64_t(blockIdx.y) * FG_T, l0 = int64_t(blockIdx.x) * FG_T;
    double ar = 0, ai = 0;
    for (int64_t k0 = 0; k0 < N; k0 += FG_K) {
        for (int e = threadIdx.x; e < FG_T * FG_K; e += 256) {
            const int r = e / FG_K, c = e - r * FG_K;
            const int64_t n = k0 + c, f = f0 + r, l = l0 + r;
            sU[r][c] = (f < n_fields && n < N) ? U[f * N + n] : make_double2(0.0, 0.0);
            sR[r][c] = (l < npc && n < N) ? R[l * N + n] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < FG_K; ++c) {
            const double2 u = sU[ty][c], w = sR[tx][c];
            ar += u.x * w.x - u.y * w.y;
            ai += u.x * w.y + u.y * w.x;
        }
        __syncthreads();
    }
    const int64_t f = f0 + ty, l = l0 + tx;
    if (f >= n_fields || l >= npc) return;
    const int64_t ip = p0 + l;
    if (has_inc && wreg[ip] == 0) {
        const double x[3] = {pts[3 * ip], pts[3 * ip + 1], pts[3 * ip + 2]}, nz[3] = {0, 0, 1};
        double pr, pim, qr, qi;
        incident(I, int(f), x, nz, pr, pim, qr, qi);
        ar += pr;
        ai += pim;
    }
    field[f * np + ip] = make_double2(ar, ai);
}

void launch_field(bem_problem &p, const double2 *u, const bem_incident *inc, int n_fields, const double *pts,
                  int64_t np, double2 *field, int32_t *region)
{
    double *d_params = nullptr;
    DevScratch params_mem, doms_mem, wreg_mem, rows_mem;
    IncDev I{};
    if (inc) I = upload_incident(p, *inc, &d_params);
    params_mem.p = d_params;
    std::vector<DomDev> hd;
    for (const auto &d : p.doms) {
        // mean edge length (every edge counted from both of its triangles)
        double sum = 0.0;
        for (int64_t t = d.t_off; t < d.t_off + d.nt; ++t)
            for (int e = 0; e < 3; ++e) {
                const double *P = &p.h_verts[3 * size_t(p.h_tris[3 * t + e])];
                const double *Q = &p.h_verts[3 * size_t(p.h_tris[3 * t + (e + 1) % 3])];
                sum += std::sqrt((P[0] - Q[0]) * (P[0] - Q[0]) + (P[1] - Q[1]) * (P[1] - Q[1]) +
                                 (P[2] - Q[2]) * (P[2] - Q[2]));
            }
        hd.push_back(DomDev{d.v_off, d.t_off, d.nt, d.nv, d.kre, d.kim, d.rho, sum / double(3 * d.nt)});
    }
    DomDev *d_doms = nullptr;
    dmalloc(reinterpret_cast<void **>(&d_doms), hd.size() * sizeof(DomDev));
    doms_mem.p = d_doms;
    BEM_HIP(hipMemcpyAsync(d_doms, hd.data(), hd.size() * sizeof(DomDev), hipMemcpyHostToDevice, p.stream));
    const int B = 128;
    int32_t *wreg = nullptr;
    double2 *R = nullptr;
    if (np > 0) {
        // every point's sums over the source triangles split S ways, so that a
        // few ten thousand points still give about eight waves per SIMD; the
        // partials (at most FIELD_ROWS_BYTES) are added in split order
        const int n_dom = int(hd.size());
        const int64_t per_split = 16 * std::max<int64_t>(n_fields <= FIELD_DIRECT_MAX ? n_fields : 0, 1) * np +
                                  (8 * int64_t(n_dom) + 4) * np;
        int S = int(std::clamp<int64_t>((FIELD_TARGET_THREADS + np - 1) / np, 1, FIELD_MAX_SPLIT));
        while (S > 1 && S * per_split > FIELD_ROWS_BYTES) S /= 2;
        DevScratch rpart_mem, npart_mem, fpart_mem;
        double *rpart = nullptr;
        int32_t *npart = nullptr;
        dmalloc(reinterpret_cast<void **>(&wreg), size_t(np) * sizeof(int32_t));
        wreg_mem.p = wreg;
        dmalloc(reinterpret_cast<void **>(&rpart), size_t(S) * n_dom * np * sizeof(double));
        rpart_mem.p = rpart;
        dmalloc(reinterpret_cast<void **>(&npart), size_t(S) * np * sizeof(int32_t));
        npart_mem.p = npart;
        k_region<<<dim3(blocks_1d(np, B), unsigned(S)), dim3(B), 0, p.stream>>>(d_doms, n_dom, p.d_verts, p.d_tris,
                                                                                pts, np, rpart, npart);
        BEM_HIP(hipGetLastError());
        k_region_reduce<<<dim3(blocks_1d(np, 256)), dim3(256), 0, p.stream>>>(rpart, npart, n_dom, S, np, wreg, region);
        BEM_HIP(hipGetLastError());
        if (n_fields <= FIELD_DIRECT_MAX) {
            double2 *fpart = nullptr;
            dmalloc(reinterpret_cast<void **>(&fpart), size_t(S) * n_fields * np * sizeof(double2));
            fpart_mem.p = fpart;
            k_field<<<dim3(blocks_1d(np, B), unsigned(S)), dim3(B), 0, p.stream>>>(
                d_doms, n_dom, p.k0re, p.k0im, p.rho0, p.d_verts, p.d_tris, p.d_area, p.d_normal, p.d_rowD,
                p.d_rowN, u, p.N, n_fields, pts, np, wreg, fpart);
            BEM_HIP(hipGetLastError());
            k_field_reduce<<<dim3(blocks_1d(np, 256)), dim3(256), 0, p.stream>>>(I, inc ? 1 : 0, fpart, S, n_fields,
                                                                                 pts, np, wreg, field);
            BEM_HIP(hipGetLastError());
        } else {
            // points in chunks whose rows take at most FIELD_ROWS_BYTES
            // (BEM_FIELD_CHUNK_POINTS sets a smaller chunk, for tests of the chunk loop)
            int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(np, FIELD_ROWS_BYTES / (16 * p.N)));
            if (const char *e = std::getenv("BEM_FIELD_CHUNK_POINTS")) {
                const long long c = std::atoll(e);
                if (c > 0) chunk = std::min<int64_t>(chunk, c);
            }
            dmalloc(reinterpret_cast<void **>(&R), size_t(chunk) * p.N * sizeof(double2));
            rows_mem.p = R;
            for (int64_t p0 = 0; p0 < np; p0 += chunk) {
                const int64_t npc = std::min(chunk, np - p0);
                k_field_rows<<<dim3(blocks_1d(npc * p.NV, 256)), dim3(256), 0, p.stream>>>(
                    d_doms, int(hd.size()), p.k0re, p.k0im, p.rho0, p.d_verts, p.d_tris, p.d_area, p.d_normal,
                    p.d_v2t_ptr, p.d_v2t, p.d_rowD, p.d_rowN, p.NV, p.N, pts, wreg, p0, npc, R);
                BEM_HIP(hipGetLastError());
                const dim3 grid(unsigned((npc + FG_T - 1) / FG_T), unsigned((n_fields + FG_T - 1) / FG_T));
                k_field_gemm<<<grid, dim3(256), 0, p.stream>>>(u, p.N, n_fields, R, p0, npc, np, pts, wreg, I,
                                                               inc ? 1 : 0, field);
                BEM_HIP(hipGetLastError());
            }
        }
    }
    BEM_HIP(hipStreamSynchronize(p.stream));
}

}  // namespace bem
