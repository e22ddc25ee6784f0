/*
 * FP64 CPU oracle: Galerkin P1 boundary operators of the Helmholtz equation
 * (single layer V, double layer K, adjoint double layer K', hypersingular W)
 * on closed triangular surfaces, layer potentials and the solid-angle
 * winding number.
 *
 * TEST INFRASTRUCTURE.  This file is the independent reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the GPU library never includes,
 * links or calls it, and it shares no code, header or table with it.
 *
 * Definitions followed (paper, Appendix A "Calderon operator"):
 *   G_k(x,y) = exp(i k r) / (4 pi r), r = |x - y|          (Green's function)
 *   V psi(x)  = int G psi(y)                                 (single layer)
 *   K phi(x)  = int dG/dn(y) phi(y)                          (double layer)
 *   K' psi(x) = d/dn(x) int G psi(y)                         (adjoint double layer)
 *   W phi(x)  = - d/dn(x) int dG/dn(y) phi(y)                (hypersingular)
 * with the normal pointing out of the bounded domain (model section, traces).
 * With d = x - y and F = G (1 - i k r) / r^2:
 *   dG/dn(y) =  F (d . n_y),   dG/dn(x) = -F (d . n_x).
 * W is used in its integrated-by-parts (Maue) weak form
 *   <W phi, eta> = int int G [curl phi(y) . curl eta(x) - k^2 (n_x . n_y) phi(y) eta(x)],
 * whose sign agrees with the jump relation gamma_N DL = -W.
 *
 * Galerkin discretisation (paper, "Operator preconditioning" section): test and
 * trial spaces are continuous piecewise-linear functions on the triangles.
 * Quadrature (the paper defers to its library and does not state it): a
 * 6-point degree-4 symmetric rule on each triangle for pairs of triangles that
 * share no vertex, and the Sauter-Schwab regularising transformations with
 * n-point Gauss-Legendre factors for coincident, edge-adjacent and
 * vertex-adjacent pairs (Sauter & Schwab, Boundary Element Methods, 5.2).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ---------------------------------------------------------------------- */
/* Quadrature rules                                                         */
/* ---------------------------------------------------------------------- */

/* 6-point degree-4 symmetric rule on the reference triangle
 * {xi1, xi2 >= 0, xi1 + xi2 <= 1}; the returned weights sum to 1 so that
 * int_T f ~ |T| sum_q w_q f(x_q).  Two orbits of barycentric points
 * (a, a, 1-2a) with weight wa (Strang & Fix; Dunavant 1985). */
int orc_far_rule(double *xi1, double *xi2, double *w)
{
    const double a[2] = {0.44594849091596488632, 0.091576213509770743460};
    const double wa[2] = {0.22338158967801146570, 0.10995174365532186764};
    int q = 0;
    for (int o = 0; o < 2; ++o) {
        const double l[3][3] = {{a[o], a[o], 1.0 - 2.0 * a[o]},
                                {a[o], 1.0 - 2.0 * a[o], a[o]},
                                {1.0 - 2.0 * a[o], a[o], a[o]}};
        for (int p = 0; p < 3; ++p) {
            /* barycentric (l0, l1, l2) -> parameters (xi1, xi2) = (l1, l2) */
            xi1[q] = l[p][1];
            xi2[q] = l[p][2];
            w[q] = wa[o];
            ++q;
        }
    }
    return q;
}

/* Legendre polynomial P_n and its derivative at z (three-term recurrence). */
static void legendre(int n, double z, double *p, double *dp)
{
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = n * (z * p1 - p0) / (z * z - 1.0);
}

/* Gauss-Legendre nodes (increasing) and weights on [0,1]: Newton iteration
 * for the roots z of P_n on [-1,1], mapped by x = (1 - z)/2; the weight
 * 2/((1 - z^2) P_n'(z)^2) is halved for the unit interval. */
int orc_gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, &p, &dp);
            const double dz = p / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(n, z, &p, &dp);
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return n;
}

/* Pair classes. */
enum { ORC_FAR = 0, ORC_VERTEX = 1, ORC_EDGE = 2, ORC_COINCIDENT = 3 };

/* Number of points of the Sauter-Schwab rule of a class at order n. */
int orc_ss_rule_size(int cls, int n)
{
    int n4 = n * n * n * n;
    switch (cls) {
    case ORC_COINCIDENT: return 6 * n4;
    case ORC_EDGE: return 5 * n4;
    case ORC_VERTEX: return 2 * n4;
    default: return 0;
    }
}

/* Sauter-Schwab rule on the product of two reference triangles
 * T = {(s1, s2): 0 <= s2 <= s1 <= 1} (each of area 1/2).  The singular set is
 * x = y (coincident), the common edge s2 = 0 (edge) or the common corner 0
 * (vertex).  The 4-cube [0,1]^4 with coordinates (xi, e1, e2, e3) is mapped
 * onto the pieces of T x T; each map's Jacobian carries enough powers of xi
 * and e1 to cancel the 1/r singularity.  Output: points (xh[2], yh[2]) in T
 * and weights w (sum 1/4 = |T|^2). */
int orc_ss_rule(int cls, int n, double *xh, double *yh, double *w)
{
    double g[64], gw[64];
    if (n < 1 || n > 64) return -1;
    orc_gauss_legendre01(n, g, gw);
    int m = 0;
    for (int i0 = 0; i0 < n; ++i0)
    for (int i1 = 0; i1 < n; ++i1)
    for (int i2 = 0; i2 < n; ++i2)
    for (int i3 = 0; i3 < n; ++i3) {
        const double xi = g[i0], e1 = g[i1], e2 = g[i2], e3 = g[i3];
        const double ww = gw[i0] * gw[i1] * gw[i2] * gw[i3];
        if (cls == ORC_COINCIDENT) {
            const double J = xi * xi * xi * e1 * e1 * e2;
            const double p[6][4] = {
                {xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1)},
                {xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2)},
                {xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2)},
                {xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3)},
                {xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2)},
                {xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)}};
            for (int k = 0; k < 6; ++k) {
                xh[2 * m] = p[k][0]; xh[2 * m + 1] = p[k][1];
                yh[2 * m] = p[k][2]; yh[2 * m + 1] = p[k][3];
                w[m] = ww * J;
                ++m;
            }
        } else if (cls == ORC_EDGE) {
            const double p[5][4] = {
                {xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2)},
                {xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)},
                {xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3},
                {xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1},
                {xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2}};
            const double J0 = xi * xi * xi * e1 * e1;
            for (int k = 0; k < 5; ++k) {
                xh[2 * m] = p[k][0]; xh[2 * m + 1] = p[k][1];
                yh[2 * m] = p[k][2]; yh[2 * m + 1] = p[k][3];
                w[m] = ww * (k == 0 ? J0 : J0 * e2);
                ++m;
            }
        } else if (cls == ORC_VERTEX) {
            const double J = xi * xi * xi * e2;
            xh[2 * m] = xi;          xh[2 * m + 1] = xi * e1;
            yh[2 * m] = xi * e2;     yh[2 * m + 1] = xi * e2 * e3;
            w[m] = ww * J; ++m;
            xh[2 * m] = xi * e2;     xh[2 * m + 1] = xi * e2 * e3;
            yh[2 * m] = xi;          yh[2 * m + 1] = xi * e1;
            w[m] = ww * J; ++m;
        } else {
            return -1;
        }
    }
    return m;
}

/* ---------------------------------------------------------------------- */
/* Geometry                                                                 */
/* ---------------------------------------------------------------------- */

static void sub3(const double *a, const double *b, double *c) { c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

typedef struct {
    int nv, nt;
    const double *v;   /* [nv][3] */
    const int *t;      /* [nt][3] */
    double *area;      /* [nt] */
    double *normal;    /* [nt][3]   unit normal (P1-P0) x (P2-P0) / (2|T|) */
    double *curl;      /* [nt][3][3] surface curl of lambda_a: -e_a / (2|T|),  e_a = P_{a+2} - P_{a+1} */
} mesh_t;

static int mesh_init(mesh_t *m, const double *v, int nv, const int *t, int nt)
{
    m->nv = nv; m->nt = nt; m->v = v; m->t = t;
    m->area = malloc(sizeof(double) * (size_t)nt);
    m->normal = malloc(sizeof(double) * 3 * (size_t)nt);
    m->curl = malloc(sizeof(double) * 9 * (size_t)nt);
    if (!m->area || !m->normal || !m->curl) return -1;
    for (int i = 0; i < nt; ++i) {
        const double *P[3] = {v + 3 * t[3 * i], v + 3 * t[3 * i + 1], v + 3 * t[3 * i + 2]};
        double e1[3], e2[3], c[3];
        sub3(P[1], P[0], e1);
        sub3(P[2], P[0], e2);
        cross3(e1, e2, c);
        double twice = sqrt(dot3(c, c));
        m->area[i] = 0.5 * twice;
        for (int d = 0; d < 3; ++d) m->normal[3 * i + d] = c[d] / twice;
        for (int a = 0; a < 3; ++a) {
            double e[3];
            sub3(P[(a + 2) % 3], P[(a + 1) % 3], e);
            for (int d = 0; d < 3; ++d) m->curl[9 * i + 3 * a + d] = -e[d] / twice;
        }
    }
    return 0;
}

static void mesh_free(mesh_t *m)
{
    free(m->area); free(m->normal); free(m->curl);
}

/* Classify a pair of triangles of the same mesh by shared vertex indices and
 * return the local vertex orders that put the shared vertices first (in the
 * same order in both triangles). */
static int classify(const int *tt, const int *ts, int *pt, int *ps)
{
    int ia[3], ja[3], ns = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (tt[a] == ts[b]) { ia[ns] = a; ja[ns] = b; ++ns; }
    if (ns == 0) return ORC_FAR;
    if (ns == 3) {
        /* same triangle: identical parametrisation; ps[a] is the local index
         * in s of the test vertex tt[a] */
        for (int a = 0; a < 3; ++a) {
            pt[a] = a;
            for (int b = 0; b < 3; ++b)
                if (ts[b] == tt[a]) ps[a] = b;
        }
        return ORC_COINCIDENT;
    }
    if (ns == 2) {
        pt[0] = ia[0]; pt[1] = ia[1]; pt[2] = 3 - ia[0] - ia[1];
        ps[0] = ja[0]; ps[1] = ja[1]; ps[2] = 3 - ja[0] - ja[1];
        return ORC_EDGE;
    }
    pt[0] = ia[0]; pt[1] = (ia[0] + 1) % 3; pt[2] = (ia[0] + 2) % 3;
    ps[0] = ja[0]; ps[1] = (ja[0] + 1) % 3; ps[2] = (ja[0] + 2) % 3;
    return ORC_VERTEX;
}

/* ---------------------------------------------------------------------- */
/* Element integrals                                                        */
/* ---------------------------------------------------------------------- */

/* Accumulate the integrand of the four operators at one pair of points.
 * lx, ly: P1 basis values of the test/trial triangle (original local order);
 * wgt: full quadrature weight including the area elements. */
static void add_pair(const double *x, const double *y, const double *lx, const double *ly, double wgt,
                     const double *nt, const double *ns, const double *ct, const double *cs,
                     cplx kappa, cplx E[4][3][3])
{
    double d[3];
    sub3(x, y, d);
    const double r = sqrt(dot3(d, d));
    const cplx G = cexp(I * kappa * r) / (4.0 * M_PI * r);
    const cplx F = G * (1.0 - I * kappa * r) / (r * r);
    const double dny = dot3(d, ns);
    const double dnx = dot3(d, nt);
    const double nn = dot3(nt, ns);
    const cplx k2 = kappa * kappa;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double ll = lx[a] * ly[b] * wgt;
            E[0][a][b] += ll * G;
            E[1][a][b] += ll * F * dny;
            E[2][a][b] += -ll * F * dnx;
            E[3][a][b] += wgt * G * dot3(ct + 3 * a, cs + 3 * b) - ll * k2 * nn * G;
        }
}

typedef struct {
    int n;
    int size[4];
    double *xh[4], *yh[4], *w[4];
} ss_rules_t;

static int ss_rules_init(ss_rules_t *R, int n)
{
    R->n = n;
    for (int c = 1; c <= 3; ++c) {
        int s = orc_ss_rule_size(c, n);
        R->size[c] = s;
        R->xh[c] = malloc(sizeof(double) * 2 * (size_t)s);
        R->yh[c] = malloc(sizeof(double) * 2 * (size_t)s);
        R->w[c] = malloc(sizeof(double) * (size_t)s);
        if (!R->xh[c] || !R->yh[c] || !R->w[c]) return -1;
        orc_ss_rule(c, n, R->xh[c], R->yh[c], R->w[c]);
    }
    return 0;
}

static void ss_rules_free(ss_rules_t *R)
{
    for (int c = 1; c <= 3; ++c) { free(R->xh[c]); free(R->yh[c]); free(R->w[c]); }
}

/* Element matrices E[op][a][b] (op = V, K, K', W) for test triangle it of mesh
 * mt and trial triangle is of mesh ms.  cls selects the rule. */
static void element(const mesh_t *mt, int it, const mesh_t *ms, int is, int cls, const int *pt, const int *ps,
                    cplx kappa, const ss_rules_t *R, cplx E[4][3][3])
{
    memset(E, 0, sizeof(cplx) * 36);
    const double *nt = mt->normal + 3 * it, *ns = ms->normal + 3 * is;
    const double *ct = mt->curl + 9 * it, *cs = ms->curl + 9 * is;
    const double *Pt[3], *Ps[3];
    for (int a = 0; a < 3; ++a) {
        Pt[a] = mt->v + 3 * mt->t[3 * it + a];
        Ps[a] = ms->v + 3 * ms->t[3 * is + a];
    }
    if (cls == ORC_FAR) {
        double xi1[6], xi2[6], wq[6];
        orc_far_rule(xi1, xi2, wq);
        for (int q = 0; q < 6; ++q) {
            const double lx[3] = {1.0 - xi1[q] - xi2[q], xi1[q], xi2[q]};
            double x[3];
            for (int d = 0; d < 3; ++d) x[d] = lx[0] * Pt[0][d] + lx[1] * Pt[1][d] + lx[2] * Pt[2][d];
            for (int p = 0; p < 6; ++p) {
                const double ly[3] = {1.0 - xi1[p] - xi2[p], xi1[p], xi2[p]};
                double y[3];
                for (int d = 0; d < 3; ++d) y[d] = ly[0] * Ps[0][d] + ly[1] * Ps[1][d] + ly[2] * Ps[2][d];
                const double wgt = mt->area[it] * wq[q] * ms->area[is] * wq[p];
                add_pair(x, y, lx, ly, wgt, nt, ns, ct, cs, kappa, E);
            }
        }
        return;
    }
    /* Sauter-Schwab: reparametrise both triangles as
     * chi(s) = Q0 + s1 (Q1 - Q0) + s2 (Q2 - Q1), Q_i = P_{perm[i]}, so that the
     * shared vertices come first; its barycentric coordinates are
     * (1 - s1, s1 - s2, s2) and its Jacobian is 2|T|. */
    const double jac = (2.0 * mt->area[it]) * (2.0 * ms->area[is]);
    const double *xh = R->xh[cls], *yh = R->yh[cls], *w = R->w[cls];
    for (int m = 0; m < R->size[cls]; ++m) {
        const double bx[3] = {1.0 - xh[2 * m], xh[2 * m] - xh[2 * m + 1], xh[2 * m + 1]};
        const double by[3] = {1.0 - yh[2 * m], yh[2 * m] - yh[2 * m + 1], yh[2 * m + 1]};
        double lx[3], ly[3], x[3] = {0, 0, 0}, y[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i) {
            lx[pt[i]] = bx[i];
            ly[ps[i]] = by[i];
            for (int d = 0; d < 3; ++d) {
                x[d] += bx[i] * Pt[pt[i]][d];
                y[d] += by[i] * Ps[ps[i]][d];
            }
        }
        add_pair(x, y, lx, ly, w[m] * jac, nt, ns, ct, cs, kappa, E);
    }
}

/* Element matrices of one pair, for tests: E[4][3][3] complex (interleaved
 * re/im doubles).  Triangles given by coordinates; the class and local orders
 * are found from the integer vertex labels lt, ls (equal labels = shared
 * vertex).  force_far != 0 evaluates the 6-point rule regardless. */
int orc_element_pair(const double *Pt9, const int *lt, const double *Ps9, const int *ls,
                     double kre, double kim, int ss_n, int force_far, double *out)
{
    double v[18];
    memcpy(v, Pt9, sizeof(double) * 9);
    memcpy(v + 9, Ps9, sizeof(double) * 9);
    int tri[6] = {0, 1, 2, 3, 4, 5};
    mesh_t m;
    if (mesh_init(&m, v, 6, tri, 2)) return -1;
    int pt[3], ps[3];
    int cls = force_far ? ORC_FAR : classify(lt, ls, pt, ps);
    ss_rules_t R;
    if (ss_rules_init(&R, ss_n)) { mesh_free(&m); return -1; }
    cplx E[4][3][3];
    element(&m, 0, &m, 1, cls, pt, ps, kre + I * kim, &R, E);
    memcpy(out, E, sizeof(E));
    ss_rules_free(&R);
    mesh_free(&m);
    return cls;
}

/* ---------------------------------------------------------------------- */
/* Operator rows                                                            */
/* ---------------------------------------------------------------------- */

/* Rows of the Galerkin matrices of V, K, K', W for test functions at the
 * given vertices of the test mesh and every trial function of the trial
 * mesh.  Each output is [n_rows][nv_trial] complex (interleaved doubles),
 * zeroed here.  same_mesh != 0 declares that test and trial meshes are the
 * same surface, which enables the singular rules for touching pairs.
 * Returns 0, or -1 on allocation failure. */
int orc_operator_rows(const double *vt, int nvt, const int *tt, int ntt,
                      const double *vs, int nvs, const int *ts, int nts,
                      int same_mesh, double kre, double kim, int ss_n,
                      const long long *rows, int n_rows,
                      double *Vout, double *Kout, double *Kpout, double *Wout)
{
    mesh_t mt, ms;
    if (mesh_init(&mt, vt, nvt, tt, ntt) || mesh_init(&ms, vs, nvs, ts, nts)) return -1;
    ss_rules_t R;
    if (ss_rules_init(&R, ss_n)) return -1;
    /* vertex -> incident (triangle, corner) lists of the test mesh */
    int *cnt = calloc((size_t)nvt + 1, sizeof(int));
    int *lst = malloc(sizeof(int) * 3 * (size_t)ntt);
    int *fill = calloc((size_t)nvt, sizeof(int));
    for (int i = 0; i < 3 * ntt; ++i) cnt[tt[i] + 1]++;
    for (int i = 0; i < nvt; ++i) cnt[i + 1] += cnt[i];
    for (int i = 0; i < ntt; ++i)
        for (int a = 0; a < 3; ++a) {
            int r = tt[3 * i + a];
            lst[cnt[r] + fill[r]++] = 3 * i + a;
        }
    const cplx kappa = kre + I * kim;
    const size_t nvs_ = (size_t)nvs;
    cplx *V = (cplx *)Vout, *K = (cplx *)Kout, *Kp = (cplx *)Kpout, *W = (cplx *)Wout;
    memset(V, 0, sizeof(cplx) * nvs_ * n_rows);
    memset(K, 0, sizeof(cplx) * nvs_ * n_rows);
    memset(Kp, 0, sizeof(cplx) * nvs_ * n_rows);
    memset(W, 0, sizeof(cplx) * nvs_ * n_rows);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_rows; ++i) {
        const int r = (int)rows[i];
        for (int k = cnt[r]; k < cnt[r + 1]; ++k) {
            const int it = lst[k] / 3, a = lst[k] % 3;
            for (int is = 0; is < nts; ++is) {
                int pt[3], ps[3];
                int cls = same_mesh ? classify(tt + 3 * it, ts + 3 * is, pt, ps) : ORC_FAR;
                cplx E[4][3][3];
                element(&mt, it, &ms, is, cls, pt, ps, kappa, &R, E);
                for (int b = 0; b < 3; ++b) {
                    const size_t c = (size_t)i * nvs_ + ts[3 * is + b];
                    V[c] += E[0][a][b];
                    K[c] += E[1][a][b];
                    Kp[c] += E[2][a][b];
                    W[c] += E[3][a][b];
                }
            }
        }
    }
    free(cnt); free(lst); free(fill);
    ss_rules_free(&R);
    mesh_free(&mt); mesh_free(&ms);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Layer potentials and winding number                                      */
/* ---------------------------------------------------------------------- */

/* Single-layer potential of psi and double-layer potential of phi (P1
 * coefficients on the mesh vertices) at points off the surface, with the
 * 6-point rule on every source triangle (paper, Appendix A, SL and DL). */
int orc_potentials(const double *v, int nv, const int *t, int nt, double kre, double kim,
                   const double *phi_in, const double *psi_in, const double *pts, int np,
                   double *sl_out, double *dl_out)
{
    mesh_t m;
    if (mesh_init(&m, v, nv, t, nt)) return -1;
    const cplx *phi = (const cplx *)phi_in, *psi = (const cplx *)psi_in;
    cplx *SL = (cplx *)sl_out, *DL = (cplx *)dl_out;
    const cplx kappa = kre + I * kim;
    double xi1[6], xi2[6], wq[6];
    orc_far_rule(xi1, xi2, wq);
#pragma omp parallel for schedule(static)
    for (int p = 0; p < np; ++p) {
        const double *x = pts + 3 * p;
        cplx sl = 0, dl = 0;
        for (int is = 0; is < nt; ++is) {
            const double *P[3] = {v + 3 * t[3 * is], v + 3 * t[3 * is + 1], v + 3 * t[3 * is + 2]};
            for (int q = 0; q < 6; ++q) {
                const double l[3] = {1.0 - xi1[q] - xi2[q], xi1[q], xi2[q]};
                double y[3], d[3];
                for (int k = 0; k < 3; ++k) y[k] = l[0] * P[0][k] + l[1] * P[1][k] + l[2] * P[2][k];
                sub3(x, y, d);
                const double r = sqrt(dot3(d, d));
                const cplx G = cexp(I * kappa * r) / (4.0 * M_PI * r);
                const cplx F = G * (1.0 - I * kappa * r) / (r * r);
                const double wgt = m.area[is] * wq[q];
                cplx ps = 0, ph = 0;
                for (int a = 0; a < 3; ++a) {
                    ps += l[a] * psi[t[3 * is + a]];
                    ph += l[a] * phi[t[3 * is + a]];
                }
                sl += wgt * G * ps;
                dl += wgt * F * dot3(d, m.normal + 3 * is) * ph;
            }
        }
        SL[p] = sl;
        DL[p] = dl;
    }
    mesh_free(&m);
    return 0;
}

/* Winding number of a closed oriented surface about each point: the sum of
 * the signed solid angles of its triangles over 4 pi (Van Oosterom &
 * Strackee).  1 inside, 0 outside for outward-oriented surfaces. */
int orc_winding(const double *v, int nv, const int *t, int nt, const double *pts, int np, double *out)
{
    (void)nv;
#pragma omp parallel for schedule(static)
    for (int p = 0; p < np; ++p) {
        const double *x = pts + 3 * p;
        double s = 0.0;
        for (int i = 0; i < nt; ++i) {
            double a[3], b[3], c[3], bc[3];
            sub3(v + 3 * t[3 * i], x, a);
            sub3(v + 3 * t[3 * i + 1], x, b);
            sub3(v + 3 * t[3 * i + 2], x, c);
            const double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b)), lc = sqrt(dot3(c, c));
            cross3(b, c, bc);
            const double num = dot3(a, bc);
            const double den = la * lb * lc + dot3(a, b) * lc + dot3(a, c) * lb + dot3(b, c) * la;
            s += 2.0 * atan2(num, den);
        }
        out[p] = s / (4.0 * M_PI);
    }
    return 0;
}
