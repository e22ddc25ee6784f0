// Host-side mesh checks and topology: validation of closed oriented surfaces,
// touching triangle pairs (coincident / edge / vertex) and the sparsity pattern
// of the FP64 singular correction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "bem_internal.h"

namespace bem {

static Error mesh_error(int dom, const std::string &what)
{
    return Error{BEM_ERR_MESH, "domain " + std::to_string(dom) + ": " + what};
}

void validate_mesh(const double *v, int64_t nv, const int32_t *t, int64_t nt, int dom)
{
    if (nv < 4 || nt < 4) throw mesh_error(dom, "a closed surface needs at least 4 vertices and 4 triangles");
    if (nt > (int64_t(1) << 28) || nv > (int64_t(1) << 28)) throw mesh_error(dom, "mesh too large");
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(v[i])) throw Error{BEM_ERR_INVALID_ARG, "domain " + std::to_string(dom) + ": non-finite vertex coordinate"};
    // indices in range, no repeated vertex, positive area
    double scale = 0.0;
    for (int64_t i = 0; i < 3 * nv; ++i) scale = std::max(scale, std::fabs(v[i]));
    for (int64_t i = 0; i < nt; ++i) {
        const int32_t a = t[3 * i], b = t[3 * i + 1], c = t[3 * i + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            throw mesh_error(dom, "triangle " + std::to_string(i) + " has a vertex index out of range");
        if (a == b || b == c || a == c) throw mesh_error(dom, "triangle " + std::to_string(i) + " repeats a vertex");
        double e1[3], e2[3], cr[3];
        for (int d = 0; d < 3; ++d) { e1[d] = v[3 * b + d] - v[3 * a + d]; e2[d] = v[3 * c + d] - v[3 * a + d]; }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double ar = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(ar > 1e-14 * (scale * scale + 1e-300))) throw mesh_error(dom, "triangle " + std::to_string(i) + " has zero area");
    }
    // every directed edge once, and its reverse once (closed, consistently oriented, manifold)
    std::unordered_map<uint64_t, int> edges;
    edges.reserve(size_t(3 * nt * 2));
    for (int64_t i = 0; i < nt; ++i)
        for (int k = 0; k < 3; ++k) {
            const uint64_t a = uint32_t(t[3 * i + k]), b = uint32_t(t[3 * i + (k + 1) % 3]);
            if (++edges[(a << 32) | b] > 1)
                throw mesh_error(dom, "directed edge used twice (inconsistent orientation or non-manifold)");
        }
    for (const auto &e : edges) {
        const uint64_t a = e.first >> 32, b = e.first & 0xffffffffu;
        if (edges.find((b << 32) | a) == edges.end()) throw mesh_error(dom, "open edge (surface not closed)");
    }
    // outward orientation: positive enclosed volume
    double vol = 0.0;
    for (int64_t i = 0; i < nt; ++i) {
        const double *A = v + 3 * t[3 * i], *B = v + 3 * t[3 * i + 1], *C = v + 3 * t[3 * i + 2];
        vol += A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0]) + A[2] * (B[0] * C[1] - B[1] * C[0]);
    }
    if (!(vol > 0.0)) throw mesh_error(dom, "normals point inwards (negative enclosed volume)");
}

void validate_disjoint(const std::vector<DomInfo> &doms, const std::vector<double> &verts)
{
    // min vertex-vertex distance between different domains through a uniform grid
    const int64_t NV = int64_t(verts.size() / 3);
    if (doms.size() < 2) return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < NV; ++i)
        for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], verts[3 * i + d]); hi[d] = std::max(hi[d], verts[3 * i + d]); }
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    const double tol = 1e-9 * ext;
    const double cell = ext / std::max<double>(1.0, std::cbrt(double(NV)));
    std::unordered_map<int64_t, std::vector<int32_t>> grid;
    std::vector<int> dom_of(NV);
    for (size_t j = 0; j < doms.size(); ++j)
        for (int64_t i = 0; i < doms[j].nv; ++i) dom_of[doms[j].v_off + i] = int(j);
    auto key = [&](int64_t a, int64_t b, int64_t c) { return (a * 1048576 + b) * 1048576 + c; };
    for (int64_t i = 0; i < NV; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = int64_t((verts[3 * i + d] - lo[d]) / cell);
        grid[key(c[0], c[1], c[2])].push_back(int32_t(i));
    }
    for (int64_t i = 0; i < NV; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = int64_t((verts[3 * i + d] - lo[d]) / cell);
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = grid.find(key(c[0] + dx, c[1] + dy, c[2] + dz));
                    if (it == grid.end()) continue;
                    for (int32_t j : it->second) {
                        if (dom_of[j] == dom_of[i]) continue;
                        double d2 = 0;
                        for (int d = 0; d < 3; ++d) { double q = verts[3 * i + d] - verts[3 * j + d]; d2 += q * q; }
                        if (d2 <= tol * tol)
                            throw Error{BEM_ERR_MESH, "domains " + std::to_string(dom_of[i]) + " and " +
                                                          std::to_string(dom_of[j]) + " touch (shared vertex position)"};
                    }
                }
    }
}

// Vertex -> incident triangles (global indices).
static void vertex_triangles(const bem_problem &p, std::vector<int32_t> &ptr, std::vector<int32_t> &lst)
{
    ptr.assign(p.NV + 1, 0);
    for (int64_t i = 0; i < 3 * p.NT; ++i) ptr[p.h_tris[i] + 1]++;
    for (int64_t i = 0; i < p.NV; ++i) ptr[i + 1] += ptr[i];
    lst.resize(3 * p.NT);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t t = 0; t < p.NT; ++t)
        for (int a = 0; a < 3; ++a) lst[fill[p.h_tris[3 * t + a]]++] = int32_t(t);
}

void touching_pairs(const bem_problem &p, std::vector<SingularItem> &items)
{
    std::vector<int32_t> ptr, lst;
    vertex_triangles(p, ptr, lst);
    std::vector<SingularItem> by_cls[4];
    std::vector<int32_t> nb;
    // triangle -> domain (contiguous triangle ranges)
    std::vector<int> tdom(p.NT);
    for (size_t j = 0; j < p.doms.size(); ++j)
        for (int64_t i = 0; i < p.doms[j].nt; ++i) tdom[p.doms[j].t_off + i] = int(j);
    for (int64_t t = 0; t < p.NT; ++t) {
        nb.clear();
        for (int a = 0; a < 3; ++a) {
            const int32_t g = p.h_tris[3 * t + a];
            for (int32_t k = ptr[g]; k < ptr[g + 1]; ++k) nb.push_back(lst[k]);
        }
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        const int32_t *T = &p.h_tris[3 * t];
        for (int32_t s : nb) {
            const int32_t *S = &p.h_tris[3 * s];
            int ti[3], si[3], ns = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    if (T[a] == S[b]) { ti[ns] = a; si[ns] = b; ++ns; }
            SingularItem it{};
            it.t = int(t);
            it.s = s;
            if (ns == 3) {
                it.cls = COINCIDENT;
                for (int a = 0; a < 3; ++a) {
                    it.pt[a] = a;
                    for (int b = 0; b < 3; ++b)
                        if (S[b] == T[a]) it.ps[a] = b;
                }
            } else if (ns == 2) {
                it.cls = EDGE;
                it.pt[0] = ti[0]; it.pt[1] = ti[1]; it.pt[2] = 3 - ti[0] - ti[1];
                it.ps[0] = si[0]; it.ps[1] = si[1]; it.ps[2] = 3 - si[0] - si[1];
            } else {
                it.cls = VERTEX;
                it.pt[0] = ti[0]; it.pt[1] = (ti[0] + 1) % 3; it.pt[2] = (ti[0] + 2) % 3;
                it.ps[0] = si[0]; it.ps[1] = (si[0] + 1) % 3; it.ps[2] = (si[0] + 2) % 3;
            }
            // exterior pass (index 0) and the interior pass of the domain (index 1 + j)
            it.pass = 0;
            by_cls[it.cls].push_back(it);
            it.pass = 1 + tdom[t];
            by_cls[it.cls].push_back(it);
        }
    }
    items.clear();
    for (int c = COINCIDENT; c >= VERTEX; --c) items.insert(items.end(), by_cls[c].begin(), by_cls[c].end());
}

void correction_pattern(const bem_problem &p, const std::vector<SingularItem> &items,
                        std::vector<int32_t> &cptr, std::vector<int32_t> &ccol,
                        std::vector<int32_t> &contrib_ptr, std::vector<int32_t> &contrib_idx)
{
    // pattern per test vertex: sorted unique trial vertices of touching pairs
    std::vector<std::vector<int32_t>> rows(p.NV);
    for (const auto &it : items) {
        if (it.pass != 0) continue;  // both passes share the pattern
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) rows[p.h_tris[3 * it.t + a]].push_back(p.h_tris[3 * it.s + b]);
    }
    cptr.assign(p.NV + 1, 0);
    for (int64_t g = 0; g < p.NV; ++g) {
        auto &r = rows[g];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        cptr[g + 1] = cptr[g] + int32_t(r.size());
    }
    ccol.resize(cptr[p.NV]);
    for (int64_t g = 0; g < p.NV; ++g) std::copy(rows[g].begin(), rows[g].end(), ccol.begin() + cptr[g]);
    // slot of every (item, a, b) contribution: counting sort in item order
    const int64_t nnz = cptr[p.NV];
    std::vector<int32_t> slot_of(items.size() * 9);
    contrib_ptr.assign(nnz + 1, 0);
    for (size_t i = 0; i < items.size(); ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const int32_t g = p.h_tris[3 * items[i].t + a], h = p.h_tris[3 * items[i].s + b];
                const int32_t *beg = &ccol[cptr[g]], *end = &ccol[cptr[g + 1]];
                const int32_t s = int32_t(std::lower_bound(beg, end, h) - ccol.data());
                slot_of[9 * i + 3 * a + b] = s;
                contrib_ptr[s + 1]++;
            }
    for (int64_t s = 0; s < nnz; ++s) contrib_ptr[s + 1] += contrib_ptr[s];
    contrib_idx.resize(items.size() * 9);
    std::vector<int32_t> fill(contrib_ptr.begin(), contrib_ptr.end() - 1);
    for (size_t c = 0; c < items.size() * 9; ++c) contrib_idx[fill[slot_of[c]]++] = int32_t(c);
}

// Gauss-Legendre on [0,1] by Newton iteration on the three-term recurrence.
static void gauss01(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                p0 = 1.0; p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        x[i] = 0.5 * (1.0 + z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

std::vector<double> singular_rule(int cls, int n)
{
    std::vector<double> g, gw, out;
    gauss01(n, g, gw);
    auto put = [&](double a, double b, double c, double d, double w) {
        out.push_back(a); out.push_back(b); out.push_back(c); out.push_back(d); out.push_back(w);
    };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                for (int l = 0; l < n; ++l) {
                    const double u = g[i], a = g[j], b = g[k], c = g[l];
                    const double w = gw[i] * gw[j] * gw[k] * gw[l];
                    const double u3 = u * u * u;
                    if (cls == COINCIDENT) {
                        // six simplices around the diagonal x = y; Jacobian u^3 a^2 b
                        const double J = w * u3 * a * a * b;
                        put(u, u * (1 - a + a * b), u * (1 - a * b * c), u * (1 - a), J);
                        put(u * (1 - a * b * c), u * (1 - a), u, u * (1 - a + a * b), J);
                        put(u, u * a * (1 - b + b * c), u * (1 - a * b), u * a * (1 - b), J);
                        put(u * (1 - a * b), u * a * (1 - b), u, u * a * (1 - b + b * c), J);
                        put(u * (1 - a * b * c), u * a * (1 - b * c), u, u * a * (1 - b), J);
                        put(u, u * a * (1 - b), u * (1 - a * b * c), u * a * (1 - b * c), J);
                    } else if (cls == EDGE) {
                        // five pieces around the common edge s2 = 0
                        put(u, u * a * c, u * (1 - a * b), u * a * (1 - b), w * u3 * a * a);
                        const double J = w * u3 * a * a * b;
                        put(u, u * a, u * (1 - a * b * c), u * a * b * (1 - c), J);
                        put(u * (1 - a * b), u * a * (1 - b), u, u * a * b * c, J);
                        put(u * (1 - a * b * c), u * a * b * (1 - c), u, u * a, J);
                        put(u * (1 - a * b * c), u * a * (1 - b * c), u, u * a * b, J);
                    } else {
                        // two pieces around the common corner
                        const double J = w * u3 * b;
                        put(u, u * a, u * b, u * b * c, J);
                        put(u * b, u * b * c, u, u * a, J);
                    }
                }
    return out;
}

}  // namespace bem
