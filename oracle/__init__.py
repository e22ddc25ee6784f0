"""FP64 CPU oracle for the multiple-domain PMCHWT boundary element method.

TEST INFRASTRUCTURE.  This package is the independent, plain and slow
reference implementation that the GPU library is checked against.  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the GPU library (``paper_1910_01011_amd``) never
imports it and shares no code with it.  The compiled part lives in
``bem_oracle.c`` and is built by ``oracle/build.py``.

What it computes (paper sections cited per function):

* Galerkin P1 matrices of V, K, K', W for one pair of surfaces (Appendix A
  operator definitions; Galerkin discretisation in "Operator preconditioning").
* The PMCHWT block matrix (eq. Form2_matrix_format_p1 with the Calderon
  operator [[-K, V], [W, K']] and the density scaling D_j^-1 A D_j of
  eq. Form1_calderon_sys_int_ptot) and its right-hand side
  (eq. Galerkin_disc_rhs1).
* GMRES(restart) and dense LU solves (numerical experiments section).
* Single/double layer potentials and the representation formula
  (eq. rep_formula_gen) for the field off the surface.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BEM_ORACLE_LIB selects another build of bem_oracle.c (the sanitizer build)
_LIB_PATH = os.path.join(_HERE, os.environ.get("BEM_ORACLE_LIB", "_bem_oracle.so"))
_lib = None

FAR, VERTEX, EDGE, COINCIDENT = 0, 1, 2, 3


def lib():
    """Load the compiled oracle (built by ``oracle/build.py``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        L.orc_far_rule.argtypes = [dp, dp, dp]
        L.orc_gauss_legendre01.argtypes = [ctypes.c_int, dp, dp]
        L.orc_ss_rule_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_ss_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_element_pair.argtypes = [dp, ip, dp, ip, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, dp]
        L.orc_operator_rows.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int,
                                        dp, ctypes.c_int, ip, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        lp, ctypes.c_int, dp, dp, dp, dp]
        L.orc_potentials.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     dp, dp, dp, ctypes.c_int, dp, dp]
        L.orc_winding.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _l(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))


def _mesh(v, t):
    return (np.ascontiguousarray(v, dtype=np.float64), np.ascontiguousarray(t, dtype=np.int32))


# --------------------------------------------------------------------------
# quadrature rules (exposed so the tests can pin them)
# --------------------------------------------------------------------------

def far_rule():
    """6-point degree-4 triangle rule: (xi1, xi2, w) with sum(w) = 1."""
    x1, x2, w = np.zeros(6), np.zeros(6), np.zeros(6)
    lib().orc_far_rule(_d(x1), _d(x2), _d(w))
    return x1, x2, w


def gauss_legendre01(n):
    x, w = np.zeros(n), np.zeros(n)
    lib().orc_gauss_legendre01(n, _d(x), _d(w))
    return x, w


def ss_rule(cls, n):
    """Sauter-Schwab rule of a pair class on T x T, T = {0 <= s2 <= s1 <= 1}."""
    m = lib().orc_ss_rule_size(cls, n)
    xh, yh, w = np.zeros((m, 2)), np.zeros((m, 2)), np.zeros(m)
    lib().orc_ss_rule(cls, n, _d(xh), _d(yh), _d(w))
    return xh, yh, w


def element_pair(Pt, lt, Ps, ls, kappa, ss_n=6, force_far=False):
    """Element matrices [4 (V,K,K',W), 3, 3] of one pair of triangles.

    ``lt``/``ls`` are integer vertex labels; equal labels mark shared vertices
    and select the singular rule.  Returns (class, E).
    """
    Pt = np.ascontiguousarray(Pt, dtype=np.float64).reshape(9)
    Ps = np.ascontiguousarray(Ps, dtype=np.float64).reshape(9)
    lt = np.ascontiguousarray(lt, dtype=np.int32)
    ls = np.ascontiguousarray(ls, dtype=np.int32)
    out = np.zeros(4 * 9, dtype=np.complex128)
    kappa = complex(kappa)
    cls = lib().orc_element_pair(_d(Pt), _i(lt), _d(Ps), _i(ls), kappa.real, kappa.imag, int(ss_n),
                                 int(bool(force_far)), _d(out.view(np.float64)))
    return cls, out.reshape(4, 3, 3)


# --------------------------------------------------------------------------
# Galerkin matrices
# --------------------------------------------------------------------------

def operator_rows(test_mesh, trial_mesh, same_mesh, kappa, rows=None, ss_n=6):
    """Rows of V, K, K', W (test vertices ``rows`` x all trial vertices).

    Returns a tuple of four complex arrays [len(rows), n_v_trial].
    """
    vt, tt = _mesh(*test_mesh)
    vs, ts = _mesh(*trial_mesh)
    if rows is None:
        rows = np.arange(vt.shape[0])
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    nr, nvs = rows.shape[0], vs.shape[0]
    outs = [np.zeros((nr, nvs), dtype=np.complex128) for _ in range(4)]
    kappa = complex(kappa)
    rc = lib().orc_operator_rows(_d(vt), vt.shape[0], _i(tt), tt.shape[0],
                                 _d(vs), vs.shape[0], _i(ts), ts.shape[0],
                                 int(bool(same_mesh)), kappa.real, kappa.imag, int(ss_n),
                                 _l(rows), nr, *[_d(o.view(np.float64)) for o in outs])
    if rc != 0:
        raise MemoryError("oracle: operator_rows allocation failed")
    return tuple(outs)


def operators(mesh, kappa, ss_n=6):
    """Full Galerkin matrices (V, K, K', W) of one closed surface."""
    return operator_rows(mesh, mesh, True, kappa, None, ss_n)


def single_layer_matrix(problem, ss_n=6):
    """Galerkin single-layer matrix at k0 on the union of all boundaries
    (Appendix A, single-layer operator): block (i, j) is V_k0 with test
    functions on boundary i and trial functions on boundary j (singular rules
    only within one boundary).  Vertices in domain order."""
    meshes = [(d.vertices, d.triangles) for d in problem.domains]
    nv = [d.n_vertices for d in problem.domains]
    off = np.concatenate([[0], np.cumsum(nv)])
    V = np.zeros((off[-1], off[-1]), dtype=np.complex128)
    for i, mi in enumerate(meshes):
        for j, mj in enumerate(meshes):
            V[off[i]:off[i + 1], off[j]:off[j + 1]] = operator_rows(mi, mj, i == j, problem.k0, None, ss_n)[0]
    return V


def mass_matrix(v, t):
    """P1 mass matrix: M^T_ab = |T| (1 + delta_ab) / 12 (dense)."""
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t)
    nv = v.shape[0]
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)
    M = np.zeros((nv, nv))
    for a in range(3):
        for b in range(3):
            np.add.at(M, (t[:, a], t[:, b]), area * (2.0 if a == b else 1.0) / 12.0)
    return M


def stiffness_matrix(v, t):
    """P1 Laplace-Beltrami stiffness: S^T_ab = e_a . e_b / (4 |T|), e_a = P_{a+2} - P_{a+1}."""
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t)
    nv = v.shape[0]
    P = [v[t[:, a]] for a in range(3)]
    area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]), axis=1)
    e = [P[(a + 2) % 3] - P[(a + 1) % 3] for a in range(3)]
    S = np.zeros((nv, nv))
    for a in range(3):
        for b in range(3):
            np.add.at(S, (t[:, a], t[:, b]), np.einsum("ij,ij->i", e[a], e[b]) / (4.0 * area))
    return S


# --------------------------------------------------------------------------
# PMCHWT system
# --------------------------------------------------------------------------

def offsets(problem):
    """Start of each domain's [u_D; u_N] block in the unknown vector."""
    off = [0]
    for d in problem.domains:
        off.append(off[-1] + 2 * d.n_vertices)
    return off


def _add_block(A, r0, c0, nr, nc, V, K, Kp, W, sV=1.0, sW=1.0, row_sel=None):
    """Add the Calderon block [[-K, sV V], [sW W, K']] at (r0, c0)."""
    A[r0:r0 + nr, c0:c0 + nc] += -K
    A[r0:r0 + nr, c0 + nc:c0 + 2 * nc] += sV * V
    A[r0 + nr:r0 + 2 * nr, c0:c0 + nc] += sW * W
    A[r0 + nr:r0 + 2 * nr, c0 + nc:c0 + 2 * nc] += Kp


def pmchwt_matrix(problem, ss_n=6):
    """Dense PMCHWT Galerkin matrix.

    Block (j, i) = A^{ji}_{k0}; the diagonal blocks add the interior
    operator D_j^-1 A^j_{kj} D_j with D_j = diag(1, rho_j/rho_0), i.e.
    [[-K_kj, (rho_j/rho_0) V_kj], [(rho_0/rho_j) W_kj, K'_kj]]
    (paper eqs. Form1_BCs, Form1_calderon_sys_int_ptot, Form2_calderon_sys_simp3,
    Form2_matrix_format_p1).  No identity terms remain.
    """
    off = offsets(problem)
    n = off[-1]
    A = np.zeros((n, n), dtype=np.complex128)
    doms = problem.domains
    for j, dj in enumerate(doms):
        for i, di in enumerate(doms):
            ops = operator_rows((dj.vertices, dj.triangles), (di.vertices, di.triangles), i == j,
                                problem.k0, None, ss_n)
            Aj = np.zeros((2 * dj.n_vertices, 2 * di.n_vertices), dtype=np.complex128)
            _add_block(Aj, 0, 0, dj.n_vertices, di.n_vertices, *ops)
            A[off[j]:off[j + 1], off[i]:off[i + 1]] += Aj
        ops = operators((dj.vertices, dj.triangles), dj.k, ss_n)
        Aj = np.zeros((2 * dj.n_vertices, 2 * dj.n_vertices), dtype=np.complex128)
        _add_block(Aj, 0, 0, dj.n_vertices, dj.n_vertices, *ops,
                   sV=dj.rho / problem.rho0, sW=problem.rho0 / dj.rho)
        A[off[j]:off[j + 1], off[j]:off[j + 1]] += Aj
    return A


def pmchwt_rows(problem, rows, ss_n=6):
    """Selected rows of the dense PMCHWT matrix (same definition as pmchwt_matrix)."""
    rows = np.asarray(rows, dtype=np.int64)
    off = offsets(problem)
    n = off[-1]
    out = np.zeros((rows.shape[0], n), dtype=np.complex128)
    doms = problem.domains
    for j, dj in enumerate(doms):
        sel = np.nonzero((rows >= off[j]) & (rows < off[j + 1]))[0]
        if sel.size == 0:
            continue
        loc = rows[sel] - off[j]
        is_n = loc >= dj.n_vertices
        vtx = np.where(is_n, loc - dj.n_vertices, loc)
        uv, inv = np.unique(vtx, return_inverse=True)
        mj = (dj.vertices, dj.triangles)

        def put(i, c0, nc, V, K, Kp, W, sV=1.0, sW=1.0):
            Vr, Kr, Kpr, Wr = V[inv], K[inv], Kp[inv], W[inv]
            d_rows = ~is_n
            blockD = np.concatenate([-Kr, sV * Vr], axis=1)
            blockN = np.concatenate([sW * Wr, Kpr], axis=1)
            out[sel[d_rows], c0:c0 + 2 * nc] += blockD[d_rows]
            out[sel[is_n], c0:c0 + 2 * nc] += blockN[is_n]

        for i, di in enumerate(doms):
            ops = operator_rows(mj, (di.vertices, di.triangles), i == j, problem.k0, uv, ss_n)
            put(i, off[i], di.n_vertices, *ops)
        ops = operator_rows(mj, mj, True, dj.k, uv, ss_n)
        put(j, off[j], dj.n_vertices, *ops, sV=dj.rho / problem.rho0, sW=problem.rho0 / dj.rho)
    return out


def _points_on(v, t):
    """Far-rule points, P1 basis values and weights |T| w_q per triangle."""
    x1, x2, w = far_rule()
    lam = np.stack([1.0 - x1 - x2, x1, x2], axis=1)            # [6, 3]
    P = np.stack([v[t[:, a]] for a in range(3)], axis=1)        # [nt, 3, 3]
    X = np.einsum("qa,tad->tqd", lam, P)                        # [nt, 6, 3]
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    nrm = nrm / (2.0 * area[:, None])
    return X, lam, area[:, None] * w[None, :], nrm


def project_rhs(v, t, p_fn, dpdn_fn):
    """Galerkin projections <g, phi_r> of Dirichlet and Neumann data.

    ``p_fn(X)`` and ``dpdn_fn(X, n)`` evaluate the data at points [.., 3] with
    normals; the integrals use the 6-point rule (eq. Galerkin_disc_rhs1).
    """
    X, lam, W, nrm = _points_on(v, t)
    p = p_fn(X)                                                  # [nt, 6]
    g = dpdn_fn(X, np.broadcast_to(nrm[:, None, :], X.shape))
    bD = np.zeros(v.shape[0], dtype=np.complex128)
    bN = np.zeros(v.shape[0], dtype=np.complex128)
    for a in range(3):
        np.add.at(bD, t[:, a], np.sum(W * lam[None, :, a] * p, axis=1))
        np.add.at(bN, t[:, a], np.sum(W * lam[None, :, a] * g, axis=1))
    return bD, bN


def plane_wave(k0, direction=(0.0, 0.0, 1.0), amplitude=1.0):
    """p_inc = A exp(i k0 d.x) and its normal derivative i k0 (d.n) p_inc."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    k0 = complex(k0)

    def p(X):
        return amplitude * np.exp(1j * k0 * (X @ d))

    def dpdn(X, n):
        return 1j * k0 * (n @ d) * p(X)

    return p, dpdn


def point_sources(k0, positions, amplitudes):
    """Sum of monopoles a_s G_k0(x, s): a radiating solution away from the sources."""
    S = np.atleast_2d(np.asarray(positions, dtype=np.float64))
    a = np.atleast_1d(np.asarray(amplitudes, dtype=np.complex128))
    k0 = complex(k0)

    def p(X):
        out = np.zeros(X.shape[:-1], dtype=np.complex128)
        for s, am in zip(S, a):
            r = np.linalg.norm(X - s, axis=-1)
            out += am * np.exp(1j * k0 * r) / (4.0 * np.pi * r)
        return out

    def dpdn(X, n):
        out = np.zeros(X.shape[:-1], dtype=np.complex128)
        for s, am in zip(S, a):
            d = X - s
            r = np.linalg.norm(d, axis=-1)
            G = np.exp(1j * k0 * r) / (4.0 * np.pi * r)
            out += am * G * (1j * k0 * r - 1.0) / r ** 2 * np.sum(d * n, axis=-1)
        return out

    return p, dpdn


def rhs(problem, p_fn, dpdn_fn):
    """b_j = <gamma^{j,+} p_inc, phi> for every domain, stacked like the unknowns."""
    parts = []
    for d in problem.domains:
        bD, bN = project_rhs(d.vertices, d.triangles, p_fn, dpdn_fn)
        parts += [bD, bN]
    return np.concatenate(parts)


def solve_lu(A, b):
    """Dense LU solve (LAPACK through numpy)."""
    return np.linalg.solve(A, b)


def gmres(matvec, b, restart=100, tol=1e-5, maxiter=1000):
    """Restarted GMRES with zero initial guess (Saad & Schultz).

    Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
    matrix; stops when ||b - A x|| / ||b|| <= tol.  Returns
    (x, iterations, relative residual history).
    """
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    hist = [1.0]
    it = 0
    while it < maxiter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        m = restart
        Q = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        Q[0] = r / beta
        j_used = 0
        for j in range(m):
            w = matvec(Q[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(Q[i], w)
                w = w - H[i, j] * Q[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                Q[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            # unitary rotation [[c, s], [-conj(s), conj(c)]] that maps
            # (H[j,j], H[j+1,j]) to (rho, 0)
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            cs[j] = np.conj(H[j, j]) / den
            sn[j] = np.conj(H[j + 1, j]) / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_used = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if hist[-1] <= tol or it >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + Q[:j_used].T @ y
        if hist[-1] <= tol:
            break
    return x, it, hist


# --------------------------------------------------------------------------
# potentials and field (eq. rep_formula_gen, eqs. SLP/DLP off the surface)
# --------------------------------------------------------------------------

def potentials(mesh, kappa, phi, psi, points):
    """(SL psi, DL phi) at points off the surface (6-point rule on sources)."""
    v, t = _mesh(*mesh)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    sl = np.zeros(pts.shape[0], dtype=np.complex128)
    dl = np.zeros(pts.shape[0], dtype=np.complex128)
    kappa = complex(kappa)
    lib().orc_potentials(_d(v), v.shape[0], _i(t), t.shape[0], kappa.real, kappa.imag,
                         _d(phi.view(np.float64)), _d(psi.view(np.float64)), _d(pts), pts.shape[0],
                         _d(sl.view(np.float64)), _d(dl.view(np.float64)))
    return sl, dl


def winding(mesh, points):
    v, t = _mesh(*mesh)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    lib().orc_winding(_d(v), v.shape[0], _i(t), t.shape[0], _d(pts), pts.shape[0], _d(out))
    return out


def mean_edge(v, t):
    """Mean edge length h of a triangle mesh, every edge counted from both of its
    triangles (each triangle's three sides averaged over the mesh)."""
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t)
    sides = [np.linalg.norm(v[t[:, (e + 1) % 3]] - v[t[:, e]], axis=1) for e in range(3)]
    return float(np.mean(np.concatenate(sides)))


def triangle_distance(v, t, x):
    """Distance from the point x to each triangle of (v, t).

    The nearest point of triangle (A, B, C) is A + s (B - A) + r (C - A) with
    (s, r) minimising the squared distance over s, r >= 0, s + r <= 1: the free
    minimiser (normal equations of the 2 x 2 least-squares problem) if it lies
    in that set, else the best point of the three sides, each a clamped 1-D
    minimisation.
    """
    v = np.asarray(v, dtype=np.float64)
    A, B, C = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    x = np.asarray(x, dtype=np.float64)
    e1, e2, d = B - A, C - A, x - A
    g11, g12, g22 = (e1 * e1).sum(1), (e1 * e2).sum(1), (e2 * e2).sum(1)
    r1, r2 = (e1 * d).sum(1), (e2 * d).sum(1)
    det = g11 * g22 - g12 * g12
    s = (g22 * r1 - g12 * r2) / det
    r = (g11 * r2 - g12 * r1) / det
    free = (s >= 0) & (r >= 0) & (s + r <= 1)
    p_free = A + s[:, None] * e1 + r[:, None] * e2

    def side(P, Q):
        u = Q - P
        tt = np.clip(((x - P) * u).sum(1) / (u * u).sum(1), 0.0, 1.0)
        return np.linalg.norm(P + tt[:, None] * u - x, axis=1)

    best_side = np.minimum(np.minimum(side(A, B), side(B, C)), side(C, A))
    return np.where(free, np.linalg.norm(p_free - x, axis=1), best_side)


def near_surface(mesh, points, factor=2.0):
    """True where a point is closer than factor * h to the surface (h = mean edge)."""
    v, t = np.asarray(mesh[0], dtype=np.float64), np.asarray(mesh[1])
    h = mean_edge(v, t)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    return np.array([triangle_distance(v, t, x).min() < factor * h for x in pts], dtype=bool)


def field(problem, u, points, p_inc=None):
    """Total pressure at points from the boundary traces u = gamma^+ p_tot.

    Exterior: p = p_inc + sum_j [DL_k0 u_D^j - SL_k0 u_N^j]; inside domain j:
    p = SL_kj((rho_j/rho_0) u_N^j) - DL_kj u_D^j.  Region from the winding
    number (0 = exterior, j = domain j); the returned code is -1 for points
    closer than 2 h_j to boundary j (h_j its mean edge length), where the
    6-point rule is inaccurate; their field still uses the winding region.
    """
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    off = offsets(problem)
    region = np.zeros(pts.shape[0], dtype=np.int32)
    for j, d in enumerate(problem.domains):
        wn = winding((d.vertices, d.triangles), pts)
        region[np.rint(wn).astype(int) == 1] = j + 1
    p = np.zeros(pts.shape[0], dtype=np.complex128)
    ext = region == 0
    if p_inc is not None:
        p[ext] += p_inc(pts[ext])
    for j, d in enumerate(problem.domains):
        uD = u[off[j]:off[j] + d.n_vertices]
        uN = u[off[j] + d.n_vertices:off[j + 1]]
        m = (d.vertices, d.triangles)
        sl, dl = potentials(m, problem.k0, uD, uN, pts[ext])
        p[ext] += dl - sl
        inside = region == j + 1
        if inside.any():
            sl, dl = potentials(m, d.k, uD, (d.rho / problem.rho0) * uN, pts[inside])
            p[inside] += sl - dl
    flagged = region.copy()
    for d in problem.domains:
        flagged[near_surface((d.vertices, d.triangles), pts)] = -1
    return p, flagged


def piston_sources(k0, centres, normals, radius, amplitudes):
    """Monopoles equivalent to flat baffled pistons (test infrastructure).

    Each piston of radius a radiates p(x) = (-i k0 / 2 pi) A int_disc e^{i k0 r}/r dS
    (Rayleigh integral, unit rho c u).  The disc integral uses 3 Gauss-Legendre
    radii on [0, a] with the weight r dr and 8 equally spaced angles, i.e. 24
    monopoles a_s G(x, s) with a_s = (-i k0 / 2 pi) 4 pi A w_r r dtheta.
    Returns (positions [S, 3], amplitudes [S], piston index [S]).
    """
    g, gw = np.polynomial.legendre.leggauss(3)
    g, gw = (g + 1.0) / 2.0, gw / 2.0
    k0 = complex(k0)
    C = np.atleast_2d(np.asarray(centres, dtype=np.float64))
    Nn = np.atleast_2d(np.asarray(normals, dtype=np.float64))
    A = np.broadcast_to(np.asarray(amplitudes, dtype=np.complex128), (C.shape[0],))
    pos, amp, idx = [], [], []
    for e, (c, n, a_e) in enumerate(zip(C, Nn, A)):
        n = n / np.linalg.norm(n)
        helper = np.eye(3)[np.argmin(np.abs(n))]
        e1 = np.cross(n, helper)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(n, e1)
        for gi, wi in zip(g, gw):
            r = radius * gi
            for j in range(8):
                th = 2.0 * np.pi * j / 8.0
                pos.append(c + r * (np.cos(th) * e1 + np.sin(th) * e2))
                amp.append((-1j * k0 / (2.0 * np.pi)) * 4.0 * np.pi * a_e * (radius * wi) * r * (2.0 * np.pi / 8.0))
                idx.append(e)
    return np.asarray(pos), np.asarray(amp), np.asarray(idx)


def piston_field(k0, centres, normals, radius, amplitudes):
    """(p_fn, dpdn_fn) of the summed pistons (see piston_sources)."""
    pos, amp, _ = piston_sources(k0, centres, normals, radius, amplitudes)
    return point_sources(k0, pos, amp)
