"""Semi-analytic Laplace double integrals over pairs of triangles.

Independent of the Sauter-Schwab rule: the inner integral of 1/|x - y| over a
flat triangle has a closed form (sum over edges of logarithms minus the
height times the subtended solid angle; Wilton et al. 1984, Graglia 1993),
and the outer integral over the test triangle is done with tanh-sinh
quadrature on the collapsed square, which converges exponentially even with
the logarithmic edge singularities of the inner potential.
"""
from __future__ import annotations

import numpy as np


def inner_potential(P, x):
    """int_T dA_y / |x - y| for triangle P [3, 3] and points x [..., 3]."""
    P = np.asarray(P, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n = n / np.linalg.norm(n)
    w = (x - P[0]) @ n                                  # height above the plane
    xp = x - w[..., None] * n                           # projection onto the plane
    out = np.zeros(x.shape[:-1])
    aw = np.abs(w)
    for i in range(3):
        a, b = P[i], P[(i + 1) % 3]
        l = np.linalg.norm(b - a)
        s = (b - a) / l
        m = np.cross(s, n)                              # in-plane outward edge normal (CCW)
        d = (a - xp) @ m                                # signed distance projection->edge (>0 inside)
        lm = (a - xp) @ s
        lp = (b - xp) @ s
        Rm = np.linalg.norm(x - a, axis=-1)
        Rp = np.linalg.norm(x - b, axis=-1)
        R0sq = d * d + w * w
        with np.errstate(divide="ignore", invalid="ignore"):
            # R + l without cancellation: (R + l)(R - l) = d^2 + w^2
            Ap = np.where(lp >= 0.0, Rp + lp, R0sq / (Rp - lp))
            Am = np.where(lm >= 0.0, Rm + lm, R0sq / (Rm - lm))
            lg = np.log(Ap / Am)
            dlg = np.where(np.abs(d) < 1e-15, 0.0, d * lg)
            at = np.arctan2(d * lp, R0sq + aw * Rp) - np.arctan2(d * lm, R0sq + aw * Rm)
        out += dlg - aw * at
    return out


def tanh_sinh(n=40, h=None):
    """Tanh-sinh nodes/weights on [0, 1]."""
    if h is None:
        h = 6.0 / n
    k = np.arange(-n, n + 1) * h
    u = 0.5 * np.pi * np.sinh(k)
    x = 0.5 * (1.0 + np.tanh(u))
    w = 0.5 * h * 0.5 * np.pi * np.cosh(k) / np.cosh(u) ** 2
    keep = (x > 0) & (x < 1)
    return x[keep], w[keep]


def outer_integral(P, f, n=40):
    """int_T f(x) dA over triangle P via the collapsed square (Duffy) map."""
    P = np.asarray(P, dtype=np.float64)
    t, wt = tanh_sinh(n)
    U, V = np.meshgrid(t, t, indexing="ij")
    WU, WV = np.meshgrid(wt, wt, indexing="ij")
    # (u, v) in [0,1]^2 -> (s1, s2) = (u, u v) on {0 <= s2 <= s1 <= 1}, Jacobian u
    s1, s2 = U, U * V
    X = P[0] + s1[..., None] * (P[1] - P[0]) + s2[..., None] * (P[2] - P[1])
    J = np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[1]))
    return float(np.sum(WU * WV * U * J * f(X)))


def laplace_pair(Pt, Ps, n=40):
    """int_t int_s 1 / |x - y| over two triangles (any relative position)."""
    return outer_integral(Pt, lambda X: inner_potential(Ps, X), n)
