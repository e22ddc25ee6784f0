"""Closed forms for a sphere (test infrastructure; used only as pins).

* Plane-wave transmission through a penetrable sphere by separation of
  variables (the analytic solution the paper validates against in its
  single-sphere model problem; Anderson 1950, Morse & Ingard 1968).
* Eigenvalues of V, K, K', W on a sphere for spherical harmonics of degree l.

Time dependence exp(-i w t), outgoing exp(i k r); h_l = h_l^(1) = j_l + i y_l.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _jh(l, z):
    j = special.spherical_jn(l, z)
    jd = special.spherical_jn(l, z, derivative=True)
    y = special.spherical_yn(l, z)
    yd = special.spherical_yn(l, z, derivative=True)
    return j, jd, j + 1j * y, jd + 1j * yd


def sphere_eigenvalues(l, k, a=1.0):
    """(lambda_V, lambda_K, lambda_K', lambda_W) for Y_l on a sphere of radius a.

    lambda_V = i k a^2 j_l h_l; lambda_K = lambda_K' = i k^2 a^2 j_l h_l' + 1/2;
    lambda_W = -i k^3 a^2 j_l' h_l' (arguments k a), for real k > 0.  They
    satisfy lambda_K^2 + lambda_V lambda_W = 1/4 (Calderon identity A^2 = I/4).
    """
    z = k * a
    j, jd, h, hd = _jh(l, z)
    lv = 1j * k * a * a * j * h
    lk = 1j * k * k * a * a * j * hd + 0.5
    lw = -1j * k ** 3 * a * a * jd * hd
    return lv, lk, lk, lw


def laplace_sphere_eigenvalues(l, a=1.0):
    """Laplace (k -> 0) limits: a/(2l+1), -1/(2(2l+1)), -1/(2(2l+1)), l(l+1)/((2l+1)a)."""
    return a / (2 * l + 1), -0.5 / (2 * l + 1), -0.5 / (2 * l + 1), l * (l + 1) / ((2 * l + 1) * a)


def n_terms(k0, a):
    return int(np.ceil(k0 * a + 4.0 * (k0 * a) ** (1.0 / 3.0) + 10))


def penetrable_sphere_coefficients(a, k0, k1, rho0, rho1, L=None):
    """A_l (scattered) and B_l (interior) for an incident exp(i k0 z).

    From continuity of p and of (1/rho) dp/dr at r = a (paper, model eq.):
    A_l = [q j_l(k0a) j_l'(k1a) - j_l'(k0a) j_l(k1a)] / [h_l'(k0a) j_l(k1a) - q h_l(k0a) j_l'(k1a)],
    q = (k1 rho0)/(k0 rho1); B_l = (j_l(k0a) + A_l h_l(k0a)) / j_l(k1a).
    """
    if L is None:
        L = n_terms(abs(k0), a)
    ls = np.arange(L + 1)
    q = (k1 * rho0) / (k0 * rho1)
    j0, j0d, h0, h0d = _jh(ls, k0 * a)
    j1 = special.spherical_jn(ls, k1 * a)
    j1d = special.spherical_jn(ls, k1 * a, derivative=True)
    A = (q * j0 * j1d - j0d * j1) / (h0d * j1 - q * h0 * j1d)
    B = (j0 + A * h0) / j1
    return ls, A, B


def sphere_traces(points, a, k0, k1, rho0, rho1):
    """(gamma_D p_tot, gamma_N p_tot) at points on the sphere |x| = a (normal = x/a)."""
    ls, A, _ = penetrable_sphere_coefficients(a, k0, k1, rho0, rho1)
    pts = np.asarray(points, dtype=np.float64)
    ct = pts[:, 2] / np.linalg.norm(pts, axis=1)
    j0, j0d, h0, h0d = _jh(ls, k0 * a)
    c = (1j ** ls) * (2 * ls + 1)
    P = np.stack([special.eval_legendre(l, ct) for l in ls], axis=1)
    gD = P @ (c * (j0 + A * h0))
    gN = k0 * (P @ (c * (j0d + A * h0d)))
    return gD, gN


def sphere_field(points, a, k0, k1, rho0, rho1):
    """Total pressure of the series solution at arbitrary points."""
    ls, A, B = penetrable_sphere_coefficients(a, k0, k1, rho0, rho1)
    pts = np.asarray(points, dtype=np.float64)
    r = np.linalg.norm(pts, axis=1)
    ct = np.where(r > 0, pts[:, 2] / np.where(r > 0, r, 1.0), 1.0)
    c = (1j ** ls) * (2 * ls + 1)
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    P = np.stack([special.eval_legendre(l, ct) for l in ls], axis=1)
    ext = r >= a
    if ext.any():
        h = special.spherical_jn(ls[None, :], k0 * r[ext, None]) + 1j * special.spherical_yn(ls[None, :], k0 * r[ext, None])
        out[ext] = np.exp(1j * k0 * pts[ext, 2]) + np.sum(P[ext] * c * A * h, axis=1)
    inn = ~ext
    if inn.any():
        j = special.spherical_jn(ls[None, :], k1 * r[inn, None])
        out[inn] = np.sum(P[inn] * c * B * j, axis=1)
    return out
