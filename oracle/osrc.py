"""FP64 oracle of the OSRC block-diagonal preconditioner (test infrastructure).

Paper, section "Operator preconditioning": the preconditioner is
C = blockdiag_j(diag(Lambda_DtN^{j,+}, Lambda_NtD^{j,+})) (eqs. OSRC_prec,
OSRC_prec_blocks) with the on-surface radiation condition approximations
(eq. OSRC_DtN_NtD_maps)
    Lambda_DtN ~ i k sqrt(1 + Delta_G / k_eps^2),
    Lambda_NtD ~ (1/(i k)) (1 + Delta_G / k_eps^2)^(-1/2),
k_eps = k + i eps, and the square root replaced by an N-term Pade expansion.
The maps act on the Dirichlet-equation row (-K u_D + V u_N: Lambda_DtN V ~
-1/2 + K') and on the Neumann-equation row (W u_D + K' u_N: Lambda_NtD W ~
-1/2 - K) of every domain (eq. OSRC_maps_properties).

Readings (the paper is silent or garbled here): k = k0 (exterior); damping
eps = 0.4 k^(1/3) R_eps^(-2/3) (the printed exponent -1/3 on k is not
dimensionally a wavenumber); the Pade expansion is the branch-rotated one of
Milinazzo, Zala & Brooke (angle theta); Delta_G is discretised in strong form
as -M^-1 S with the P1 mass M and stiffness S; the Galerkin residual is
mapped to coefficients by M^-1 before the maps act.
"""
from __future__ import annotations

import numpy as np

from . import mass_matrix, stiffness_matrix, offsets


def damped_wavenumber(k, r_eps):
    k = complex(k)
    return k + 1j * 0.4 * k.real ** (1.0 / 3.0) * r_eps ** (-2.0 / 3.0)


def pade_coefficients(n_pade, theta):
    """C0, A_l, B_l with sqrt(1 + z) ~ C0 + sum_l A_l z / (1 + B_l z).

    Standard Pade of sqrt(1 + w): 1 + sum a_l w / (1 + b_l w) with
    a_l = 2/(2N+1) sin^2(l pi/(2N+1)), b_l = cos^2(l pi/(2N+1)); the branch cut
    is rotated by writing sqrt(1 + z) = e^{i theta/2} sqrt(1 + w),
    w = e^{-i theta}(1 + z) - 1, and re-expanding in z.
    """
    N = int(n_pade)
    l = np.arange(1, N + 1)
    a = 2.0 / (2 * N + 1) * np.sin(l * np.pi / (2 * N + 1)) ** 2
    b = np.cos(l * np.pi / (2 * N + 1)) ** 2
    e = np.exp(-1j * theta)
    c = e - 1.0
    D = 1.0 + b * c
    C0 = np.exp(1j * theta / 2.0) * (1.0 + np.sum(a * c / D))
    A = np.exp(-1j * theta / 2.0) * a / D ** 2
    B = e * b / D
    return C0, A, B


def pade_sqrt(z, n_pade, theta):
    C0, A, B = pade_coefficients(n_pade, theta)
    z = np.asarray(z, dtype=np.complex128)
    return C0 + np.sum(A[:, None] * z[None, :] / (1.0 + B[:, None] * z[None, :]), axis=0)


def osrc_maps(v, t, k, r_eps, n_pade, theta):
    """Dense strong-form matrices (Lambda_DtN, Lambda_NtD) on one surface."""
    M = mass_matrix(v, t)
    S = stiffness_matrix(v, t)
    ke = damped_wavenumber(k, r_eps)
    Sp = S / ke ** 2                       # S' = S / k_eps^2, X = -M^-1 S'
    C0, A, B = pade_coefficients(n_pade, theta)
    n = M.shape[0]
    # sqrt(1 + X) = C0 I - sum_l A_l (M - B_l S')^-1 S'
    root = C0 * np.eye(n, dtype=np.complex128)
    for Al, Bl in zip(A, B):
        root -= Al * np.linalg.solve(M - Bl * Sp, Sp)
    ik = 1j * complex(k)
    dtn = ik * root
    # (1 + X)^-1/2 = (1 + X)^-1 sqrt(1 + X),  (1 + X)^-1 = (M - S')^-1 M
    ntd = (1.0 / ik) * np.linalg.solve(M - Sp, M @ root)
    return dtn, ntd, M


def preconditioner_matrix(problem, r_eps, n_pade=4, theta=np.pi / 3):
    """Dense left preconditioner in the unknown order of the PMCHWT system.

    The paper permutes the unknowns of every domain to [u_N; u_D] so that V and
    W sit on the diagonal of the Calderon blocks, and applies
    C = diag(Lambda_DtN, Lambda_NtD) to the (unchanged) rows:
    C A Pi y = C b with u = Pi y.  GMRES on that system is identical (up to the
    same permutation of all vectors) to GMRES on (Pi C) A u = Pi C b, so the
    returned matrix is P = Pi C: its u_D positions receive
    Lambda_NtD M^-1 (Neumann-equation rows) and its u_N positions
    Lambda_DtN M^-1 (Dirichlet-equation rows).
    """
    off = offsets(problem)
    n = off[-1]
    P = np.zeros((n, n), dtype=np.complex128)
    for j, d in enumerate(problem.domains):
        dtn, ntd, M = osrc_maps(d.vertices, d.triangles, problem.k0, r_eps, n_pade, theta)
        Minv = np.linalg.inv(M)
        nv = d.n_vertices
        P[off[j] + nv:off[j + 1], off[j]:off[j] + nv] = dtn @ Minv
        P[off[j]:off[j] + nv, off[j] + nv:off[j + 1]] = ntd @ Minv
    return P
