"""Pins of the OSRC preconditioner oracle (operator preconditioning section).

* The rotated Pade expansion converges to sqrt(1 + z) on the principal branch
  as the number of terms grows, including on the negative real axis beyond -1
  where the unrotated expansion has its branch cut.
* On a sphere, Delta_G Y_l = -l(l+1)/a^2 Y_l, so the discrete maps applied to
  the interpolant of Y_l reproduce the closed-form symbols
  i k R(-l(l+1)/(k_eps^2 a^2)) and R(.)/((i k)(1 - l(l+1)/(k_eps^2 a^2))) with
  O(h^2) error.
* The preconditioned PMCHWT system needs fewer GMRES iterations, independent
  of the mesh size, and has the same solution (low and high contrast).
"""
from __future__ import annotations

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import osrc
from bem_inputs import configs, meshes

pytestmark = pytest.mark.cpu


def test_pade_converges_to_principal_sqrt():
    # the OSRC spectrum: z = -lambda / k_eps^2, lambda >= 0, Im k_eps^2 > 0, so
    # 1 + z stays off the rotated cut (arg(1 + z) = theta - pi)
    ke = osrc.damped_wavenumber(10.0, 0.1)
    lam = np.array([0.0, 1.0, 30.0, 200.0, 1e3, 1e4])
    z = np.concatenate([-lam / ke ** 2, np.array([-0.5, 0.3, 2.0, -3.0 + 0.5j, -10 + 1j, 5j])])
    errs = [np.abs(osrc.pade_sqrt(z, N, np.pi / 3) - np.sqrt(1 + z + 0j)).max() for N in (2, 4, 8, 16, 32)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3   # slowest at the largest |z| (~86 here)
    # theta = 0 is the classical Pade expansion: exact on z = 0, accurate for small z
    C0, A, B = osrc.pade_coefficients(8, 0.0)
    assert abs(C0 - 1.0) < 1e-15
    small = np.array([0.01, -0.02, 0.05j])
    assert np.abs(osrc.pade_sqrt(small, 8, 0.0) - np.sqrt(1 + small)).max() < 1e-12


def test_damping_is_a_wavenumber():
    ke = osrc.damped_wavenumber(10.0, 0.1)
    assert abs(ke.real - 10.0) < 1e-15
    assert abs(ke.imag - 0.4 * 10 ** (1 / 3) * 0.1 ** (-2 / 3)) < 1e-12


def test_sphere_symbols_converge():
    k, reps, N, th = 2.0, 0.1, 4, np.pi / 3
    ke = osrc.damped_wavenumber(k, reps)
    errs = {}
    for lev in (2, 3):
        v, t = meshes.icosphere(lev)
        dtn, ntd, M = osrc.osrc_maps(v, t, k, reps, N, th)
        for l in (1, 2, 4):
            y = special.eval_legendre(l, v[:, 2])
            zz = -l * (l + 1) / ke ** 2
            ex_d = 1j * k * osrc.pade_sqrt([zz], N, th)[0]
            ex_n = osrc.pade_sqrt([zz], N, th)[0] / ((1j * k) * (1 + zz))
            got_d = (y @ M @ dtn @ y) / (y @ M @ y)
            got_n = (y @ M @ ntd @ y) / (y @ M @ y)
            errs[(lev, l)] = (abs(got_d - ex_d) / abs(ex_d), abs(got_n - ex_n) / abs(ex_n))
    for l in (1, 2, 4):
        assert max(errs[(3, l)]) < 0.02
        assert errs[(2, l)][0] / errs[(3, l)][0] > 3.0
        assert errs[(2, l)][1] / errs[(3, l)][1] > 3.0


def test_preconditioned_gmres_fewer_iterations_same_solution():
    prob = configs.config1()
    A = oracle.pmchwt_matrix(prob)
    b = oracle.rhs(prob, *oracle.plane_wave(prob.k0))
    P = osrc.preconditioner_matrix(prob, 0.1, 4, np.pi / 3)
    x, it, _ = oracle.gmres(lambda z: A @ z, b, restart=100, tol=1e-8)
    xp, itp, _ = oracle.gmres(lambda z: P @ (A @ z), P @ b, restart=100, tol=1e-8)
    assert itp < 0.75 * it, (it, itp)
    assert np.linalg.norm(xp - x) / np.linalg.norm(x) < 1e-6


def test_preconditioned_iterations_mesh_independent():
    its = []
    for level in (2, 3):
        prob = configs.sphere_problem(level, 6.0, 6.3, 1.05)
        A = oracle.pmchwt_matrix(prob)
        b = oracle.rhs(prob, *oracle.plane_wave(prob.k0))
        P = osrc.preconditioner_matrix(prob, 0.1, 4, np.pi / 3)
        _, it0, _ = oracle.gmres(lambda z: A @ z, b, restart=100, tol=1e-5)
        _, it1, _ = oracle.gmres(lambda z: P @ (A @ z), P @ b, restart=100, tol=1e-5)
        assert it1 < 0.7 * it0, (level, it0, it1)
        its.append(it1)
    assert abs(its[1] - its[0]) <= 3, its


def test_preconditioner_helps_high_contrast():
    prob = configs.sphere_problem(3, 10.0, 10.0 / 1.87, 1.9)
    A = oracle.pmchwt_matrix(prob)
    b = oracle.rhs(prob, *oracle.plane_wave(prob.k0))
    P = osrc.preconditioner_matrix(prob, 0.1, 4, np.pi / 3)
    _, it0, _ = oracle.gmres(lambda z: A @ z, b, restart=100, tol=1e-5)
    _, it1, _ = oracle.gmres(lambda z: P @ (A @ z), P @ b, restart=100, tol=1e-5)
    assert it1 < 0.6 * it0, (it0, it1)
