"""Full matrix capture on the GPU against the oracle.

* Many fields (more than four): the field is evaluated as rows of the
  representation formula times the traces (rows + dense product), FP64 on both
  sides with different summation orders: relative error <= 1e-10.
* Planning: every element's forward problem solved as one block (GMRES to
  1e-9) and the transfer matrix at control points against the oracle's LU
  solutions: relative error <= 1e-6 (solve error ~ cond(A) x 1e-9).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bem_inputs import configs, pistons

pytestmark = pytest.mark.gpu


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _points():
    rng = np.random.default_rng(11)
    d = rng.standard_normal((30, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.concatenate([rng.uniform(0.2, 0.6, 15), rng.uniform(1.5, 3.0, 15)])
    return d * r[:, None]


@pytest.mark.parametrize("n_dirs", [2, 6])
def test_plane_wave_fields_match_oracle(n_dirs):
    """n_dirs = 2 takes the per-point path, 6 the rows + product path."""
    import paper_1910_01011_amd as bem
    prob = configs.config1()
    A = oracle.pmchwt_matrix(prob)
    rng = np.random.default_rng(3)
    dirs = rng.standard_normal((n_dirs, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = _points()
    P = bem.Problem.from_config(prob)
    U, F = [], []
    for d in dirs:
        p, dp = oracle.plane_wave(prob.k0, d)
        u = oracle.solve_lu(A, oracle.rhs(prob, p, dp))
        U.append(u)
        F.append(oracle.field(prob, u, pts, p)[0])
    f, reg = P.evaluate_field(np.array(U), pts, bem.Incident.plane_waves(dirs))
    ref_reg = oracle.field(prob, U[0], pts, None)[1]
    assert np.array_equal(reg, ref_reg)
    for i in range(n_dirs):
        err = _relerr(f[i], F[i])
        print(f"{n_dirs} fields, field {i}: rel err {err:.2e}", flush=True)
        assert err <= 1e-10
    P.close()


def test_planning_transfer_matrix_matches_oracle():
    import paper_1910_01011_amd as bem
    from paper_1910_01011_amd import planning
    prob = configs.config1()
    A = oracle.pmchwt_matrix(prob)
    c, nrm, a = pistons.bowl_array(n=12, focal=6.0, aperture=6.0, piston_diameter=0.6, min_spacing=0.7,
                                   focus=(0.0, 0.0, 0.0), seed=5)
    focus = np.array([0.0, 0.0, 0.3])
    spare = np.array([[0.0, 0.0, -1.4], [0.4, 0.0, -1.3], [-0.4, 0.2, -1.3]])
    P = bem.Problem.from_config(prob, device=True)
    opts = bem.solve_options(tol=1e-9, restart=100, max_iter=500)
    res = planning.plan(P, c, nrm, a, focus, spare, 0.3, opts)
    P.close()
    assert all(i["converged"] for i in res["solve_info"])
    pts = np.vstack([focus[None], spare])
    H_ref = np.zeros((pts.shape[0], len(c)), dtype=np.complex128)
    for e in range(len(c)):
        amp = np.zeros(len(c))
        amp[e] = 1.0
        p, dp = oracle.piston_field(prob.k0, c, nrm, a, amp)
        u = oracle.solve_lu(A, oracle.rhs(prob, p, dp))
        H_ref[:, e] = oracle.field(prob, u, pts, p)[0]
    err = _relerr(res["H"], H_ref)
    print(f"transfer matrix rel err {err:.2e}; phase conjugation ratio {res['phase_conjugation']['ratio']:.3f}, "
          f"sparing ratio {res['sparing']['ratio']:.3f}", flush=True)
    assert err <= 1e-6
    assert res["sparing"]["met"] and res["sparing"]["ratio"] <= 0.3 * (1 + 1e-9)
    assert np.isclose(np.max(np.abs(res["sparing"]["a"])), 1.0)


def test_many_fields_in_point_chunks_and_empty_inputs(monkeypatch):
    """The rows + product path over several ragged chunks of points (7 points
    per chunk) gives the single-chunk result; zero points and zero right-hand
    sides are accepted."""
    import paper_1910_01011_amd as bem
    prob = configs.two_spheres()
    rng = np.random.default_rng(4)
    U = rng.standard_normal((5, prob.n_unknowns)) + 1j * rng.standard_normal((5, prob.n_unknowns))
    pts = _points() + np.array([0.2, 0.1, 0.0])
    dirs = np.eye(3)[[0, 1, 2, 0, 1]]
    P = bem.Problem.from_config(prob)
    inc = bem.Incident.plane_waves(dirs)
    f1, r1 = P.evaluate_field(U, pts, inc)
    monkeypatch.setenv("BEM_FIELD_CHUNK_POINTS", "7")
    f2, r2 = P.evaluate_field(U, pts, inc)
    monkeypatch.delenv("BEM_FIELD_CHUNK_POINTS")
    assert np.array_equal(r1, r2)
    assert np.array_equal(f1, f2)
    ref = np.array([oracle.field(prob, U[i], pts, oracle.plane_wave(prob.k0, dirs[i])[0])[0] for i in range(5)])
    assert _relerr(f1, ref) <= 1e-10
    f0, r0 = P.evaluate_field(U, np.zeros((0, 3)), inc)
    assert f0.shape == (5, 0) and r0.shape == (0,)
    y0 = P.apply_single_layer(np.zeros((0, prob.n_unknowns // 2), dtype=np.complex128))
    assert y0.shape == (0, prob.n_unknowns // 2)
    P.close()


def test_field_direct_path_two_domains_matches_oracle():
    """The per-point path (at most four fields: each point's source triangles
    split over several threads, the partial sums added in split order) on two
    domains, with points outside and inside each of them, against the oracle's
    field and region codes."""
    import paper_1910_01011_amd as bem
    prob = configs.two_spheres()
    rng = np.random.default_rng(12)

    def ball(c, r, n):
        d = rng.standard_normal((n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        return np.asarray(c) + d * rng.uniform(0.0, r, n)[:, None]

    pts = np.concatenate([ball((-1.0, 0.0, 0.0), 0.4, 10), ball((1.0, 0.3, 0.2), 0.25, 10),
                          ball((0.0, 0.0, 0.0), 3.0, 40)])
    U = rng.standard_normal((2, prob.n_unknowns)) + 1j * rng.standard_normal((2, prob.n_unknowns))
    dirs = np.eye(3)[[2, 0]]
    P = bem.Problem.from_config(prob)
    f, r = P.evaluate_field(U, pts, bem.Incident.plane_waves(dirs))
    P.close()
    refs = [oracle.field(prob, U[i], pts, oracle.plane_wave(prob.k0, dirs[i])[0]) for i in range(2)]
    assert np.array_equal(r, refs[0][1])
    assert {0, 1, 2} <= set(r.tolist())   # outside, inside each domain (and near the boundaries: -1)
    assert _relerr(f, np.array([ref[0] for ref in refs])) <= 1e-10
