"""GPU OSRC preconditioner against the oracle's dense preconditioner, and the
OSRC-preconditioned solve against the oracle's LU solution.

Tolerance of the preconditioner apply: the GPU solves its sparse systems by
COCG to a relative residual of 1e-10 (FP64), the oracle by dense LU; the
shifted systems have condition numbers of order 1e2-1e3 here, so the applied
preconditioner agrees to ~1e-8; the test requires 1e-7.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import osrc
from bem_inputs import configs, vectors

pytestmark = pytest.mark.gpu


def _bem():
    import paper_1910_01011_amd as bem
    return bem


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", ["config1", "two_spheres"])
def test_osrc_apply_matches_oracle(case):
    prob = configs.config1() if case == "config1" else configs.two_spheres(level=2)
    bem = _bem()
    P = bem.Problem.from_config(prob)
    opts = bem.solve_options(precond=bem.BEM_PRECOND_OSRC, n_pade=4, r_eps=0.1, theta=np.pi / 3)
    Pm = osrc.preconditioner_matrix(prob, 0.1, 4, np.pi / 3)
    Y = vectors.random_complex(prob.n_unknowns, seed=20, n_rhs=2)
    Z = P.precondition(Y, opts)
    for r in range(2):
        err = _relerr(Z[r], Pm @ Y[r])
        print(f"{case} OSRC apply rel err {err:.2e}")
        assert err <= 1e-7


def test_osrc_preconditioned_solve():
    """Both OSRC forms against the oracle's LU solution.  The right form stops on
    the unpreconditioned residual, so its true residual meets the tolerance
    (up to the FP32 operator's rounding in the recursive estimate); the left
    form (the paper's P A u = P b) stops on the preconditioned residual, which
    here sits below the true one."""
    prob = configs.config1()
    A = oracle.pmchwt_matrix(prob)
    b = oracle.rhs(prob, *oracle.plane_wave(prob.k0))
    u_ref = oracle.solve_lu(A, b)
    bem = _bem()
    P = bem.Problem.from_config(prob)
    u0, i0 = P.solve(b, bem.solve_options(tol=1e-8, restart=100, max_iter=400))
    for pc in (bem.BEM_PRECOND_OSRC, bem.BEM_PRECOND_OSRC_LEFT):
        u1, i1 = P.solve(b, bem.solve_options(tol=1e-8, restart=100, max_iter=400, precond=pc,
                                              n_pade=4, r_eps=0.1, theta=np.pi / 3))
        e1 = _relerr(u1, u_ref)
        print(f"plain {i0}, OSRC form {pc}: {i1}, error vs LU {e1:.2e}")
        assert i1[0]["converged"] and i1[0]["iterations"] < i0[0]["iterations"]
        assert e1 <= 1e-5
    for tol in (1e-5, 1e-6):
        u1, i1 = P.solve(b, bem.solve_options(tol=tol, restart=100, max_iter=400, precond=bem.BEM_PRECOND_OSRC,
                                              n_pade=4, r_eps=0.1, theta=np.pi / 3))
        res = _relerr(A @ np.ravel(u1), b)
        print(f"right OSRC at tol {tol:g}: {i1[0]}, oracle residual {res:.2e}")
        assert i1[0]["converged"] and i1[0]["rel_residual"] <= 1.1 * tol and res <= 2 * tol


def test_osrc_graph_replays_match_eager_launches(monkeypatch):
    """The batched COCG replays a captured graph of eight iterations until every
    block has converged.  The same kernels launched one by one (BEM_COCG_EAGER)
    must give bitwise the same preconditioned vectors, on every one of several
    applies with other work and synchronisations in between, on a single and a
    two-domain problem."""
    bem = _bem()
    for prob in (configs.config1(), configs.two_spheres(level=2)):
        P = bem.Problem.from_config(prob)
        opts = bem.solve_options(precond=bem.BEM_PRECOND_OSRC, n_pade=4, r_eps=0.1, theta=np.pi / 3, osrc_tol=1e-8)
        Y = vectors.random_complex(prob.n_unknowns, seed=24, n_rhs=3)
        graph = []
        for r in range(3):
            graph.append(P.precondition(Y[r], opts))
            P.apply(Y[r])                     # eager work between the replays
        monkeypatch.setenv("BEM_COCG_EAGER", "1")
        for r in range(3):
            assert np.array_equal(P.precondition(Y[r], opts), graph[r]), (prob.name, r)
        monkeypatch.delenv("BEM_COCG_EAGER")
        assert np.array_equal(P.precondition(Y[0], opts), graph[0])
        P.close()


def test_osrc_workspace_follows_parameters_and_vector_count():
    """The OSRC apply keeps its vectors, coefficients and captured COCG graphs on
    the problem and rebuilds them when the parameters or the number of vectors
    change.  Applies that alternate between two parameter sets and between one
    and two vectors give bitwise what a fresh problem gives for each, on both
    the host-pointer and the device-pointer paths."""
    import torch
    bem = _bem()
    prob = configs.two_spheres(level=2)
    a = bem.solve_options(precond=bem.BEM_PRECOND_OSRC, n_pade=4, r_eps=0.1, theta=np.pi / 3, osrc_tol=1e-8)
    b = bem.solve_options(precond=bem.BEM_PRECOND_OSRC, n_pade=2, r_eps=0.3, theta=np.pi / 4, osrc_tol=1e-6)
    Y = vectors.random_complex(prob.n_unknowns, seed=31, n_rhs=2)

    def fresh(opts, y):
        F = bem.Problem.from_config(prob)
        z = F.precondition(y, opts)
        F.close()
        return z

    ref = {("a", 1): fresh(a, Y[0]), ("b", 1): fresh(b, Y[0]), ("a", 2): fresh(a, Y), ("b", 2): fresh(b, Y)}
    P = bem.Problem.from_config(prob)
    for key in (("a", 1), ("b", 1), ("a", 1), ("a", 2), ("b", 2), ("a", 1), ("b", 2)):
        opts = a if key[0] == "a" else b
        z = P.precondition(Y[0] if key[1] == 1 else Y, opts)
        assert np.array_equal(z, ref[key]), key
    P.close()
    D = bem.Problem.from_config(prob, device=True)
    for key in (("b", 2), ("a", 1), ("b", 2)):
        opts = a if key[0] == "a" else b
        y = torch.from_numpy(Y[0] if key[1] == 1 else Y).cuda()
        z = D.precondition(y, opts).cpu().numpy()
        assert np.array_equal(z, ref[key]), ("device", key)
    D.close()


def test_osrc_apply_rows_longer_than_one_load_step():
    """The sparse product of the COCG loads nine entries of a row at a time
    (from a slot-major copy of each row's first nine) and continues from the
    CSR for longer rows.  A capsule (pole rows of 17 entries) beside a box
    (rows of exactly nine) against the oracle's dense preconditioner."""
    from bem_inputs import meshes
    from bem_inputs.configs import Domain, Problem
    vc, tc = meshes.capsule(radius=0.25, length=1.0, h=0.1, axis=1)
    vb, tb = meshes.box((0.6, -0.5, -0.2), (1.2, 0.1, 0.2), 0.1)
    prob = Problem(domains=[Domain(vc, tc, 3.3 + 0.05j, 1.2, "capsule"), Domain(vb, tb, 2.8, 0.9, "box")],
                   k0=3.0, name="capsule_box")
    lengths = []
    for v, t in ((vc, tc), (vb, tb)):
        adj = [set() for _ in range(len(v))]
        for tri in t:
            for a in tri:
                adj[a].update(int(b) for b in tri)
        lengths += [len(s) for s in adj]
    assert max(lengths) > 9 and 9 in lengths
    bem = _bem()
    P = bem.Problem.from_config(prob)
    opts = bem.solve_options(precond=bem.BEM_PRECOND_OSRC, n_pade=4, r_eps=0.1, theta=np.pi / 3)
    Pm = osrc.preconditioner_matrix(prob, 0.1, 4, np.pi / 3)
    Y = vectors.random_complex(prob.n_unknowns, seed=33, n_rhs=2)
    Z = P.precondition(Y, opts)
    for r in range(2):
        err = _relerr(Z[r], Pm @ Y[r])
        print(f"capsule and box OSRC apply rel err {err:.2e}")
        assert err <= 1e-7
    P.close()
