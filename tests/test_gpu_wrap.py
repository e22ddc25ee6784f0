"""GPU parity at phases beyond the hardware sine's own range reduction.

v_sin / v_cos take their argument in revolutions and reduce it themselves only
below 256 revolutions; the pair kernels add the explicit reduction
ph - rint(ph) when a problem's largest phase (bounding-box diagonal times the
largest wavenumber, over 2 pi) reaches 128 revolutions.  The 642-vertex unit
sphere at k0 = 480, k1 = 500 has phases up to 2 sqrt(3) * 500 / (2 pi) = 276
revolutions, so the on-the-fly apply, the single-layer apply and the dense
assembly all run their reduced form here (no other test reaches 128).

Tolerance: the FP32 phase k r carries a relative rounding error of a few
2^-24 (coordinates, r^2, rsq): up to about 1730 rad * 3e-7 = 5e-4 rad at the
largest distances, which the sums over many pairs average down.  Required
<= 2e-3; a phase left unreduced past 256 revolutions gives errors of order one.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bem_inputs import configs, vectors

pytestmark = pytest.mark.gpu

TOL = 2e-3


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def high_k():
    prob = configs.sphere_problem(3, 480.0, 500.0, 1.0, name="sphere642_k480")
    d = prob.domains[0]
    diag = float(np.linalg.norm(d.vertices.max(axis=0) - d.vertices.min(axis=0)))
    assert diag * 500.0 / (2 * np.pi) > 256.0   # past the hardware reduction
    return prob, oracle.pmchwt_matrix(prob), oracle.single_layer_matrix(prob)


def test_reduced_phase_apply_and_assembly(high_k):
    import paper_1910_01011_amd as bem
    prob, A, V = high_k
    X = vectors.random_complex(prob.n_unknowns, seed=31, n_rhs=2)
    P = bem.Problem.from_config(prob)
    Y = P.apply(X)
    for r in range(2):
        err = _relerr(Y[r], A @ X[r])
        print(f"on-the-fly apply rhs {r}: rel err {err:.3e}", flush=True)
        assert err <= TOL
    xs = vectors.random_complex(V.shape[0], seed=32)
    err = _relerr(P.apply_single_layer(xs), V @ xs)
    print(f"single-layer apply: rel err {err:.3e}", flush=True)
    assert err <= TOL
    P.close()
    Pa = bem.Problem.from_config(prob, mode=bem.BEM_ASSEMBLED_FP32)
    err = _relerr(Pa.apply(X[0], kernel=bem.BEM_APPLY_GEMV), A @ X[0])
    print(f"assembled GEMV apply: rel err {err:.3e}", flush=True)
    assert err <= TOL
    Pa.close()
