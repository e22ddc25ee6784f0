"""GPU parity of the assembled mode: dense complex64 PMCHWT matrix applied by a
GEMV (one right-hand side, FP64 accumulation) or by an MFMA GEMM (several
right-hand sides, FP32 MFMA or 3-term split BF16), against the FP64 oracle.

Tolerances: the dense entries are FP32 sums (relative error ~1e-7 each); the
GEMV accumulates in FP64, the FP32 GEMM in FP32 over K = 2n terms (error
~sqrt(K) * 2^-24 relative), so both stay well below 1e-5.  The split-BF16
product keeps A and X to 16 significant bits (hi + lo) and drops lo*lo:
~2^-16 = 1.5e-5 relative per product, so its raw apply is held to 1e-4 (the
solver's flexible-GMRES refinement recovers the FP32 accuracy).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bem_inputs import configs, vectors

pytestmark = pytest.mark.gpu


def _bem():
    import paper_1910_01011_amd as bem
    return bem


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c1():
    prob = configs.config1()
    return prob, oracle.pmchwt_matrix(prob)


@pytest.mark.parametrize("mode_name", ["BEM_ASSEMBLED_FP32", "BEM_ASSEMBLED_SPLIT_BF16"])
def test_assembled_single_rhs_gemv(c1, mode_name):
    prob, A = c1
    bem = _bem()
    P = bem.Problem.from_config(prob, mode=getattr(bem, mode_name))
    x = vectors.random_complex(prob.n_unknowns, seed=0)
    err = _relerr(P.apply(x), A @ x)
    print(f"{mode_name} GEMV rel err {err:.3e}")
    assert err <= 1e-5


def test_assembled_fp32_gemm_multi_rhs(c1):
    prob, A = c1
    bem = _bem()
    P = bem.Problem.from_config(prob, mode=bem.BEM_ASSEMBLED_FP32)
    X = vectors.random_complex(prob.n_unknowns, seed=1, n_rhs=5)
    Y = P.apply(X)
    errs = [_relerr(Y[r], A @ X[r]) for r in range(5)]
    print("FP32 MFMA GEMM rel errs", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5


def test_assembled_split_bf16_gemm_multi_rhs(c1):
    prob, A = c1
    bem = _bem()
    P = bem.Problem.from_config(prob, mode=bem.BEM_ASSEMBLED_SPLIT_BF16)
    X = vectors.random_complex(prob.n_unknowns, seed=2, n_rhs=70)   # 2R = 140: two n-tiles, ragged
    Y = P.apply(X)
    errs = [_relerr(Y[r], A @ X[r]) for r in range(70)]
    print(f"split-BF16 GEMM rel err max {max(errs):.2e} median {np.median(errs):.2e}")
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("kernel_name", ["BEM_APPLY_MFMA_SPLIT_BF16_W4", "BEM_APPLY_MFMA_SPLIT_BF16_W8"])
def test_split_bf16_tile_shapes(c1, kernel_name):
    """Both split-BF16 tile shapes (256 x 128 four-wave, 384 x 128 eight-wave;
    n = 1,284 leaves a ragged last m-tile for both) against the oracle, at R = 70
    (two n-tiles, the second ragged)."""
    prob, A = c1
    bem = _bem()
    P = bem.Problem.from_config(prob, mode=bem.BEM_ASSEMBLED_SPLIT_BF16)
    X = vectors.random_complex(prob.n_unknowns, seed=6, n_rhs=70)
    Y = P.apply(X, kernel=getattr(bem, kernel_name))
    errs = [_relerr(Y[r], A @ X[r]) for r in range(70)]
    print(f"{kernel_name} rel err max {max(errs):.2e}")
    assert max(errs) <= 1e-4
    # the FP32 MFMA GEMM of the same matrix agrees to the split's precision
    Yf = P.apply(X, kernel=bem.BEM_APPLY_MFMA_FP32)
    assert max(_relerr(Y[r], Yf[r]) for r in range(70)) <= 1e-4


def test_assembled_two_domains_matches_oracle():
    prob = configs.two_spheres(level=2)
    A = oracle.pmchwt_matrix(prob)
    bem = _bem()
    P = bem.Problem.from_config(prob, mode=bem.BEM_ASSEMBLED_FP32)
    X = vectors.random_complex(prob.n_unknowns, seed=3, n_rhs=3)
    Y = P.apply(X)
    assert max(_relerr(Y[r], A @ X[r]) for r in range(3)) <= 1e-5
    y1 = P.apply(X[0])
    assert _relerr(y1, A @ X[0]) <= 1e-5


def test_assembled_matches_on_the_fly_level4():
    """Dense and on-the-fly applies of the same operator agree (10,242-v would
    need 3.4 GB; level 4 keeps the test small) and match oracle rows."""
    prob = configs.sphere_problem(4, 10.0, 10.5, 1.05)
    bem = _bem()
    Pd = bem.Problem.from_config(prob, mode=bem.BEM_ASSEMBLED_FP32)
    Po = bem.Problem.from_config(prob)
    x = vectors.random_complex(prob.n_unknowns, seed=4)
    yd, yo = Pd.apply(x), Po.apply(x)
    assert _relerr(yd, yo) <= 2e-6
    rows = vectors.random_rows(prob.n_unknowns, 24, seed=5)
    R = oracle.pmchwt_rows(prob, rows)
    assert _relerr(yd[rows], R @ x) <= 1e-5
