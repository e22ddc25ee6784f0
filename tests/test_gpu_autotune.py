"""GPU: the autotuned launch shapes keep parity with the FP64 oracle.

The tuner picks the pair kernel's test points per lane and trial splits (and
the GEMM's K-slice count) by timing; whichever shape it picks, the operator
must be the same to the FP32 tolerance.  Forced shapes go through the tuner's
cache file (one "key value" line per choice, last line wins), which also
covers the cache path; a fresh file makes the tuner search.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bem_inputs import configs, vectors

pytestmark = pytest.mark.gpu

APPLY_TOL = 1e-5


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c1():
    prob = configs.config1()
    return prob, oracle.pmchwt_matrix(prob)


def _problem(bem, prob, **kw):
    return bem.Problem.from_config(prob, **kw)


def test_tuned_pair_shapes_keep_parity(c1, tmp_path, monkeypatch):
    import paper_1910_01011_amd as bem
    prob, A = c1
    x = vectors.random_complex(prob.n_unknowns, seed=3)
    ref = A @ x
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("BEM_TUNE_CACHE", str(cache))
    P = _problem(bem, prob, autotune=True)
    tpl, ns = P.pair_launch_shape()
    err = _relerr(P.apply(x), ref)
    P.close()
    lines = cache.read_text().split()
    assert len(lines) == 2 and lines[0].startswith("pairs"), lines
    assert int(lines[1]) == 100 * tpl + ns
    print(f"searched shape tpl={tpl} n_split={ns}: rel err {err:.3e}")
    assert err <= APPLY_TOL
    key = lines[0]
    for forced in ((1, 1), (1, 8), (2, 4), (2, 16)):
        f2 = tmp_path / f"forced_{forced[0]}_{forced[1]}.txt"
        f2.write_text(f"{key} {100 * forced[0] + forced[1]}\n")
        monkeypatch.setenv("BEM_TUNE_CACHE", str(f2))
        P = _problem(bem, prob, autotune=True)
        assert P.pair_launch_shape() == forced
        y = P.apply(x)
        P.close()
        err = _relerr(y, ref)
        print(f"forced shape {forced}: rel err {err:.3e}")
        assert err <= APPLY_TOL


def test_tuned_gemm_slices_keep_parity(c1, tmp_path, monkeypatch):
    import paper_1910_01011_amd as bem
    prob, A = c1
    monkeypatch.setenv("BEM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    X = vectors.random_complex(prob.n_unknowns, seed=5, n_rhs=24)
    ref = X @ A.T
    for mode, kernel, tol in ((bem.BEM_ASSEMBLED_FP32, bem.BEM_APPLY_MFMA_FP32, 2e-5),
                              (bem.BEM_ASSEMBLED_SPLIT_BF16, bem.BEM_APPLY_MFMA_SPLIT_BF16, 2e-5)):
        P = _problem(bem, prob, mode=mode, autotune=True)
        Y1 = P.apply(X, kernel=kernel)
        Y2 = P.apply(X, kernel=kernel)     # cached choice
        P.close()
        err = _relerr(Y1, ref)
        print(f"mode {mode}: tuned GEMM rel err {err:.3e}")
        assert err <= tol
        assert np.array_equal(Y1, Y2)
    text = (tmp_path / "tune.txt").read_text()
    assert "bf16x3" in text and "f32" in text


def test_tuned_single_layer_shape_keeps_parity(tmp_path, monkeypatch):
    """The single-layer kernel's shape is timed on first use when autotuning is
    on.  On the 2,562-vertex sphere (several candidate shapes) the tuned
    operator equals the untuned one (the fused kernel's shape, parity-tested
    against the oracle's V_k0) to two FP32 summation orders, and repeated calls
    with the chosen shape are bitwise equal."""
    import paper_1910_01011_amd as bem
    monkeypatch.setenv("BEM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    prob = configs.sphere_problem(4, 4.0, 4.4, 1.0)
    nv = prob.domains[0].n_vertices
    x = vectors.random_complex(nv, seed=9)
    P = _problem(bem, prob, autotune=True)
    y1 = P.apply_single_layer(x)
    y2 = P.apply_single_layer(x)
    P.close()
    Q = _problem(bem, prob)
    y0 = Q.apply_single_layer(x)
    Q.close()
    assert np.array_equal(y1, y2)
    assert _relerr(y1, y0) <= 1e-6
