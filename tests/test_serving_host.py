"""Host logic of the serving loop (no GPU): mode policy and request building."""
from __future__ import annotations

import numpy as np

from bem_inputs import configs


def test_choose_mode_policy():
    import paper_1910_01011_amd as bem
    from paper_1910_01011_amd import serving
    free = 250 << 30
    # dense matrix 32 N_V^2 bytes over a quarter of free HBM: on the fly
    assert serving.choose_mode(60000, 64, free) == (bem.BEM_OTF, bem.BEM_PREC_FP32)
    # fits: GEMV per right-hand side for one or two, split-BF16 block FGMRES otherwise
    assert serving.choose_mode(30000, 1, free) == (bem.BEM_ASSEMBLED_FP32, bem.BEM_PREC_FP32)
    assert serving.choose_mode(30000, 2, free) == (bem.BEM_ASSEMBLED_FP32, bem.BEM_PREC_FP32)
    assert serving.choose_mode(30000, 3, free) == (bem.BEM_ASSEMBLED_SPLIT_BF16, bem.BEM_PREC_SPLIT_BF16_FGMRES)


def test_requests_from_stream_one_rhs_per_piston():
    from paper_1910_01011_amd import serving
    items = configs.serving_stream(10.0, 4, 5010, 6010)
    reqs = serving.requests_from_stream(items, 250 << 30)
    assert [r.arrival for r in reqs] == sorted(r.arrival for r in reqs)
    for it, r in zip(items, reqs):
        assert r.incident.n_fields == len(it["piston_centres"])
        assert r.restart == (100 if r.precision == 0 else 30)
        assert np.isclose(r.k0, it["problem"].k0)
