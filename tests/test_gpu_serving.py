"""Serving loop on the GPU: each request's result is bitwise the same alone and
in a mix of concurrent requests, admission respects the HBM budget, and the
piston right-hand sides match the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bem_inputs import configs, pistons

pytestmark = pytest.mark.gpu


def _bem():
    import paper_1910_01011_amd as bem
    return bem


def _requests(bem, serving):
    c, n, a = pistons.bowl_array(256, 27.0, 20.0, axis=(1.0, -1.0, 0.0))
    base = configs.kidney(1.0, level=3)
    out = []
    specs = [(0.6, 1, bem.BEM_OTF, bem.BEM_PREC_FP32),
             (0.8, 5, bem.BEM_ASSEMBLED_SPLIT_BF16, bem.BEM_PREC_SPLIT_BF16_FGMRES),
             (0.7, 3, bem.BEM_ASSEMBLED_FP32, bem.BEM_PREC_FP32_MFMA_FGMRES),
             (0.9, 2, bem.BEM_OTF, bem.BEM_PREC_FP32),
             (0.5, 1, bem.BEM_ASSEMBLED_FP32, bem.BEM_PREC_FP32)]
    for rid, (f, R, mode, prec) in enumerate(specs):
        k0 = 2 * np.pi * f
        doms = [configs.Domain(d.vertices, d.triangles, complex(k0 / s), d.rho) for d, s in zip(base.domains, (1.04, 0.941))]
        sel = np.arange(R) * 7 + rid
        inc = bem.Incident.pistons(c[sel], n[sel], a, 1.0, np.arange(R))
        out.append(serving.Request(rid, doms, complex(k0), inc, mode=mode, precision=prec, tol=1e-6,
                                   restart=30 if mode != bem.BEM_OTF else 100, max_iter=300))
    return out


def test_result_is_the_same_alone_and_in_a_mix():
    """Five requests (two on the fly, three assembled: split-BF16 and FP32-MFMA
    flexible GMRES, FP32 GEMV GMRES) alone and all together.  In the mix their
    operator applies are launched together: the two on-the-fly requests' pair
    kernels share grouped launches.  Every result is bitwise the same."""
    bem = _bem()
    from paper_1910_01011_amd import serving
    reqs = _requests(bem, serving)
    alone = {}
    for r in reqs:
        srv = serving.Server(max_inflight=1)
        res = srv.run([r])
        alone[r.rid] = res[0]
        assert srv.last_batch_stats["multi_problem_launches"] == 0
    # a long gather window: the requests in a solve step in lockstep, so the
    # two on-the-fly requests' applies meet in the same dispatches
    srv = serving.Server(max_inflight=5, batch_window_s=0.05)
    mix = srv.run(reqs)
    stats = srv.last_batch_stats
    print(serving.summarize(mix))
    print(f"batch: {stats}")
    for res in mix:
        assert all(i["converged"] for i in res.info), res.info
        assert np.array_equal(res.u, alone[res.rid].u), res.rid
    # the requests were admitted together, and the device work of the two
    # on-the-fly requests ran in shared launches
    assert max(r.admitted for r in mix) < min(r.finished for r in mix)
    assert stats["multi_problem_launches"] > 0 and stats["max_problems_per_launch"] == 2
    assert stats["applies"] > stats["dispatches"]


def test_admission_waits_for_memory():
    bem = _bem()
    from paper_1910_01011_amd import serving
    reqs = _requests(bem, serving)[:2]
    for r in reqs:
        r.arrival = 0.0
    fp = [serving.footprint(r) for r in reqs]
    res = serving.Server(hbm_budget_bytes=max(fp) + min(fp) // 2, max_inflight=4).run(reqs)
    first, second = sorted(res, key=lambda r: r.admitted)
    assert second.admitted >= first.finished - 1e-3


def test_piston_rhs_matches_oracle():
    bem = _bem()
    prob = configs.config1()
    c, n, a = pistons.bowl_array(16, 6.0, 4.0, piston_diameter=0.5, min_spacing=0.6, focus=(0, 0, 0),
                                 axis=(0.0, 0.0, 1.0), seed=3)
    P = bem.Problem.from_config(prob)
    amps = np.exp(1j * np.linspace(0, 2, 16))
    inc = bem.Incident.pistons(c, n, a, amps, np.zeros(16, dtype=int))
    b = P.rhs(inc)
    ref = oracle.rhs(prob, *oracle.piston_field(prob.k0, c, n, a, amps))
    assert np.linalg.norm(b[0] - ref) / np.linalg.norm(ref) < 1e-12
