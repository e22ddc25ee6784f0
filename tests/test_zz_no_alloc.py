"""The allocation-free apply (bem_apply_noalloc) against bem_apply.

Same kernels and summation order with the scratch in the library's file-scope
device array, so the outputs must be bitwise equal; both are also checked
against the FP64 oracle to the apply tolerance of the parity tests (1e-5).
Two calls in a row, the second on a smaller problem, so the second runs on
what the first left in the shared array.  The call must not change the
device's free memory (no allocation), and problems whose scratch exceeds the
array are rejected.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bem_inputs import configs, meshes, vectors

pytestmark = pytest.mark.gpu


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _two_sphere_problem():
    """Two disjoint spheres of 2,562 and 642 vertices (two interior passes)."""
    v1, t1 = meshes.icosphere(4, 1.0, (-1.6, 0.0, 0.0))
    v2, t2 = meshes.icosphere(3, 0.5, (1.2, 0.3, 0.0))
    return configs.Problem([configs.Domain(v1, t1, complex(3.3), 1.2, "a"),
                            configs.Domain(v2, t2, complex(2.6, 0.1), 0.8, "b")], complex(3.0), 1.0, "two_spheres_3204")


def test_noalloc_apply_matches_apply_twice_shrinking():
    import torch
    import paper_1910_01011_amd as bem
    torch.cuda.set_device(0)
    big = _two_sphere_problem()
    small = configs.config1()
    for step, (prob, n_rhs, seed) in enumerate(((big, 2, 31), (small, 1, 32))):
        print(f"noalloc step {step}: {prob.name}, {prob.n_unknowns} unknowns, {n_rhs} rhs", flush=True)
        P = bem.Problem.from_config(prob, device=True)
        X = vectors.random_complex(prob.n_unknowns, seed=seed, n_rhs=n_rhs)
        x = torch.from_numpy(X).cuda()
        y_ref = P.apply(x)
        torch.cuda.synchronize()
        y = torch.empty_like(x)
        y.fill_(complex(np.nan, np.nan))
        P.apply_noalloc(x, out=y)        # first call on this device looks the scratch up
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        y.fill_(complex(np.nan, np.nan))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        P.apply_noalloc(x, out=y)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        assert torch.equal(y, y_ref)
        A = oracle.pmchwt_matrix(prob)
        Y = y.cpu().numpy().reshape(n_rhs, -1)
        for r in range(n_rhs):
            err = _relerr(Y[r], A @ X.reshape(n_rhs, -1)[r])
            print(f"  rhs {r}: rel err vs oracle {err:.2e}", flush=True)
            assert err <= 1e-5
        P.close()


def test_noalloc_rejects_what_it_cannot_serve():
    import torch
    import paper_1910_01011_amd as bem
    prob = configs.config1()
    P = bem.Problem.from_config(prob)                          # host vectors: rejected by the C entry point
    xh = np.zeros(prob.n_unknowns, dtype=np.complex128)
    yh = np.empty_like(xh)
    assert bem._L.bem_apply_noalloc(P._h, xh.ctypes.data, yh.ctypes.data, 1) == bem.BEM_ERR_INVALID_ARG
    assert b"device vectors" in bem._L.bem_last_error()
    P.close()
    Pa = bem.Problem.from_config(prob, device=True, mode=bem.BEM_ASSEMBLED_FP32)
    x = torch.zeros(prob.n_unknowns, dtype=torch.complex128, device="cuda")
    with pytest.raises(bem.BemError) as e:
        Pa.apply_noalloc(x)
    assert e.value.status == bem.BEM_ERR_INVALID_ARG
    Pa.close()
    # the 40,962-vertex sphere needs about 700 MB of scratch (8 splits)
    big = configs.sphere_problem(6, 2.0, 2.2, 1.0)
    Pb = bem.Problem.from_config(big, device=True)
    xb = torch.zeros(big.n_unknowns, dtype=torch.complex128, device="cuda")
    with pytest.raises(bem.BemError) as e:
        Pb.apply_noalloc(xb)
    assert e.value.status == bem.BEM_ERR_UNSUPPORTED, str(e.value)
    Pb.close()
