"""Host-side behaviour of the HIP library that needs no GPU.

The shared library loads without a device; argument and mesh validation run
before any HIP call, so these error paths are exercised on the CPU.
"""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

from bem_inputs import configs, meshes

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bem():
    return pytest.importorskip("paper_1910_01011_amd")


def test_library_exports_every_declared_symbol():
    bem = _bem()
    header = open(os.path.join(ROOT, "include", "bem.h")).read()
    declared = set(re.findall(r"^\s*(?:bem_status|int64_t|void|const char \*)\s*(bem_\w+)\s*\(", header, re.M))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(bem._L, name), name
    assert declared == set(bem.EXPORTED)


def _dom(v, t, k=2.0, rho=1.0):
    return configs.Domain(np.asarray(v, dtype=np.float64), np.asarray(t, dtype=np.int32), complex(k), rho)


def _expect(status, domains, k0=2.0, rho0=1.0):
    bem = _bem()
    with pytest.raises(bem.BemError) as e:
        bem.Problem(domains, k0, rho0)
    assert e.value.status == status, str(e.value)


def test_argument_errors():
    bem = _bem()
    v, t = meshes.icosphere(1)
    _expect(bem.BEM_ERR_INVALID_ARG, [])
    _expect(bem.BEM_ERR_INVALID_ARG, [_dom(v, t)], k0=complex(2.0, -0.1))
    _expect(bem.BEM_ERR_INVALID_ARG, [_dom(v, t)], rho0=0.0)
    _expect(bem.BEM_ERR_INVALID_ARG, [_dom(v, t, rho=-1.0)])
    _expect(bem.BEM_ERR_INVALID_ARG, [_dom(v, t, k=complex(2.0, -1.0))])
    vv = v.copy()
    vv[3, 1] = np.nan
    _expect(bem.BEM_ERR_INVALID_ARG, [_dom(vv, t)])
    with pytest.raises(bem.BemError) as e:
        bem.Problem([_dom(v, t)], 2.0, 1.0, ss_order=40)
    assert e.value.status == bem.BEM_ERR_INVALID_ARG


def test_entry_points_reject_null_handles():
    """Argument checks that run before any device call."""
    import ctypes
    bem = _bem()
    L = bem._L
    info = bem.bem_hmatrix_info()
    assert L.bem_hmatrix_build(None, 1e-4, 64, 1.0, ctypes.byref(info)) == bem.BEM_ERR_INVALID_ARG
    assert L.bem_apply_single_layer(None, None, None, 1) == bem.BEM_ERR_INVALID_ARG
    assert L.bem_apply_with(None, None, None, 1, bem.BEM_APPLY_HMATRIX) == bem.BEM_ERR_INVALID_ARG
    assert L.bem_evaluate_field(None, None, None, None, 0, None, None) == bem.BEM_ERR_INVALID_ARG


def test_mesh_errors():
    bem = _bem()
    v, t = meshes.icosphere(1)
    _expect(bem.BEM_ERR_MESH, [_dom(v, t[:, ::-1])])                    # inward normals
    tf = t.copy()
    tf[5] = tf[5, ::-1]
    _expect(bem.BEM_ERR_MESH, [_dom(v, tf)])                           # one flipped triangle
    _expect(bem.BEM_ERR_MESH, [_dom(v, t[1:])])                        # open surface
    tb = t.copy()
    tb[0, 0] = v.shape[0]
    _expect(bem.BEM_ERR_MESH, [_dom(v, tb)])                           # index out of range
    tr = t.copy()
    tr[0, 1] = tr[0, 0]
    _expect(bem.BEM_ERR_MESH, [_dom(v, tr)])                           # repeated vertex
    vz = v.copy()
    a, b, c = t[0]
    vz[c] = 0.5 * (vz[a] + vz[b])
    _expect(bem.BEM_ERR_MESH, [_dom(vz, t)])                           # zero-area triangle
    _expect(bem.BEM_ERR_MESH, [_dom(v, t), _dom(v.copy(), t.copy())])  # touching domains


def test_unsupported_options():
    bem = _bem()
    v, t = meshes.icosphere(1)
    with pytest.raises(bem.BemError) as e:
        bem.Problem([_dom(v, t)], 2.0, 1.0, mode=bem.BEM_ASSEMBLED_SPLIT_BF16 + 7)
    assert e.value.status in (bem.BEM_ERR_UNSUPPORTED, bem.BEM_ERR_INVALID_ARG)


def test_footprint_grows_with_rhs_and_restart():
    bem = _bem()
    prob = configs.config1()
    a = bem.footprint_bytes(prob.domains, 1, 30)
    b = bem.footprint_bytes(prob.domains, 8, 30)
    c = bem.footprint_bytes(prob.domains, 8, 100)
    assert 0 < a < b < c


@pytest.mark.parametrize("cname", ["bem_solve_opts", "bem_solve_info", "bem_assemble_opts", "bem_hmatrix_info"])
def test_binding_structs_follow_the_header(cname):
    """The ctypes structures of the binding list the C structs' fields in the
    header's order (names as declared), so the two cannot drift apart."""
    bem = _bem()
    header = open(os.path.join(ROOT, "include", "bem.h")).read()
    structs = dict((name, body) for body, name in re.findall(r"typedef struct\s*\{([^{}]*)\}\s*(\w+)\s*;", header))
    assert cname in structs, cname
    body = re.sub(r"/\*.*?\*/", "", structs[cname], flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            names.append(re.findall(r"\**(\w+)\s*$", part.strip())[0])
    assert [f[0] for f in getattr(bem, cname)._fields_] == names


@pytest.mark.parametrize("leaf,eta", [(8, 2.0), (8, 1.0), (16, 2.0), (16, 4.0)])
def test_hmatrix_tree_keeps_touching_pairs_out_of_lowrank_blocks(leaf, eta):
    """Every vertex pair that the singular pass corrects (touching triangles of
    one boundary) lies in a dense block of the hierarchical matrix: the
    clusters' boxes bound the supports of their basis functions, so such pairs
    are at distance 0 and never admissible.  Checked on the host on the trees
    the build uses, at leaf sizes and eta values that admit many blocks."""
    bem = _bem()
    for prob in (configs.config1(), configs.two_spheres()):
        plan = bem.hmatrix_plan(prob.domains, leaf_vertices=leaf, eta=eta)
        assert plan["n_admissible"] > 0 and plan["n_touching"] > 0, plan
        assert plan["n_touching_admissible"] == 0, (prob.name, leaf, eta, plan)


def test_hmatrix_plan_errors():
    bem = _bem()
    v, t = meshes.icosphere(1)
    with pytest.raises(bem.BemError) as e:
        bem.hmatrix_plan([_dom(v, t)], leaf_vertices=4)
    assert e.value.status == bem.BEM_ERR_INVALID_ARG
    tt = t.copy()
    tt[0, 0] = v.shape[0] + 3
    with pytest.raises(bem.BemError) as e:
        bem.hmatrix_plan([_dom(v, tt)], leaf_vertices=8)
    assert e.value.status == bem.BEM_ERR_MESH
