"""Synthetic mesh generators: closed, consistently oriented surfaces of the
stated sizes (host logic only; no boundary-element arithmetic)."""
from __future__ import annotations

import numpy as np
import pytest

from bem_inputs import configs, meshes


def _closed_and_oriented(v, t):
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    directed = set(map(tuple, e))
    # every directed edge once, and its reverse present: a closed 2-manifold
    # with consistent orientation
    return len(directed) == len(e) and all((b, a) in directed for a, b in e)


def _signed_volume(v, t):
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


@pytest.mark.parametrize("freq", [1, 2, 3, 5, 8, 13])
def test_geodesic_sphere_counts_closed_outward(freq):
    v, t = meshes.geodesic_sphere(freq)
    assert len(v) == 10 * freq ** 2 + 2 and len(t) == 20 * freq ** 2
    assert _closed_and_oriented(v, t)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    vol = _signed_volume(v, t)
    assert 0 < vol < 4.0 / 3.0 * np.pi          # inscribed polyhedron, outward normals
    if freq >= 8:
        assert vol > 0.98 * 4.0 / 3.0 * np.pi


def test_geodesic_matches_icosphere_counts_at_powers_of_two():
    for level in range(4):
        vi, ti = meshes.icosphere(level)
        vg, tg = meshes.geodesic_sphere(2 ** level)
        assert len(vi) == len(vg) and len(ti) == len(tg)


def test_geodesic_shell_inner_surface_reversed():
    v, t = meshes.geodesic_shell(4, (1.0, 1.0, 1.0), (2.0, 2.0, 2.0))
    assert _closed_and_oriented(v, t)
    # outer volume minus inner volume: the shell material's volume
    expect = 4.0 / 3.0 * np.pi * (8.0 - 1.0)
    assert 0.8 * expect < _signed_volume(v, t) < expect


def test_kidney_stream_sizes_follow_h_continuously():
    items = configs.serving_stream(5.0, 12, 5005, 6005)
    nv = [sum(d.n_vertices for d in it["problem"].domains) for it in items]
    assert all(2000 <= n <= 40000 for n in nv)
    assert len(set(nv)) >= 6                      # not quantised to a few levels
    for it, n in zip(items, nv):
        assert n == configs.kidney_vertices(it["freq"])
        # element size within the requested elements-per-wavelength rule
        h = min(meshes.mesh_size(d.vertices, d.triangles) for d in it["problem"].domains)
        assert h <= 0.941 / it["f_rel"] / 4.0 * 1.05
