"""Closed triangular surface meshes used as synthetic inputs.

Every mesh is a pair ``(vertices, triangles)``: ``vertices`` is float64 [n_v, 3],
``triangles`` is int32 [n_t, 3] with 0-based vertex indices.  Triangles are
ordered counter-clockwise when seen from the side the unit normal points to,
and the normal points out of the domain the surface bounds (the convention of
the traces in the paper's model section: n^j points from Omega^j into the
exterior).  For a shell domain the inner surface is reversed so that its normal
points into the cavity, i.e. still out of the shell material.

These generators contain no boundary-element arithmetic: they only place
vertices and connect them.  Both the oracle and the GPU library consume them.
"""
from __future__ import annotations

import numpy as np


def _orient_outward(v: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Flip all triangles if the signed enclosed volume is negative."""
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    if vol < 0:
        t = t[:, [0, 2, 1]]
    return np.ascontiguousarray(t, dtype=np.int32)


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron inscribed in the unit sphere (12 v, 20 t)."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
         [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
         [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    return v, _orient_outward(v, t)


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Icosahedron refined ``level`` times by 1->4 splitting.

    New vertices are projected onto the sphere after every split.  Sizes:
    10*4**level + 2 vertices and 20*4**level triangles (level 3: 642/1280,
    level 5: 10242/20480).
    """
    v, t = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                m = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
                m /= np.linalg.norm(m)
                verts.append(tuple(m))
                k = len(verts) - 1
                cache[key] = k
            return k

        nt = []
        for a, b, c in t:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nt += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        t = np.asarray(nt, dtype=np.int32)
    v = np.asarray(verts, dtype=np.float64) * radius + np.asarray(center, dtype=np.float64)
    return v, _orient_outward(v, t)


def ellipsoid(level: int, semi_axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0)):
    """Icosphere scaled along the coordinate axes."""
    v, t = icosphere(level)
    v = v * np.asarray(semi_axes, dtype=np.float64) + np.asarray(center, dtype=np.float64)
    return v, _orient_outward(v, t)


def tetrahedron(scale: float = 1.0):
    """A non-regular tetrahedron: every pair of its faces shares an edge."""
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.3, 0.25, 0.8]]) * scale
    t = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], dtype=np.int32)
    return v, _orient_outward(v, t)


def bipyramid(scale: float = 1.0):
    """Triangular bipyramid (5 v, 6 t).

    Every pair of faces touches: each face shares an edge or exactly one vertex
    with every other face, so a Galerkin operator on it has no far pairs.
    """
    v = np.array([[1.0, 0.0, 0.05], [-0.45, 0.85, -0.05], [-0.5, -0.8, 0.0],
                  [0.05, 0.02, 1.1], [-0.03, 0.05, -0.9]]) * scale
    t = np.array([[0, 1, 3], [1, 2, 3], [2, 0, 3], [1, 0, 4], [2, 1, 4], [0, 2, 4]], dtype=np.int32)
    return v, _orient_outward(v, t)


def box(lo, hi, h: float):
    """Axis-aligned box surface with a conforming structured triangulation.

    Each face is split into a grid of ceil(extent/h) cells per direction and
    every cell into two triangles.  Grid vertices on shared edges and corners
    are merged, so the mesh is closed and conforming.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    n = np.maximum(1, np.ceil((hi - lo) / h - 1e-9).astype(int))
    index: dict[tuple[int, int, int], int] = {}
    verts: list[np.ndarray] = []

    def vid(ijk):
        k = index.get(ijk)
        if k is None:
            k = len(verts)
            index[ijk] = k
            verts.append(lo + (hi - lo) * np.asarray(ijk, dtype=np.float64) / n)
        return k

    tris = []
    for axis in range(3):
        u, w = [a for a in range(3) if a != axis]
        for side in (0, n[axis]):
            for i in range(n[u]):
                for j in range(n[w]):
                    def g(di, dj):
                        ijk = [0, 0, 0]
                        ijk[axis] = side
                        ijk[u] = i + di
                        ijk[w] = j + dj
                        return vid(tuple(ijk))
                    a, b, c, d = g(0, 0), g(1, 0), g(1, 1), g(0, 1)
                    # alternate the diagonal to avoid a directional bias
                    if (i + j) % 2 == 0:
                        tris += [[a, b, c], [a, c, d]]
                    else:
                        tris += [[a, b, d], [b, c, d]]
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int32)
    # orient each triangle so that its normal points away from the box centre
    ctr = 0.5 * (lo + hi)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, (a + b + c) / 3.0 - ctr) < 0
    t[flip] = t[flip][:, [0, 2, 1]]
    return v, np.ascontiguousarray(t)


def capsule(radius: float, length: float, h: float, axis: int = 1, center=(0.0, 0.0, 0.0)):
    """Cylinder of the given radius with hemispherical caps (total ``length``).

    Built from rings of ``m`` vertices (m ~ 2*pi*radius/h) placed along the
    axis; each cap closes with a pole vertex.  Cap rings sit at equal polar
    angle steps so the triangles stay close to the target size ``h``.
    """
    cyl = max(length - 2.0 * radius, 0.0)
    m = max(6, int(round(2.0 * np.pi * radius / h)))
    n_cyl = max(1, int(np.ceil(cyl / h - 1e-9)))
    n_cap = max(2, int(np.ceil(0.5 * np.pi * radius / h - 1e-9)))
    rings = []  # (axial coordinate, ring radius, angular offset)
    for k in range(n_cap - 1, 0, -1):  # bottom cap, from near the pole to the equator
        phi = 0.5 * np.pi * k / n_cap
        rings.append((-0.5 * cyl - radius * np.sin(phi), radius * np.cos(phi)))
    for k in range(n_cyl + 1):
        rings.append((-0.5 * cyl + cyl * k / n_cyl, radius))
    for k in range(1, n_cap):
        phi = 0.5 * np.pi * k / n_cap
        rings.append((0.5 * cyl + radius * np.sin(phi), radius * np.cos(phi)))
    verts = [np.array([-0.5 * cyl - radius, 0.0, 0.0])]  # bottom pole (axial, u, w)
    ring_ids = []
    for r_i, (s, rr) in enumerate(rings):
        ids = []
        off = 0.5 * (r_i % 2) * 2.0 * np.pi / m
        for j in range(m):
            th = 2.0 * np.pi * j / m + off
            verts.append(np.array([s, rr * np.cos(th), rr * np.sin(th)]))
            ids.append(len(verts) - 1)
        ring_ids.append(ids)
    verts.append(np.array([0.5 * cyl + radius, 0.0, 0.0]))  # top pole
    top = len(verts) - 1
    tris = []
    for j in range(m):
        tris.append([0, ring_ids[0][(j + 1) % m], ring_ids[0][j]])
    for r_i in range(len(ring_ids) - 1):
        a, b = ring_ids[r_i], ring_ids[r_i + 1]
        for j in range(m):
            tris.append([a[j], a[(j + 1) % m], b[j]])
            tris.append([a[(j + 1) % m], b[(j + 1) % m], b[j]])
    last = ring_ids[-1]
    for j in range(m):
        tris.append([top, last[j], last[(j + 1) % m]])
    loc = np.asarray(verts)
    v = np.zeros_like(loc)
    others = [a for a in range(3) if a != axis]
    v[:, axis] = loc[:, 0]
    v[:, others[0]] = loc[:, 1]
    v[:, others[1]] = loc[:, 2]
    v += np.asarray(center, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int32)
    # orient outward from the axis / centre
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0 - np.asarray(center)
    radial = cen.copy()
    ax_c = np.clip(cen[:, axis], -0.5 * cyl, 0.5 * cyl)
    radial[:, axis] = cen[:, axis] - ax_c
    flip = np.einsum("ij,ij->i", nrm, radial) < 0
    t[flip] = t[flip][:, [0, 2, 1]]
    return v, np.ascontiguousarray(t)


def shell(level: int, inner_axes, outer_axes, center=(0.0, 0.0, 0.0)):
    """Thick shell between two ellipsoids (one domain with two boundary parts).

    The outer surface keeps its outward normal; the inner surface is reversed
    so that its normal points into the cavity (out of the shell material).
    """
    vo, to = ellipsoid(level, outer_axes, center)
    vi, ti = ellipsoid(level, inner_axes, center)
    ti = ti[:, [0, 2, 1]]
    v = np.concatenate([vo, vi])
    t = np.concatenate([to, ti + len(vo)]).astype(np.int32)
    return v, np.ascontiguousarray(t)


def geodesic_sphere(freq: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Class-I geodesic sphere: every icosahedron face split into freq**2
    triangles on a barycentric grid, grid points projected onto the sphere.

    Sizes: 10*freq**2 + 2 vertices and 20*freq**2 triangles, for any
    freq >= 1 (freq = 2**level gives the icosphere's counts), so the element
    size can follow a target h continuously.  Grid points on shared edges and
    corners are merged through their integer barycentric weights on the
    icosahedron's vertex ids.
    """
    if freq < 1:
        raise ValueError("freq must be >= 1")
    v0, t0 = icosahedron()
    index: dict[tuple, int] = {}
    verts: list[np.ndarray] = []

    def vid(ids, wts):
        key = tuple(sorted((int(i), int(w)) for i, w in zip(ids, wts) if w > 0))
        k = index.get(key)
        if k is None:
            k = len(verts)
            index[key] = k
            p = sum(w * v0[i] for i, w in key) / float(freq)
            verts.append(p / np.linalg.norm(p))
        return k

    tris = []
    for a, b, c in t0:
        g = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                g[i, j] = vid((a, b, c), (freq - i - j, i, j))
        for i in range(freq):
            for j in range(freq - i):
                tris.append([g[i, j], g[i + 1, j], g[i, j + 1]])
                if i + j <= freq - 2:
                    tris.append([g[i + 1, j], g[i + 1, j + 1], g[i, j + 1]])
    v = np.asarray(verts, dtype=np.float64) * radius + np.asarray(center, dtype=np.float64)
    return v, _orient_outward(v, np.asarray(tris, dtype=np.int32))


def geodesic_ellipsoid(freq: int, semi_axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0)):
    """Geodesic sphere of frequency ``freq`` scaled along the coordinate axes."""
    v, t = geodesic_sphere(freq)
    v = v * np.asarray(semi_axes, dtype=np.float64) + np.asarray(center, dtype=np.float64)
    return v, _orient_outward(v, t)


def geodesic_shell(freq: int, inner_axes, outer_axes, center=(0.0, 0.0, 0.0)):
    """Thick shell between two geodesic ellipsoids (inner surface reversed)."""
    vo, to = geodesic_ellipsoid(freq, outer_axes, center)
    vi, ti = geodesic_ellipsoid(freq, inner_axes, center)
    ti = ti[:, [0, 2, 1]]
    v = np.concatenate([vo, vi])
    t = np.concatenate([to, ti + len(vo)]).astype(np.int32)
    return v, np.ascontiguousarray(t)


def mesh_size(v: np.ndarray, t: np.ndarray) -> float:
    """Mean edge length (used only to report h for a generated mesh)."""
    e = np.concatenate([v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 1]], v[t[:, 0]] - v[t[:, 2]]])
    return float(np.linalg.norm(e, axis=1).mean())
