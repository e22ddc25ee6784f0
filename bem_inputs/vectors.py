"""Seeded random coefficient vectors (inputs only; no method arithmetic)."""
from __future__ import annotations

import numpy as np


def random_complex(n: int, seed: int = 0, n_rhs: int | None = None) -> np.ndarray:
    """Complex vector(s) with independent N(0,1) real and imaginary parts.

    Drawn with ``numpy.random.default_rng(seed)``: real parts first, then
    imaginary parts.  Shape [n] or, with ``n_rhs``, [n_rhs, n] (RHS-major).
    """
    rng = np.random.default_rng(seed)
    shape = (n,) if n_rhs is None else (n_rhs, n)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex128)


def random_rows(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted sample of ``count`` distinct row indices in [0, n)."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def stratified_rows(n_vertices, per_domain: int, seed: int) -> np.ndarray:
    """Unknown indices sampled from every domain: for each domain (vertex
    counts ``n_vertices``, unknowns laid out domain by domain as [u_D; u_N])
    its first and last vertex plus ``per_domain - 2`` distinct random ones
    (``default_rng(seed)``), each with both its u_D and u_N row.  Sorted."""
    rng = np.random.default_rng(seed)
    rows = []
    off = 0
    for nv in n_vertices:
        nv = int(nv)
        k = max(0, min(per_domain, nv) - 2)
        inner = rng.choice(np.arange(1, nv - 1), size=min(k, max(0, nv - 2)), replace=False) if nv > 2 else []
        vtx = np.unique(np.concatenate([[0, nv - 1], np.asarray(inner, dtype=np.int64)]))
        rows += list(off + vtx) + list(off + nv + vtx)
        off += 2 * nv
    return np.sort(np.asarray(rows, dtype=np.int64))
