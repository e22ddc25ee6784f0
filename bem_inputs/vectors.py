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
