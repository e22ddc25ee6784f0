"""Geometry of a spherical-bowl array of flat circular pistons (inputs only).

The paper's HIFU array: pseudo-random positions of 256 pistons on a spherical
cap facing the geometric focus (numerical experiments, anatomical models).
Here the cap has radius of curvature ``focal`` (centre of curvature = focus),
aperture diameter ``aperture``; centres are drawn area-uniformly on the cap
and rejected when closer than ``min_spacing`` to an accepted one.  Each piston
faces the focus.  Only positions and orientations are produced; the field
model lives with the solvers.
"""
from __future__ import annotations

import numpy as np


def _frame(axis):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    helper = np.eye(3)[np.argmin(np.abs(a))]
    e1 = np.cross(a, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    return a, e1, e2


def bowl_array(n=256, focal=27.0, aperture=20.0, piston_diameter=0.8, min_spacing=0.88,
               focus=(0.0, 0.0, 0.0), axis=(0.0, 0.0, 1.0), seed=1910, max_tries=200000):
    """Centres [n, 3], unit normals [n, 3] (towards the focus) and the piston radius.

    ``axis`` is the propagation direction: the bowl sits at focus - focal * axis.
    """
    rng = np.random.default_rng(seed)
    ax, e1, e2 = _frame(axis)
    focus = np.asarray(focus, dtype=np.float64)
    half = np.arcsin(min(1.0, 0.5 * aperture / focal))
    cmin = np.cos(half)
    centres = []
    tries = 0
    while len(centres) < n and tries < max_tries:
        tries += 1
        ct = 1.0 - rng.random() * (1.0 - cmin)
        st = np.sqrt(max(0.0, 1.0 - ct * ct))
        ph = 2.0 * np.pi * rng.random()
        p = focus - focal * (ct * ax - st * (np.cos(ph) * e1 + np.sin(ph) * e2))
        if centres and np.min(np.linalg.norm(np.asarray(centres) - p, axis=1)) < min_spacing:
            continue
        centres.append(p)
    if len(centres) < n:
        raise RuntimeError(f"could only place {len(centres)} of {n} pistons")
    c = np.asarray(centres)
    nrm = focus - c
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return c, nrm, 0.5 * piston_diameter
