"""Treatment planning from a full matrix capture of a piston array.

The paper's use case for batched solves (wave equation section): one forward
solve per array element, then a constrained optimisation of the array
excitation vector that keeps the field below a threshold where healthy tissue
is to be spared.  Here:

* capture: every element's forward problem is solved in one right-hand-side
  block (``Problem.solve``), and the total pressure of every element's field at
  control points is evaluated in one call (``Problem.evaluate_field``): the
  transfer matrix H [points, elements], H[p, e] = pressure at p for unit
  excitation of element e;
* excitation: phase conjugation, a_e = exp(-i arg H[f, e]) (the largest focal
  pressure under |a_e| <= 1), and a sparing excitation,
      a(mu) = (H_s^H H_s + mu I)^-1 h_f^H,
  the minimiser of |H_s a|^2 + mu |a|^2 for a fixed focal pressure, with mu
  the largest value (closest to focusing alone) for which the peak pressure
  over the sparing points is at most ``ratio`` times the focal pressure,
  scaled so that max |a_e| = 1.

The solves and field evaluations run in the library's kernels; the
optimisation is a dense problem the size of the array (E x E, E <= 1024) on
the host.
"""
from __future__ import annotations

import time

import numpy as np


def transfer_matrix(problem_handle, centres, normals, radius, points, options):
    """Full matrix capture: H [n_points, n_elements], the solver infos, the
    region codes of the points and the seconds spent solving and evaluating.
    ``problem_handle`` is a ``Problem``; all elements are solved as one block of
    right-hand sides."""
    from . import Incident
    E = len(centres)
    inc = Incident.pistons(centres, normals, radius, 1.0, np.arange(E))
    P = problem_handle
    t0 = time.perf_counter()
    b = P.rhs(inc)
    u, info = P.solve(b, options)
    t1 = time.perf_counter()
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    if P.device:
        import torch
        pts = torch.from_numpy(pts).cuda()
    f, region = P.evaluate_field(u, pts, inc)
    if P.device:
        f = f.cpu().numpy()
        region = region.cpu().numpy()
    t2 = time.perf_counter()
    return np.ascontiguousarray(np.asarray(f).T), info, np.asarray(region), {"solve_s": t1 - t0, "field_s": t2 - t1}


def phase_conjugation(h_focus):
    """a_e = exp(-i arg h_e): every element arrives at the focus in phase."""
    h = np.asarray(h_focus, dtype=np.complex128)
    return np.exp(-1j * np.angle(h))


def sparing_excitation(h_focus, H_spare, ratio, mu_range=(1e-8, 1e8), steps=60):
    """Excitation with max_s |(H_s a)_s| <= ratio * |h_f . a| and max |a_e| = 1.

    a(mu) = (H_s^H H_s + mu I)^-1 h_f^H minimises |H_s a|^2 + mu |a|^2 among
    excitations with the same focal pressure; large mu tends to conjugation of
    h_f, small mu to the least exposure of the sparing points.  mu is the
    largest value on a log-bisection of ``mu_range`` that meets the ratio
    (scaled by the mean eigenvalue of H_s^H H_s).  Returns (a, info).
    """
    h = np.asarray(h_focus, dtype=np.complex128)
    Hs = np.asarray(H_spare, dtype=np.complex128).reshape(-1, h.shape[0])
    if Hs.shape[0] == 0:   # nothing to spare: the limit mu -> infinity
        a = h.conj() / np.max(np.abs(h))
        return a, {"mu": float("inf"), "exposure_ratio": 0.0, "met": True}
    G = Hs.conj().T @ Hs
    lam, Q = np.linalg.eigh(G)
    lam = np.maximum(lam, 0.0)
    scale = max(float(np.mean(lam)), 1e-300)
    c = Q.conj().T @ h.conj()

    def excite(mu):
        a = Q @ (c / (lam + mu * scale))
        return a / np.max(np.abs(a))

    def exposure(a):
        pf = abs(h @ a)
        return float(np.max(np.abs(Hs @ a)) / pf) if pf > 0 else np.inf

    lo, hi = np.log(mu_range[0]), np.log(mu_range[1])
    if exposure(excite(np.exp(hi))) <= ratio:
        mu = np.exp(hi)
    elif exposure(excite(np.exp(lo))) > ratio:
        mu = np.exp(lo)   # the threshold cannot be met: least exposure reachable
    else:
        for _ in range(steps):
            mid = 0.5 * (lo + hi)
            if exposure(excite(np.exp(mid))) <= ratio:
                lo = mid
            else:
                hi = mid
        mu = np.exp(lo)
    a = excite(mu)
    return a, {"mu": float(mu * scale), "exposure_ratio": exposure(a), "met": exposure(a) <= ratio * (1 + 1e-12)}


def summarise(h_focus, H_spare, a):
    """Focal pressure, peak sparing pressure and their ratio, element power."""
    pf = abs(np.asarray(h_focus) @ a)
    ps = float(np.max(np.abs(np.asarray(H_spare) @ a))) if len(H_spare) else 0.0
    return {"focal_pressure": float(pf), "max_spared_pressure": ps, "ratio": ps / pf if pf else np.inf,
            "power": float(np.sum(np.abs(a) ** 2))}


def plan(P, centres, normals, radius, focus, spare_points, ratio, options):
    """Capture, then both excitations; timings of each stage."""
    pts = np.vstack([np.atleast_2d(focus), np.atleast_2d(spare_points)])
    t0 = time.perf_counter()
    H, info, region, times = transfer_matrix(P, centres, normals, radius, pts, options)
    t_capture = time.perf_counter() - t0
    t0 = time.perf_counter()
    hf, Hs = H[0], H[1:]
    a_pc = phase_conjugation(hf)
    a_sp, sp_info = sparing_excitation(hf, Hs, ratio)
    t_opt = time.perf_counter() - t0
    return {"H": H, "region": region, "solve_info": info, "capture_s": t_capture, **times, "optimise_s": t_opt,
            "phase_conjugation": {"a": a_pc, **summarise(hf, Hs, a_pc)},
            "sparing": {"a": a_sp, **summarise(hf, Hs, a_sp), **sp_info}}
