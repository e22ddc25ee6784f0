"""Host logic of the excitation optimisation (no GPU)."""
from __future__ import annotations

import numpy as np

from paper_1910_01011_amd import planning


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_phase_conjugation_reaches_the_amplitude_bound():
    """|h . a| <= sum |h_e| for |a_e| <= 1, with equality for conjugation."""
    rng = np.random.default_rng(0)
    h = _rand(rng, 64)
    a = planning.phase_conjugation(h)
    assert np.allclose(np.abs(a), 1.0)
    assert np.isclose(abs(h @ a), np.abs(h).sum())
    for _ in range(20):
        b = np.exp(1j * rng.uniform(0, 2 * np.pi, 64)) * rng.uniform(0, 1, 64)
        assert abs(h @ b) <= np.abs(h).sum() + 1e-12


def test_sparing_meets_the_threshold_when_a_null_space_exists():
    rng = np.random.default_rng(1)
    h = _rand(rng, 32)
    Hs = _rand(rng, 5, 32)
    pc = planning.summarise(h, Hs, planning.phase_conjugation(h))
    a, info = planning.sparing_excitation(h, Hs, ratio=0.05)
    s = planning.summarise(h, Hs, a)
    assert info["met"] and s["ratio"] <= 0.05 * (1 + 1e-12)
    assert np.isclose(np.max(np.abs(a)), 1.0)
    assert pc["ratio"] > 0.05


def test_sparing_is_the_regularised_minimiser():
    """a(mu) minimises |H_s a|^2 + mu |a|^2 among vectors with the same focal
    pressure: perturbations along the focal constraint never lower it."""
    rng = np.random.default_rng(2)
    h = _rand(rng, 16)
    Hs = _rand(rng, 6, 16)
    a, info = planning.sparing_excitation(h, Hs, ratio=0.2)
    mu = info["mu"]
    obj = lambda v: np.linalg.norm(Hs @ v) ** 2 + mu * np.linalg.norm(v) ** 2
    pf = h @ a
    for _ in range(50):
        d = _rand(rng, 16)
        d -= (h @ d) / (h @ h.conj()) * h.conj()   # keeps h . (a + d) = h . a
        assert np.isclose(h @ (a + 1e-3 * d), pf)
        assert obj(a + 1e-3 * d) >= obj(a) - 1e-12 * obj(a)


def test_loose_threshold_returns_near_conjugation():
    rng = np.random.default_rng(3)
    h = _rand(rng, 16)
    Hs = 1e-6 * _rand(rng, 3, 16)
    a, info = planning.sparing_excitation(h, Hs, ratio=0.5)
    cos = abs(np.vdot(a, h.conj())) / (np.linalg.norm(a) * np.linalg.norm(h))
    assert info["met"] and cos > 0.999


def test_no_points_to_spare():
    rng = np.random.default_rng(4)
    h = _rand(rng, 8)
    a, info = planning.sparing_excitation(h, np.zeros((0, 8)), ratio=0.1)
    assert info["met"] and np.isclose(np.max(np.abs(a)), 1.0)
    assert np.isclose(abs(h @ a), np.linalg.norm(h) ** 2 / np.max(np.abs(h)))
