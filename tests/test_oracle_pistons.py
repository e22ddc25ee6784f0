"""Pin of the piston model: the on-axis field of a flat baffled disc of radius
a is p(z) = e^{ikz} - e^{ik sqrt(z^2 + a^2)} (unit rho c u), exactly; the
24-point disc rule reproduces it to the rule's accuracy at z >= 5a."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.cpu


@pytest.mark.parametrize("k,a", [(2 * np.pi, 0.4), (2 * np.pi * 1.5, 0.4), (3.0, 0.7)])
def test_piston_on_axis_closed_form(k, a):
    c = np.array([0.3, -0.2, 0.1])
    n = np.array([0.2, 0.5, 0.84])
    n /= np.linalg.norm(n)
    p, _ = oracle.piston_field(k, [c], [n], a, [1.0])
    z = np.linspace(5 * a, 40 * a, 12)
    pts = c[None, :] + z[:, None] * n[None, :]
    exact = np.exp(1j * k * z) - np.exp(1j * k * np.sqrt(z ** 2 + a ** 2))
    err = np.abs(p(pts) - exact).max() / np.abs(exact).max()
    assert err < 1e-3, err


def test_piston_normal_derivative_matches_finite_difference():
    k, a = 2 * np.pi, 0.4
    c, n = np.zeros(3), np.array([0.0, 0.0, 1.0])
    p, dp = oracle.piston_field(k, [c], [n], a, [0.7 - 0.2j])
    x = np.array([[0.3, -0.1, 2.0]])
    nn = np.array([[0.6, 0.0, 0.8]])
    h = 1e-5
    fd = (p(x + h * nn) - p(x - h * nn)) / (2 * h)
    assert abs(dp(x, nn)[0] - fd[0]) < 1e-6 * abs(fd[0]) + 1e-9
