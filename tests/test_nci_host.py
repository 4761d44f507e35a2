"""Host logic of the NCI harness (no GPU): the strongest-mode finder, the
growth-window detection and the growth-rate fit on synthetic histories."""
import math

import numpy as np

from paper_1502_01376_amd import nci


def test_peak_mode_finds_the_planted_mode():
    n1, n2, dx1, dx2 = 128, 64, 0.2, 0.25
    i = np.arange(n1)[None, :]
    j = np.arange(n2)[:, None]
    E2 = np.cos(2 * np.pi * (17 * i / n1 + 5 * j / n2)) + 0.1 * np.cos(2 * np.pi * 3 * i / n1)
    p = nci.peak_mode(E2, dx1, dx2)
    assert abs(p["k1_over_kg1"] - 17 / n1) < 1e-12
    assert abs(p["k1"] - 2 * np.pi * 17 / (n1 * dx1)) < 1e-12
    # the conjugate partner of (17, 5) in the half spectrum is (17, -5) or (17, 5)
    assert abs(abs(p["k2"]) - 2 * np.pi * 5 / (n2 * dx2)) < 1e-12


def test_growth_window_and_rate():
    t = np.arange(0, 600, 4.0)
    gamma = 0.035
    noise = 1e-4 * (1 + 0.3 * np.sin(t))
    w = noise + 1e-6 * np.exp(2 * gamma * t)
    w = np.minimum(w, 1e5)
    lo, hi = nci.growth_window(t, w)
    assert 100 < lo < hi < 500
    assert abs(nci.growth_rate(t, w, lo, hi) - gamma) < 1e-3 * gamma * 10
    # a flat history has no window
    assert nci.growth_window(t, noise) is None


def test_growth_rate_of_a_pure_exponential():
    t = np.linspace(0, 50, 101)
    w = 3.0 * np.exp(2 * 0.2 * t)
    assert abs(nci.growth_rate(t, w, 10, 40) - 0.2) < 1e-12
    assert math.isnan(nci.growth_rate(t, w, 60, 70))
