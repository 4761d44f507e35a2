"""Pins of the NCI linear theory (Appendix A, Sec. 3, Sec. 4) against what the
mathematics and the paper's text fix.

* Without a beam the relation reduces to the hybrid solver's vacuum
  dispersion, Eqs. (19)-(20): sin(omega dt/2) = (dt/2) sqrt(k1^2 + [k]2^2).
* In the continuum limit (small grid and step at fixed k, all interpolation
  factors -> 1) the coupling term vanishes and the roots are the cold beam's
  modes omega = k1 v0 +- omega_p gamma^(-3/2) and the relativistic plasma's
  electromagnetic mode omega^2 = k^2 + omega_p^2/gamma.
* The cubic (A.4) is the expansion of (A.1) about the beam resonance: its
  growing root, refined on the full relation, stays in its neighbourhood.
* Sec. 4: with the Eq. (29) modification at the printed coefficients
  (k1l = 0.15 kg1, k1u = 0.26 kg1, dk_mod,max = 0.01 kg1) the Table 1 drift
  has no unstable (0, 0) mode; without it the fastest (0, 0) mode lies inside
  that band.
* Sec. 3: the (0, +-1) modes sit at the edge of the zone and grow about an
  order of magnitude faster than the (0, 0) modes; the k1 low-pass filter
  removes them; a smaller time step lowers the (0, 0) growth rate and moves
  the mode to larger k1 (Fig. 2 (a)-(b)).
"""
import math

import numpy as np
import pytest

from paper_1502_01376_amd import nci_theory as T


def test_no_beam_is_the_vacuum_dispersion():
    prm = T.Params(density=0.0)
    gen = np.random.default_rng(3)
    for k1, k2 in gen.uniform(0.05, 0.95, (20, 2)) * np.array([math.pi / prm.dx1, math.pi / prm.dx2]):
        kk2 = math.sin(k2 * prm.dx2 / 2) / (prm.dx2 / 2)
        w = 2 / prm.dt * math.asin(prm.dt / 2 * math.hypot(k1, kk2))
        for root in (w, -w):
            scale = abs(T.dispersion(root * 1.01, k1, k2, 0, 0, prm))
            assert scale > 0
            assert abs(T.dispersion(root, k1, k2, 0, 0, prm)) <= 1e-10 * scale


@pytest.mark.parametrize("k1,k2", [(0.7, 0.4), (1.3, -0.9), (0.2, 1.1)])
def test_continuum_limit(k1, k2):
    g, n = 5.0, 4.0
    prm = T.Params(dx1=1e-5, dx2=1e-5, dt=1e-5, gamma=g, density=n, alpha=1.0)
    v0 = prm.v0
    sy = T.symbols(k1, k2, 0, 0, prm)
    assert abs(sy["Sj1"] - 1) < 1e-9 and abs(sy["SE2"] - 1) < 1e-9
    em = math.sqrt(k1 * k1 + k2 * k2 + n / g)
    roots = [k1 * v0 + math.sqrt(n) * g ** -1.5, k1 * v0 - math.sqrt(n) * g ** -1.5, em, -em]
    for w in roots:
        scale = abs(T.dispersion(w + 0.1, k1, k2, 0, 0, prm))
        assert abs(T.dispersion(w, k1, k2, 0, 0, prm)) <= 1e-6 * scale


def test_cubic_expands_the_full_relation():
    prm = T.Params()
    k1s, k2s, g = T.growth_map(prm, 0, 0, 48, 48, (0.1, 0.35))
    order = np.argsort(g, axis=None)[::-1]
    picked = [np.unravel_index(f, g.shape) for f in order[:6]]
    assert all(g[i, j] > 0 for i, j in picked)
    for i, j in picked:
        k1, k2 = k1s[i], k2s[j]
        d = T.cubic_roots(k1, k2, 0, 0, prm)
        d = d[np.argmax(d.imag)]
        w = T.unstable_root(k1, k2, 0, 0, prm)
        assert w is not None
        assert abs(T.dispersion(w, k1, k2, 0, 0, prm)) < 1e-10
        assert abs(w - (k1 * prm.v0 + d)) < 0.1 * abs(d)
        assert 0.5 * d.imag < w.imag < 2 * d.imag


def test_kmod_removes_the_00_modes():
    """Sec. 4: the printed Eq. (29) coefficients leave no unstable (0, 0) mode
    for the Table 1 parameters; without them the mode sits inside the band."""
    ref = T.fastest(T.Params(), 0, 0, k1_range=(0.05, 0.45))
    assert ref["growth_rate"] > 0.02
    assert 0.15 <= ref["k1_over_kg1"] <= 0.26
    mod = T.fastest(T.Params(kmod=(0.15, 0.26, 0.01)), 0, 0, k1_range=(0.05, 0.45))
    assert mod["growth_rate"] == 0.0


def test_01_modes_at_the_zone_edge_and_filtered():
    f00 = T.fastest(T.Params(alpha=1.0), 0, 0, k1_range=(0.05, 0.45))
    f01 = T.fastest(T.Params(alpha=1.0), 0, -1, k1_range=(0.01, 0.5))
    assert f01["k1_over_kg1"] > 0.4
    assert f01["growth_rate"] > 4 * f00["growth_rate"]
    assert T.fastest(T.Params(alpha=0.5), 0, -1, k1_range=(0.01, 0.5))["growth_rate"] == 0.0


def test_smaller_step_slower_and_larger_k1():
    scan = T.dt_scan(ratios=(0.25, 0.35, 0.45))
    g = [r["growth_rate"] for r in scan]
    k = [r["k1_over_kg1"] for r in scan]
    assert all(r["full_relation"] for r in scan)
    assert g[0] < g[1] < g[2]
    assert k[0] > k[1] > k[2]
