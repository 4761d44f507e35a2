"""Pins of the [k]1 modification of Eq. (29) (Sec. 4).

The coefficients are the paper's (golden fixture dkmod_table1.txt).  A mode
inside the bump propagates with the modified symbol in the closed-form
dispersion of the leapfrog, a mode outside it with k1 itself, and the Gauss
residual stays constant over whole steps when the current correction is the
ratio [k]1,FD / [k]1,mod.
"""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W
from tests.golden import load


def _dk(k1, dx1):
    c = load("dkmod_table1.txt")
    kg = 2 * np.pi / dx1
    kl, ku, dmax = c["k1l_over_kg1"] * kg, c["k1u_over_kg1"] * kg, c["dkmax_over_kg1"] * kg
    km = 0.5 * (kl + ku)
    if k1 < kl or k1 > ku:
        return 0.0
    return dmax * np.cos((k1 - km) / (kl - km) * np.pi / 2) ** 2


@pytest.mark.parametrize("k1i", [40, 50, 55, 64, 80])
def test_kmod_dispersion(k1i):
    """TE mode (E3 only) of wavenumber k1 = 2 pi k1i / (n1 dx1) and one x2
    wavelength: sin(theta/2) = (dt/2) sqrt((k1 + dk)^2 + [k]2^2)."""
    n1, n2, dx1, dx2 = 256, 8, 0.2, 0.2
    dt = 0.9 * oracle.courant_limit2(dx1, dx2)
    g = oracle.grid2(n1, n2, dx1, dx2, dt, alpha=1.0, kmod=1)
    X1, X2 = np.meshgrid(np.arange(n1), np.arange(n2))
    E = np.zeros((3, n2, n1))
    E[2] = np.cos(2 * np.pi * (k1i * X1 / n1 + X2 / n2))
    B = np.zeros_like(E)
    J = np.zeros_like(E)
    E0 = E.copy()
    steps = 50
    for _ in range(steps):
        E, B = oracle.field_update2(g, E, B, J)
    k1 = 2 * np.pi * k1i / (n1 * dx1)
    kk = k1 + _dk(k1, dx1)
    kk2 = np.sin(np.pi / n2) / (dx2 / 2)
    theta = 2 * np.arcsin(0.5 * dt * np.hypot(kk, kk2))
    assert np.abs(E[2] - np.cos(steps * theta) * E0[2]).max() < 1e-11
    # the bump is where the paper puts it: modes at k1/kg1 = 0.156 .. 0.25 are shifted
    inside = 0.15 < k1 / (2 * np.pi / dx1) < 0.26
    assert (_dk(k1, dx1) > 0) == inside


def test_kmod_gauss_conserved():
    """With the modified symbol the corrected current keeps D.E - f rho constant
    (the correction [k]1,FD/[k]1,mod), for a drifting plasma over whole steps."""
    d = W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=5.0, sigma_u=0.1, jitter=True, seed=21)
    g = oracle.grid2(64, 16, 0.2, 0.2, 0.05, alpha=0.5, jbg=d["jbg"], kmod=1)
    qw = d["q"] * d["w"]
    rho_bg = -oracle.rho2(g, d["xi"][0], d["xi"][1], qw)
    st = oracle.State2(g, d["qm"], d["xi"][0], d["xi"][1], d["u"], qw)
    r0 = oracle.gauss2(g, st.E, oracle.rho2(g, st.xi1, st.xi2, qw) + rho_bg)
    st.step(30)
    r1 = oracle.gauss2(g, st.E, oracle.rho2(g, st.xi1, st.xi2, qw) + rho_bg)
    scale = np.abs(oracle.rfft_rows(oracle.rho2(g, st.xi1, st.xi2, qw))).max()
    assert np.abs(r1 - r0).max() < 1e-12 * scale
