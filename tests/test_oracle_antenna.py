"""Pins of the oracle's moving antenna (Sec. 6 launches the boosted-frame laser
with a moving antenna; the reading: a sheet of out-of-plane surface current
K(t) g(x2) moving along x1).  What fixes it:

* the sheet's current integrates over x1 to K(t) g(x2) at every time and x2
  (closed-form envelope, drive and Gaussian profile), and is zero outside
  its time window;
* in vacuum the sheet radiates the fields the 1D jump conditions of Maxwell's
  equations give for a current sheet moving at v: towards +x1
  E3 = -K(t_r) / (2 (1 - v)) with B2 = -E3, towards -x1
  E3 = -K(t_r) / (2 (1 + v)) with B2 = +E3, at the retarded times
  t_r = (t - x + x0)/(1 - v) and (t + x - x0)/(1 + v) -- amplitudes and
  Doppler-shifted waveforms, for a sheet at rest and a moving one (with the
  k1 filter at half the Nyquist wavenumber, which removes the grid noise a
  sheet stepping across the nodes radiates at high k1: without it the
  forward wave of a sheet at v = -0.5 carries noise of 13% of its amplitude,
  at any resolution);
* j3 carries no charge in 2D: the Gauss residual with particles is unchanged
  by the antenna.
"""
import numpy as np
import pytest

import oracle


def _K(a, t):
    s = t - a.t0
    on = (s >= 0) & (s <= a.T)
    return np.where(on, a.K0 * np.sin(np.pi * s / a.T) ** 2 * np.sin(a.omega * s + a.phase), 0.0)


def test_sheet_integrates_to_the_surface_current():
    n1, n2, dx1, dx2 = 64, 16, 0.2, 0.3
    g = oracle.grid2(n1, n2, dx1, dx2, 0.1)
    a = oracle.antenna(x0=5.03, v=-0.7, t0=1.0, T=20.0, K0=0.8, omega=1.3, phase=0.4, x2c=2.1,
                       waist=1.1)
    L1, L2 = n1 * dx1, n2 * dx2
    for t in (0.5, 1.0, 3.37, 9.9, 14.2, 21.0, 21.5):
        J = oracle.antenna2(g, a, t)
        assert np.abs(J[:2]).max() == 0.0
        x2 = np.arange(n2) * dx2 - 2.1
        x2 = (x2 + L2 / 2) % L2 - L2 / 2
        want = _K(a, t) * np.exp(-(x2 / 1.1) ** 2)
        np.testing.assert_allclose(J[2].sum(axis=1) * dx1, want, atol=1e-14)
        nz = np.nonzero(np.abs(J[2]).sum(axis=0))[0]
        if nz.size:
            # at most three nodes, around x_a(t) (periodic)
            xa = ((5.03 - 0.7 * t) % L1) / dx1
            assert nz.size <= 3
            d = (nz - xa + n1 / 2) % n1 - n1 / 2
            assert np.abs(d).max() <= 1.5


@pytest.mark.parametrize("v", [0.0, -0.5, 0.3])
def test_vacuum_emission_matches_the_jump_conditions(v):
    n1, n2, dx1, dt = 2048, 4, 0.2, 0.1
    x0, T, K0, omega = 204.8, 60.0, 1.0, 0.5
    g = oracle.grid2(n1, n2, dx1, 0.2, dt, alpha=0.5)
    a = oracle.antenna(x0=x0, v=v, t0=0.0, T=T, K0=K0, omega=omega)
    st = oracle.State2(g, -1.0, np.zeros(0), np.zeros(0), np.zeros((3, 0)), np.zeros(0), antenna=a)
    nsteps = 600
    st.step(nsteps)
    t = nsteps * dt
    x = np.arange(n1) * dx1
    xa = x0 + v * t
    E3, B2 = st.E[2, 0], st.B[1, 0]
    fwd = x > xa + 3 * dx1
    bwd = x < xa - 3 * dx1
    tr_f = (t - x + x0) / (1.0 - v)
    tr_b = (t + x - x0) / (1.0 + v)
    want_f = -_K(a, tr_f) / (2.0 * (1.0 - v))
    want_b = -_K(a, tr_b) / (2.0 * (1.0 + v))
    peak = max(np.abs(want_f[fwd]).max(), np.abs(want_b[bwd]).max())
    # the backward wave is the shorter one (the sheet's spline width and the
    # time step cost it up to 1.5% here, O(dx^2))
    assert np.abs(E3[fwd] - want_f[fwd]).max() < 0.01 * peak
    assert np.abs(E3[bwd] - want_b[bwd]).max() < 0.025 * peak
    # B2 sits half a cell from E3 (B is advanced in two half steps, so it is
    # at the same time): compare with the waveform at its own node
    xh = x + 0.5 * dx1
    want_bf = _K(a, (t - xh + x0) / (1.0 - v)) / (2.0 * (1.0 - v))
    want_bb = -_K(a, (t + xh - x0) / (1.0 + v)) / (2.0 * (1.0 + v))
    assert np.abs(B2[fwd] - want_bf[fwd]).max() < 0.01 * peak
    assert np.abs(B2[bwd] - want_bb[bwd]).max() < 0.025 * peak
    # the waves really are there (and Doppler-shifted for v != 0)
    assert np.abs(E3[fwd]).max() > 0.4 / (1.0 - v) * K0
    assert np.abs(E3[bwd]).max() > 0.4 / (1.0 + v) * K0


def test_antenna_carries_no_charge():
    n1, n2, dx, dt = 64, 16, 0.2, 0.05
    gen = np.random.default_rng(5)
    npart = 4 * n1 * n2
    xi = np.stack([gen.uniform(0, n1, npart), gen.uniform(0, n2, npart)])
    u = gen.normal(0, 0.2, (3, npart))
    qw = -np.ones(npart) / 4
    g = oracle.grid2(n1, n2, dx, dx, dt, alpha=0.5)
    a = oracle.antenna(x0=3.0, v=-0.6, t0=0.0, T=5.0, K0=2.0, omega=3.0, x2c=1.6, waist=0.8)
    st = oracle.State2(g, -1.0, xi[0], xi[1], u, qw, antenna=a)
    rho_bg = -oracle.rho2(g, xi[0], xi[1], qw)
    st.step(40)
    assert np.abs(st.E[2]).max() > 0.1
    R = oracle.gauss2(g, st.E, oracle.rho2(g, st.xi1, st.xi2, qw) + rho_bg)
    ref = np.abs(np.fft.rfft(oracle.rho2(g, st.xi1, st.xi2, qw) + rho_bg, axis=1)).max()
    assert np.abs(R).max() < 1e-11 * max(ref, 1e-30) * n1
