"""Pins of the oracle's hybrid field solver.

* Vacuum dispersion (Eqs. (10), (19)-(20)): a single discrete eigenmode
  (kappa1, kappa2) started with B = 0 (TE) or E = 0 (TM) evolves as
  cos(n theta) with sin(theta/2) = (dt/2) sqrt(k1^2 + [k]2^2); with the
  finite-difference x1 symbol the same holds with [k]1 (Eq. (28)).
* Courant limit (Eq. (22)): the (kappa1, kappa2) = (N1/2, N2/2) corner mode
  stays bounded just below the limit and grows just above it; for square
  cells the limit is the printed 0.537 dx1 (golden fixture).
* Yee recovery (end of Sec. 2.1): the hybrid update with the finite-difference
  x1 symbol equals a direct real-space Yee update, Eqs. (1)-(6).
* Brute force on a tiny grid: the hybrid update equals a real-space update
  built in the test from dense matrices D1+- = F^-1 diag(i k1 xi+-) F made with
  numpy's FFT, x2 differences as shifts, the Eq. (11) correction and the
  low-pass mask as F^-1 diag(.) F.
"""
import numpy as np
import pytest

import oracle
from tests.golden import load


def _mode(n1, n2, k1i, k2i, s1, s2):
    i1 = np.arange(n1) + s1
    i2 = np.arange(n2) + s2
    X1, X2 = np.meshgrid(i1, i2)
    return np.cos(2 * np.pi * (k1i * X1 / n1 + k2i * X2 / n2))


@pytest.mark.parametrize("deriv1", [0, 1])
@pytest.mark.parametrize("pol", ["TE", "TM"])
@pytest.mark.parametrize("k1i,k2i", [(1, 0), (3, 2), (7, 5), (16, 8), (0, 3)])
def test_vacuum_dispersion(deriv1, pol, k1i, k2i):
    n1, n2, dx1, dx2 = 32, 16, 0.2, 0.3
    dt = 0.9 * oracle.courant_limit2(dx1, dx2)
    g = oracle.grid2(n1, n2, dx1, dx2, dt, alpha=1.0, deriv1=deriv1)
    k1 = 2 * np.pi * k1i / (n1 * dx1)
    k2 = 2 * np.pi * k2i / (n2 * dx2)
    kk1 = np.sin(k1 * dx1 / 2) / (dx1 / 2) if deriv1 else k1
    kk2 = np.sin(k2 * dx2 / 2) / (dx2 / 2)
    theta = 2 * np.arcsin(0.5 * dt * np.sqrt(kk1 ** 2 + kk2 ** 2))
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    J = np.zeros((3, n2, n1))
    if pol == "TE":
        E[2] = _mode(n1, n2, k1i, k2i, 0.0, 0.0)      # E3 node (i1, i2)
        ref = E[2].copy()
    else:
        B[2] = _mode(n1, n2, k1i, k2i, 0.5, 0.5)      # B3 node (i1+1/2, i2+1/2)
        ref = B[2].copy()
    steps = 60
    for _ in range(steps):
        E, B = oracle.field_update2(g, E, B, J)
    got = E[2] if pol == "TE" else B[2]
    assert np.abs(got - np.cos(steps * theta) * ref).max() < 1e-11


def _corner_growth(dt_factor, dx1, dx2, steps=3000):
    n1, n2 = 16, 8
    dt = dt_factor * oracle.courant_limit2(dx1, dx2)
    g = oracle.grid2(n1, n2, dx1, dx2, dt, alpha=1.0)
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    E[2] = _mode(n1, n2, n1 // 2, n2 // 2, 0.0, 0.0) + 1e-3 * np.random.default_rng(0).standard_normal((n2, n1))
    J = np.zeros_like(E)
    amp0 = np.abs(E).max()
    for _ in range(steps):
        E, B = oracle.field_update2(g, E, B, J)
    return np.abs(E).max() / amp0


def test_courant_limit_threshold():
    dx1, dx2 = 0.2, 0.2
    assert _corner_growth(0.99, dx1, dx2, steps=3000) < 3.0
    # just above the limit the corner mode grows by ~1.33 per step
    assert _corner_growth(1.01, dx1, dx2, steps=200) > 1e6


def test_courant_square_cells_golden():
    fix = load("courant_square_cells.txt")
    dx = 0.2
    assert round(oracle.courant_limit2(dx, dx) / dx, 3) == fix["dt_over_dx1"]


def test_courant_bound_is_the_corner_mode():
    # the largest numerical frequency over all modes sits at the corner mode,
    # where (dt/2) sqrt(k1max^2 + [k]2max^2) = 1 exactly at the limit
    dx1, dx2 = 0.1, 0.2
    dt = oracle.courant_limit2(dx1, dx2)
    assert abs(0.5 * dt * np.hypot(np.pi / dx1, 2 / dx2) - 1) < 1e-15


@pytest.mark.parametrize("n1,n2", [(16, 8), (32, 5)])
def test_fd_mode_recovers_yee(n1, n2):
    dx1, dx2, dt = 0.15, 0.25, 0.05
    gen = np.random.default_rng(n1 * 100 + n2)
    E = gen.standard_normal((3, n2, n1))
    B = gen.standard_normal((3, n2, n1))
    J = gen.standard_normal((3, n2, n1))
    jbg = (0.3, -0.1, 0.2)
    g = oracle.grid2(n1, n2, dx1, dx2, dt, alpha=1.0, deriv1=1, jbg=jbg)
    Eh, Bh = oracle.field_update2(g, E, B, J)
    Ey, By = oracle.yee_update2(g, E, B, J)
    assert np.abs(Eh - Ey).max() < 1e-13 * 50
    assert np.abs(Bh - By).max() < 1e-13 * 50


def _dense_ops(n1, dx1, correct, alpha):
    kap = np.fft.fftfreq(n1, d=1.0 / n1)                    # signed mode numbers
    k1 = 2 * np.pi * kap / (n1 * dx1)
    F = np.fft.fft(np.eye(n1), axis=0)                       # F @ x = fft(x)
    Fi = np.fft.ifft(np.eye(n1), axis=0)
    h = k1 * dx1 / 2
    # i k1 xi+- ; at the Nyquist bin (fftfreq gives kappa = -n1/2) these are
    # the real numbers -pi/dx1 and +pi/dx1, the same for +-n1/2
    sym_p = 1j * k1 * np.exp(1j * h)
    sym_m = 1j * k1 * np.exp(-1j * h)
    Dp = Fi @ np.diag(sym_p) @ F
    Dm = Fi @ np.diag(sym_m) @ F
    sinc = np.ones(n1)
    nz = kap != 0
    sinc[nz] = np.sin(h[nz]) / h[nz]
    if not correct:
        sinc[:] = 1
    mask = (np.abs(kap) <= alpha * n1 / 2).astype(float)
    C = Fi @ np.diag(sinc * mask) @ F
    M = Fi @ np.diag(mask) @ F
    return Dp.real, Dm.real, C.real, M.real


@pytest.mark.parametrize("correct,alpha", [(1, 1.0), (0, 1.0), (1, 0.5)])
def test_brute_force_dense_operators(correct, alpha):
    n1, n2, dx1, dx2, dt = 8, 4, 0.2, 0.3, 0.05
    gen = np.random.default_rng(7)
    E = gen.standard_normal((3, n2, n1))
    B = gen.standard_normal((3, n2, n1))
    J = gen.standard_normal((3, n2, n1))
    g = oracle.grid2(n1, n2, dx1, dx2, dt, alpha=alpha, correct=correct)
    Eo, Bo = oracle.field_update2(g, E, B, J)

    Dp, Dm, C, M = _dense_ops(n1, dx1, correct, alpha)
    d1p = lambda f: f @ Dp.T          # act along x1 on rows
    d1m = lambda f: f @ Dm.T
    d2p = lambda f: (np.roll(f, -1, axis=0) - f) / dx2
    d2m = lambda f: (f - np.roll(f, 1, axis=0)) / dx2
    Jt = np.stack([J[0] @ C.T, J[1] @ M.T, J[2] @ M.T])

    def faraday(E, B, h):
        B = B.copy()
        B[0] -= h * d2p(E[2])
        B[1] -= h * (-d1p(E[2]))
        B[2] -= h * (d1p(E[1]) - d2p(E[0]))
        return B

    B1 = faraday(E, B, dt / 2)
    E1 = E.copy()
    E1[0] += dt * (d2m(B1[2]) - Jt[0])
    E1[1] += dt * (-d1m(B1[2]) - Jt[1])
    E1[2] += dt * (d1m(B1[1]) - d2m(B1[0]) - Jt[2])
    B2 = faraday(E1, B1, dt / 2)
    assert np.abs(Eo - E1).max() < 1e-12
    assert np.abs(Bo - B2).max() < 1e-12
