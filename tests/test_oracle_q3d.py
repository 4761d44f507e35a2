"""Pins of the quasi-3D field solver of the oracle (Sec. 5: the hybrid solver
per azimuthal mode, FFT along z = x1 and differences along r = x2).

The per-mode equations follow the cited quasi-3D method (not printed in the
paper); they are pinned here by: the closed-form TM modes of a conducting
cylinder (Bessel zeros, second-order convergence in dr), the exact vacuum
invariance of D.E per mode (div curl = 0 of the discrete operators, axis
included for m = 0), the direct real-space r-z Yee update for the FD symbol,
stability at the time step of the 4096x256 workload, and the Gauss law under a
current that obeys the deposit's finite-difference continuity equation (which
holds only with the Eq. (11) correction of jz).
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle


def _tm_mode(n1, n2, m, R, dz, k, kp):
    """E of the TM mode E_z = J_m(kp r) e^{i k z} (B = 0) on the staggered grid,
    with the divergence-free transverse part E_perp = (i k / kp^2) grad_perp E_z."""
    dr = R / n2
    z = np.arange(n1) * dz
    zh = (np.arange(n1) + 0.5) * dz
    ri = np.arange(n2 + 1) * dr
    rh = (np.arange(n2 + 1) + 0.5) * dr
    E = np.zeros((m + 1, 3, n2 + 1, n1), complex)
    Ez = sp.jv(m, kp * ri)[:, None] * np.exp(1j * k * zh)[None, :]
    Er = (1j * k / kp) * sp.jvp(m, kp * rh)[:, None] * np.exp(1j * k * z)[None, :]
    rs = np.where(ri > 0, ri, 1.0)
    Et = (-k * m / (kp ** 2 * rs))[:, None] * sp.jv(m, kp * ri)[:, None] * np.exp(1j * k * z)[None, :]
    Et[0] = (-k / (2 * kp)) * np.exp(1j * k * z) if m == 1 else 0.0
    if m >= 1:
        Ez[0] = 0
    Ez[n2] = 0
    Et[n2] = 0
    Er[n2] = 0
    E[m, 0], E[m, 1], E[m, 2] = Ez, Er, Et
    return E


def _kperp_error(n2, m, steps=400):
    R, n1, dz = 4.0, 16, 0.2
    dr = R / n2
    k = 2 * np.pi / (n1 * dz)
    kp = sp.jn_zeros(m, 1)[0] / R
    dt = 0.5 * 2 / np.sqrt(np.pi ** 2 / dz ** 2 + 4 / dr ** 2)
    g = oracle.gridq(n1, n2, m + 1, dz, dr, dt)
    E = _tm_mode(n1, n2, m, R, dz, k, kp)
    B = np.zeros_like(E)
    J = np.zeros_like(E)
    E0 = E.copy()
    ps = []
    for _ in range(steps):
        E, B = oracle.field_update_q(g, E, B, J)
        ps.append(np.vdot(E0[m, 0], E[m, 0]).real / np.vdot(E0[m, 0], E0[m, 0]).real)
    ps = np.array(ps)
    ts = dt * np.arange(1, steps + 1)
    w_ex = np.sqrt(k ** 2 + kp ** 2)
    ws = np.linspace(0.97 * w_ex, 1.03 * w_ex, 6001)
    w = ws[int(np.argmin([np.sum((ps - np.cos(w * ts)) ** 2) for w in ws]))]
    kpn = np.sqrt(max((2 / dt * np.sin(w * dt / 2)) ** 2 - k ** 2, 0.0))
    return abs(kpn / kp - 1), np.abs(ps).max()


@pytest.mark.parametrize("m", [0, 1])
def test_cylinder_tm_modes_converge_to_bessel(m):
    """omega^2 = k^2 + (j_{m,1}/R)^2 in the continuum: the discrete radial
    wavenumber approaches j_{m,1}/R at second order in dr."""
    e16, p16 = _kperp_error(16, m)
    e32, p32 = _kperp_error(32, m)
    assert p16 < 1.001 and p32 < 1.001          # a pure oscillation, no growth
    assert e32 < 6e-4
    assert e16 / e32 > 2.5


def _random_modes(gen, M, n1, n2):
    F = gen.standard_normal((M, 3, n2 + 1, n1)) + 1j * gen.standard_normal((M, 3, n2 + 1, n1))
    # zero where the axis and wall rules require it (Ez, Er, Eth / Bz, Br, Bth)
    F[:, :, n2] = 0
    for m in range(M):
        if m != 1:
            F[m, 2, 0] = 0       # Eth (Bth row 0 is a half row, free)
        if m != 0:
            F[m, 0, 0] = 0       # Ez on the axis
    return F


def test_vacuum_gauss_invariance_per_mode():
    """With J = 0, D.E per mode stays at its initial value (zero) for any B:
    the discrete divergence of the discrete curl vanishes, axis included."""
    M, n1, n2 = 3, 16, 12
    g = oracle.gridq(n1, n2, M, 0.2, 0.25, 0.04)
    gen = np.random.default_rng(1)
    B = _random_modes(gen, M, n1, n2)
    B[:, 1, 0] = 0
    B[1, 1, 0] = gen.standard_normal(n1)   # Br on the axis only for m = 1
    B[:, 1, n2] = 0
    E = np.zeros_like(B)
    J = np.zeros_like(B)
    for _ in range(30):
        E, B = oracle.field_update_q(g, E, B, J)
    R = oracle.gauss_q(g, E, np.zeros((M, n2 + 1, n1), complex))
    assert np.abs(R).max() < 1e-11 * max(np.abs(E).max(), 1.0)
    assert np.abs(E).max() > 1e-2


def test_fd_mode_equals_direct_rz_yee():
    """deriv1 = 1: the transformed update equals the direct real-space r-z Yee
    update with z differences, for every mode."""
    M, n1, n2 = 3, 16, 10
    g = oracle.gridq(n1, n2, M, 0.2, 0.3, 0.03, alpha=1.0, deriv1=1)
    gen = np.random.default_rng(2)
    E = _random_modes(gen, M, n1, n2)
    B = _random_modes(gen, M, n1, n2)
    J = _random_modes(gen, M, n1, n2)
    Eh, Bh = oracle.field_update_q(g, E, B, J)
    Ey, By = oracle.yee_update_q(g, E, B, J)
    assert np.abs(Eh - Ey).max() < 1e-12
    assert np.abs(Bh - By).max() < 1e-12


def test_stable_at_workload_time_step():
    """dz = 0.1, dr = 0.2, dt = 0.04 (the 4096x256 quasi-3D workload): random
    fields of modes 0, 1, 2 stay bounded over 1500 steps."""
    M, n1, n2 = 3, 32, 16
    g = oracle.gridq(n1, n2, M, 0.1, 0.2, 0.04)
    gen = np.random.default_rng(3)
    E = _random_modes(gen, M, n1, n2)
    B = np.zeros_like(E)
    J = np.zeros_like(E)
    a0 = np.abs(E).max()
    for _ in range(1500):
        E, B = oracle.field_update_q(g, E, B, J)
    assert np.abs(E).max() < 20 * a0


def test_gauss_with_continuity_current():
    """A current J and a charge change that obey the finite-difference
    continuity equation of the deposit (z backward differences) keep D.E - rho
    at its value when jz is corrected by Eq. (11); without the correction the
    residual changes."""
    M, n1, n2, dz, dr, dt = 3, 16, 10, 0.2, 0.3, 0.03
    gen = np.random.default_rng(4)
    J = _random_modes(gen, M, n1, n2)
    J[:, 1, n2 - 1:] = 0                    # no radial current through the wall
    # charge change from the continuity equation with FD operators in real space
    drho = np.zeros((M, n2 + 1, n1), complex)
    for m in range(M):
        Jz, Jr, Jt = J[m]
        dzJz = (Jz - np.roll(Jz, 1, axis=1)) / dz
        for j in range(n2):
            if j == 0:
                drho[m, 0] = (4 * Jr[0] / dr + dzJz[0]) if m == 0 else 0
                continue
            rj = j * dr
            divr = ((j + 0.5) * Jr[j] - (j - 0.5) * Jr[j - 1]) / (j * dr)
            drho[m, j] = divr + 1j * m / rj * Jt[j] + dzJz[j]
    drho *= -dt
    E = _random_modes(gen, M, n1, n2)
    B = _random_modes(gen, M, n1, n2)
    B[:, 1, 0] = 0
    rho = gen.standard_normal((M, n2 + 1, n1)) + 0j
    res = {}
    for correct in (1, 0):
        g = oracle.gridq(n1, n2, M, dz, dr, dt, alpha=1.0, correct=correct)
        R0 = oracle.gauss_q(g, E, rho)
        E1, _ = oracle.field_update_q(g, E, B, J)
        R1 = oracle.gauss_q(g, E1, rho + drho)
        res[correct] = np.abs(R1 - R0).max() / np.abs(drho).max()
    assert res[1] < 1e-12
    assert res[0] > 1e-4
