"""Quasi-3D field solver on the GPU against the oracle's quasi-3D update:
cylinder TM modes (m = 0, 1), random fields of modes 0..2 (FP64 form to
round-off, FP32 form to single precision), the FD symbol, the vacuum Gauss
residual, and the 4096 x 256 grid of the quasi-3D workload."""
import numpy as np
import pytest
import scipy.special as sp

import oracle

pytestmark = pytest.mark.gpu


def _random_modes(gen, M, n1, n2, scale=1.0):
    F = scale * (gen.standard_normal((M, 3, n2 + 1, n1)) + 1j * gen.standard_normal((M, 3, n2 + 1, n1)))
    F[:, :, n2] = 0
    for m in range(M):
        if m != 1:
            F[m, 2, 0] = 0
        if m != 0:
            F[m, 0, 0] = 0
    return F


def _load(sim, E, B):
    for m in range(E.shape[0]):
        sim.set_fields_mode(0, m, E[m], B[m])


def _read(sim, M):
    E = np.stack([np.stack([sim.field_mode(0, c, m) for c in range(3)]) for m in range(M)])
    B = np.stack([np.stack([sim.field_mode(0, c, m) for c in range(3, 6)]) for m in range(M)])
    return E, B


def _pair(gen, M, n1, n2):
    E = _random_modes(gen, M, n1, n2)
    B = _random_modes(gen, M, n1, n2)
    B[:, 1, 0] = 0
    B[1, 1, 0] = gen.standard_normal(n1)
    return E, B


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
@pytest.mark.parametrize("deriv1", [0, 1])
def test_q3d_random_modes_match_oracle(hpic, prec, tol, deriv1):
    M, n1, n2, dz, dr, dt = 3, 32, 12, 0.1, 0.2, 0.04
    gen = np.random.default_rng(10 + deriv1)
    E, B = _pair(gen, M, n1, n2)
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=1.0, deriv1=deriv1, precision=prec,
                                modes=M)])
    _load(sim, E, B)
    sim.step(20)
    Eg, Bg = _read(sim, M)
    g = oracle.gridq(n1, n2, M, dz, dr, dt, alpha=1.0, deriv1=deriv1)
    J = np.zeros_like(E)
    Eo, Bo = E, B
    for _ in range(20):
        Eo, Bo = oracle.field_update_q(g, Eo, Bo, J)
    scale = max(np.abs(Eo).max(), np.abs(Bo).max())
    assert np.abs(Eg - Eo).max() <= tol * scale
    assert np.abs(Bg - Bo).max() <= tol * scale
    sim.close()


@pytest.mark.parametrize("m", [0, 1])
def test_q3d_cylinder_mode(hpic, m):
    """The TM mode E_z = J_m(j_{m,1} r / R) e^{i k z} oscillates on the GPU as in
    the oracle (FP64 form, 300 steps)."""
    n1, n2, R, dz = 16, 32, 4.0, 0.2
    dr = R / n2
    k = 2 * np.pi / (n1 * dz)
    kp = sp.jn_zeros(m, 1)[0] / R
    dt = 0.5 * 2 / np.sqrt(np.pi ** 2 / dz ** 2 + 4 / dr ** 2)
    z = np.arange(n1) * dz
    zh = z + 0.5 * dz
    ri = np.arange(n2 + 1) * dr
    rh = ri + 0.5 * dr
    E = np.zeros((m + 1, 3, n2 + 1, n1), complex)
    E[m, 0] = sp.jv(m, kp * ri)[:, None] * np.exp(1j * k * zh)[None, :]
    E[m, 1] = (1j * k / kp) * sp.jvp(m, kp * rh)[:, None] * np.exp(1j * k * z)[None, :]
    rs = np.where(ri > 0, ri, 1.0)
    E[m, 2] = (-k * m / (kp ** 2 * rs))[:, None] * sp.jv(m, kp * ri)[:, None] * np.exp(1j * k * z)[None, :]
    E[m, 2, 0] = (-k / (2 * kp)) * np.exp(1j * k * z) if m == 1 else 0
    if m >= 1:
        E[m, 0, 0] = 0
    E[m, :, n2] = 0
    B = np.zeros_like(E)
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=1.0, precision="fp64", modes=m + 1)])
    _load(sim, E, B)
    sim.step(300)
    Eg, _ = _read(sim, m + 1)
    g = oracle.gridq(n1, n2, m + 1, dz, dr, dt, alpha=1.0)
    Eo, Bo = E, B
    for _ in range(300):
        Eo, Bo = oracle.field_update_q(g, Eo, Bo, np.zeros_like(E))
    assert np.abs(Eg - Eo).max() <= 1e-10 * np.abs(Eo).max()
    sim.close()


def test_q3d_vacuum_gauss(hpic):
    """Starting from E = 0 and random B, D.E stays zero per mode (FP64 form)."""
    M, n1, n2 = 3, 32, 12
    gen = np.random.default_rng(12)
    _, B = _pair(gen, M, n1, n2)
    sim = hpic.Sim([hpic.config(n1, n2, 0.1, 0.2, 0.04, alpha=1.0, precision="fp64", modes=M)])
    _load(sim, np.zeros_like(B), B)
    sim.step(40)
    d = sim.diagnostics(0)
    Eg, _ = _read(sim, M)
    assert np.abs(Eg).max() > 1e-2
    assert d["gauss_linf"] <= 1e-10 * n1 * np.abs(Eg).max() / 0.1
    sim.close()


def test_q3d_workload_grid_two_steps(hpic):
    """4096 x 256, modes 0..2, dz = 0.1, dr = 0.2, dt = 0.04: two steps of the
    FP32 form against the oracle."""
    M, n1, n2, dz, dr, dt = 3, 4096, 256, 0.1, 0.2, 0.04
    gen = np.random.default_rng(13)
    E, B = _pair(gen, M, n1, n2)
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=0.5, precision="fp32", modes=M)])
    _load(sim, E, B)
    sim.step(2)
    Eg, Bg = _read(sim, M)
    g = oracle.gridq(n1, n2, M, dz, dr, dt, alpha=0.5)
    J = np.zeros_like(E)
    Eo, Bo = E, B
    for _ in range(2):
        Eo, Bo = oracle.field_update_q(g, Eo, Bo, J)
    scale = max(np.abs(Eo).max(), np.abs(Bo).max())
    assert np.abs(Eg - Eo).max() <= 2e-5 * scale
    assert np.abs(Bg - Bo).max() <= 2e-5 * scale
    sim.close()
