"""Pins of the 3D oracle (Sec. 2.2: the hybrid solver with x3 differences added).

Each test fixes the oracle against something other than itself: the closed
form of the discrete vacuum dispersion, the direct real-space Yee scheme, the
Courant bound, exact node-by-node continuity, the independently pinned 2D
deposit, moment sum rules and exact reproduction of linear fields.
"""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W


def _mode(n, dx, kap):
    """Storage-index plane wave exp(i k.x) and the backward-difference symbols
    D-_d of the hybrid solver (spectral along x1, Yee differences along x2, x3)."""
    n1, n2, n3 = n
    k = [2 * np.pi * kap[d] / (n[d] * dx[d]) for d in range(3)]
    dm1 = 1j * k[0] * np.exp(-1j * k[0] * dx[0] / 2)
    dm2 = (1 - np.exp(-1j * k[1] * dx[1])) / dx[1]
    dm3 = (1 - np.exp(-1j * k[2] * dx[2])) / dx[2]
    i3, i2, i1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    ph = np.exp(1j * (k[0] * i1 * dx[0] + k[1] * i2 * dx[1] + k[2] * i3 * dx[2]))
    K2 = k[0] ** 2 + (2 * np.sin(k[1] * dx[1] / 2) / dx[1]) ** 2 + \
        (2 * np.sin(k[2] * dx[2] / 2) / dx[2]) ** 2
    return ph, (dm1, dm2, dm3), K2


@pytest.mark.parametrize("kap,pol", [((3, 1, 0), 0), ((5, 0, 2), 1), ((2, 1, 3), 2), ((7, 3, 1), 0)])
def test_vacuum_dispersion_3d(kap, pol):
    """A divergence-free single mode with B = 0 evolves as cos(n theta),
    sin(theta/2) = (dt/2) sqrt(k1^2 + [k]2^2 + [k]3^2) (Eqs. (10), (19) with
    the x3 term)."""
    n, dx = (16, 8, 8), (0.2, 0.25, 0.3)
    dt = 0.9 * oracle.courant_limit3(*dx)
    ph, dm, K2 = _mode(n, dx, kap)
    # polarisations with sum_d D-_d E_d = 0
    if pol == 0:
        Eh = np.array([dm[1], -dm[0], 0])
    elif pol == 1:
        Eh = np.array([dm[2], 0, -dm[0]])
    else:
        Eh = np.array([0, dm[2], -dm[1]])
    E0 = np.real(Eh[:, None, None, None] * ph[None])
    g = oracle.grid3(*n, *dx, dt, alpha=1.0)
    E, B = E0.copy(), np.zeros_like(E0)
    J = np.zeros_like(E0)
    steps = 30
    for _ in range(steps):
        E, B = oracle.field_update3(g, E, B, J)
    theta = 2 * np.arcsin(0.5 * dt * np.sqrt(K2))
    assert np.abs(E - np.cos(steps * theta) * E0).max() < 1e-11 * np.abs(E0).max()


def test_fd_mode_equals_yee_3d():
    """With the finite-difference symbol along x1 the hybrid update is the Yee
    scheme (end of Sec. 2.1), here in 3D against the direct real-space update."""
    n, dx = (8, 4, 6), (0.2, 0.3, 0.25)
    gen = np.random.default_rng(4)
    E = gen.standard_normal((3, n[2], n[1], n[0]))
    B = gen.standard_normal((3, n[2], n[1], n[0]))
    J = gen.standard_normal((3, n[2], n[1], n[0]))
    dt = 0.05
    g = oracle.grid3(*n, *dx, dt, alpha=1.0, deriv1=1, jbg=(0.1, -0.2, 0.3))
    Eh, Bh = oracle.field_update3(g, E, B, J)
    Ey, By = oracle.yee_update3(g, E, B, J)
    assert np.abs(Eh - Ey).max() < 1e-12
    assert np.abs(Bh - By).max() < 1e-12


@pytest.mark.parametrize("factor,stable", [(0.99, True), (1.01, False)])
def test_courant_3d(factor, stable):
    """The fastest mode (n1/2, n2/2, n3/2) is marginally stable below
    2 / sqrt(pi^2/dx1^2 + 4/dx2^2 + 4/dx3^2) and grows above it."""
    n, dx = (8, 4, 4), (0.2, 0.2, 0.2)
    dt = factor * oracle.courant_limit3(*dx)
    g = oracle.grid3(*n, *dx, dt, alpha=1.0, correct=0)
    ph, dm, _ = _mode(n, dx, (n[0] // 2, n[1] // 2, n[2] // 2))
    Eh = np.array([dm[1], -dm[0], 0])
    E = np.real(Eh[:, None, None, None] * ph[None])
    E0 = np.abs(E).max()
    B = np.zeros_like(E)
    J = np.zeros_like(E)
    for _ in range(200):
        E, B = oracle.field_update3(g, E, B, J)
    grow = np.abs(E).max() / E0
    assert (grow < 2.0) if stable else (grow > 1e3)


def _moves(n, npart, seed, vmax=0.9):
    gen = np.random.default_rng(seed)
    xa = np.stack([gen.random(npart) * n[d] for d in range(3)])
    xb = xa + vmax * (2 * gen.random((3, npart)) - 1)
    return gen, xa, xb


def test_deposit3_continuity_node_by_node():
    """rho(x^{n+1}) - rho(x^n) + dt div j = 0 at every node (Eq. (23) in 3D)."""
    n, dx, dt = (8, 6, 5), (0.2, 0.3, 0.25), 0.05
    g = oracle.grid3(*n, *dx, dt)
    gen, xa, xb = _moves(n, 300, 1)
    qw = gen.standard_normal(300)
    J = oracle.deposit3(g, xa, xb, qw)
    r0 = oracle.rho3(g, xa, qw)
    r1 = oracle.rho3(g, np.mod(xb, np.array(n)[:, None]), qw)
    div = (J[0] - np.roll(J[0], 1, axis=2)) / dx[0] + (J[1] - np.roll(J[1], 1, axis=1)) / dx[1] + \
        (J[2] - np.roll(J[2], 1, axis=0)) / dx[2]
    assert np.abs(r1 - r0 + dt * div).max() < 1e-12 * np.abs(r0).max()


def test_deposit3_reduces_to_2d():
    """With no motion along x3 the 3D currents j1, j2 summed over x3 equal the
    2D Esirkepov currents of the same (x1, x2) moves, and j3 vanishes."""
    n, dx, dt = (8, 6, 4), (0.2, 0.3, 0.25), 0.05
    g3 = oracle.grid3(*n, *dx, dt)
    g2 = oracle.grid2(n[0], n[1], dx[0], dx[1], dt)
    gen, xa, xb = _moves(n, 200, 2)
    xb[2] = xa[2]
    qw = gen.standard_normal(200)
    J3 = oracle.deposit3(g3, xa, xb, qw)
    J2 = oracle.deposit2(g2, xa[0], xa[1], xb[0], xb[1], np.zeros(200), qw)
    assert np.abs(J3[0].sum(axis=0) - J2[0]).max() < 1e-12
    assert np.abs(J3[1].sum(axis=0) - J2[1]).max() < 1e-12
    assert np.abs(J3[2]).max() < 1e-14


def test_deposit3_total_current():
    """The sum of j_d over the nodes is q w (x_d^{n+1} - x_d^n) dx_d / dt per
    particle (first moment of the shape)."""
    n, dx, dt = (8, 8, 8), (0.2, 0.3, 0.25), 0.05
    g = oracle.grid3(*n, *dx, dt)
    gen, xa, xb = _moves(n, 50, 3)
    qw = gen.standard_normal(50)
    J = oracle.deposit3(g, xa, xb, qw)
    for d in range(3):
        want = (qw * (xb[d] - xa[d])).sum() * dx[d] / dt
        assert abs(J[d].sum() - want) < 1e-11


def test_gather3_linear_fields_exact():
    """The quadratic B-spline reproduces linear functions: a field linear in the
    node position (at each component's stagger) is gathered exactly."""
    n = (16, 8, 8)
    g = oracle.grid3(*n, 0.2, 0.2, 0.2, 0.05)
    st_e = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
    st_b = [(0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]
    i3, i2, i1 = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    coef = [(1.0, 2.0, -0.5), (0.3, -1.0, 2.0), (-2.0, 0.5, 1.5)]

    def lin(st, c):
        return c[0] * (i1 + st[0]) + c[1] * (i2 + st[1]) + c[2] * (i3 + st[2])
    E = np.stack([lin(st_e[c], coef[c]) for c in range(3)])
    B = np.stack([lin(st_b[c], coef[(c + 1) % 3]) for c in range(3)])
    gen = np.random.default_rng(5)
    # away from the periodic seam, where the linear function jumps
    xi = np.stack([2 + gen.random(100) * (n[d] - 4) for d in range(3)])
    Ep, Bp = oracle.gather3(g, E, B, xi)
    for c in range(3):
        we = sum(coef[c][d] * xi[d] for d in range(3))
        wb = sum(coef[(c + 1) % 3][d] * xi[d] for d in range(3))
        assert np.abs(Ep[c] - we).max() < 1e-12
        assert np.abs(Bp[c] - wb).max() < 1e-12


def test_deposit3_fixed_matches_fp64():
    """The kernel-precision deposit (FP64 weights of the FP32 offsets, one
    rounding per node contribution on a 2^40 scale, integer accumulation)
    agrees with the FP64 Esirkepov current of the same positions to that
    rounding."""
    n, dx, dt = (8, 6, 5), (0.2, 0.3, 0.25), 0.05
    g = oracle.grid3(*n, *dx, dt)
    gen, xa, xb = _moves(n, 400, 6)
    qw = (1.0 + 0.05 * gen.standard_normal(400)) * -0.5
    ca = np.floor(xa).astype(np.int32)
    fa = (xa - ca).astype(np.float32)
    xa32 = ca + fa.astype(np.float64)
    xb32 = xa32 + (xb - xa)
    cb = np.floor(xb32).astype(np.int64)
    fb = (xb32 - cb).astype(np.float32)
    xb32 = cb + fb.astype(np.float64)
    cbw = np.mod(cb, np.array(n)[:, None]).astype(np.int32)
    inv_wunit = np.float32(1.0 / np.abs(qw).max())
    cj = np.float32(2.0 ** 40)
    Jf = oracle.deposit3_fixed(n, inv_wunit, cj, ca, fa, cbw, fb, qw.astype(np.float32))
    J64 = oracle.deposit3(g, xa32, xb32, qw.astype(np.float32).astype(np.float64))
    for d in range(3):
        jd = -(dx[d] / dt) * Jf[d] / (6.0 * float(inv_wunit) * float(cj))
        assert np.abs(jd - J64[d]).max() <= 1e-10 * np.abs(J64[d]).max()


def test_gauss_conserved_3d():
    """Whole steps: the Gauss residual D.E - f rho keeps its initial value with
    the current correction of Eq. (11) and drifts without it (Eqs. (25)-(27))."""
    d = W.drift3d(16, 8, 8, spread=0.05, sigma_u=0.05, gamma=3.0, jitter=True, seed=7)
    res = {}
    for correct in (1, 0):
        g = oracle.grid3(16, 8, 8, 0.2, 0.25, 0.3, 0.05, alpha=0.5, correct=correct, jbg=d["jbg"])
        qw = d["q"] * d["w"]
        rho_bg = -oracle.rho3(g, d["xi"], qw)
        st = oracle.State3(g, d["qm"], d["xi"], d["u"], qw)
        r0 = oracle.gauss3(g, st.E, oracle.rho3(g, st.xi, qw) + rho_bg)
        st.step(20)
        r1 = oracle.gauss3(g, st.E, oracle.rho3(g, st.xi, qw) + rho_bg)
        scale = np.abs(oracle.rfft_rows(oracle.rho3(g, st.xi, qw))).max()
        res[correct] = np.abs(r1 - r0).max() / scale
    assert res[1] < 1e-12
    assert res[0] > 1e-6
