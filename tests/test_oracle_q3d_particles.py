"""Pins of the quasi-3D particle side of the oracle: the gather from azimuthal
modes with the mirror rule below the axis, the push, the per-mode
charge-conserving deposit and the charge density (Sec. 5 runs the hybrid
solver per mode; the particle side follows the cited quasi-3D method, which the
paper does not print, so it is pinned here by what the mathematics fixes):

* uniform Cartesian fields written as m = 0, 1 modes, and the linear and
  quadratic fields G x and G (x^2 - y^2) as m = 1, 2 modes, are gathered
  exactly (the quadratic spline reproduces linear data and shifts quadratic
  data by dr^2 / 4), also for particles whose stencil crosses the axis;
* total charge with the node volumes written out here;
* discrete continuity per mode with the divergence of the Gauss residual;
* for m = 0 far from the axis, the deposit equals the Cartesian Esirkepov
  deposit of the same move divided by the face areas;
* the direct azimuthal current of m = 0 agrees with the continuity-derived one
  of m = 1 for a slow rotation;
* rings of N equal particles have no modes 1..N-1;
* the co-drifting background current is -v_z times the z-mean of rho_0;
* gyration in a uniform B_z at the Boris angle, and Gauss's law per mode kept
  over whole steps with particles (and broken without the current correction).
"""
import numpy as np
import pytest

import oracle


def _grid(n1=32, n2=16, M=3, dz=0.2, dr=0.25, dt=0.04, **kw):
    return oracle.gridq(n1, n2, M, dz, dr, dt, **kw)


def _uniform_fields(g, Ec, Bc):
    """Modes of uniform Cartesian E = (Ez, Ex, Ey), B likewise: m = 0 carries
    the z part, m = 1 the transverse part with F_r = Fx - i Fy, F_th = i F_r."""
    shape = (g.nmodes, 3, g.n2 + 1, g.n1)
    E = np.zeros(shape, complex)
    B = np.zeros(shape, complex)
    for F, c in ((E, Ec), (B, Bc)):
        F[0, 0] = c[0]
        F[1, 1] = c[1] - 1j * c[2]
        F[1, 2] = 1j * (c[1] - 1j * c[2])
    return E, B


def _positions(gen, g, n, rmax_cells):
    z = gen.uniform(0, g.n1 * g.dz, n)
    r = gen.uniform(0, rmax_cells * g.dr, n)
    th = gen.uniform(0, 2 * np.pi, n)
    return np.stack([z, r * np.cos(th), r * np.sin(th)])


def test_uniform_fields_gathered_exactly():
    g = _grid()
    gen = np.random.default_rng(1)
    Ec, Bc = (0.3, -1.2, 0.7), (-0.4, 0.9, 1.1)
    E, B = _uniform_fields(g, Ec, Bc)
    pos = _positions(gen, g, 400, 4.0)
    pos[1, :50] *= 0.05  # stencils across the axis
    Ep, Bp = oracle.gather_q(g, E, B, pos)
    np.testing.assert_allclose(Ep, np.array(Ec)[:, None] * np.ones((3, 400)), atol=1e-13)
    np.testing.assert_allclose(Bp, np.array(Bc)[:, None] * np.ones((3, 400)), atol=1e-13)


def test_linear_and_quadratic_mode_fields():
    """Ez = G x is the m = 1 mode G r (odd across the axis), Ez = G (x^2 - y^2)
    the m = 2 mode G r^2 (even); E = G (x, -y) is the m = 2 vector mode
    Er = G r, Eth = i G r (odd).  Linear data are reproduced exactly, quadratic
    data shifted by the spline's second moment dr^2 / 4."""
    g = _grid()
    gen = np.random.default_rng(2)
    G = 0.7
    rj = np.arange(g.n2 + 1) * g.dr
    rh = (np.arange(g.n2 + 1) + 0.5) * g.dr
    shape = (g.nmodes, 3, g.n2 + 1, g.n1)
    pos = _positions(gen, g, 300, 3.0)
    pos[1, :40] *= 0.1
    pos[2, :40] *= 0.1
    z, x, y = pos
    r = np.hypot(x, y)
    B = np.zeros(shape, complex)
    E = np.zeros(shape, complex)
    E[1, 0] = (G * rj)[:, None]
    Ep, _ = oracle.gather_q(g, E, B, pos)
    np.testing.assert_allclose(Ep[0], G * x, atol=1e-12)
    np.testing.assert_allclose(Ep[1:], 0, atol=1e-15)
    E = np.zeros(shape, complex)
    E[2, 0] = (G * rj ** 2)[:, None]
    Ep, _ = oracle.gather_q(g, E, B, pos)
    np.testing.assert_allclose(Ep[0], G * (r ** 2 + g.dr ** 2 / 4) * np.cos(2 * np.arctan2(y, x)),
                               atol=1e-12)
    E = np.zeros(shape, complex)
    E[2, 1] = (G * rh)[:, None]
    E[2, 2] = (1j * G * rj)[:, None]
    Ep, _ = oracle.gather_q(g, E, B, pos)
    np.testing.assert_allclose(Ep[1], G * x, atol=1e-12)
    np.testing.assert_allclose(Ep[2], -G * y, atol=1e-12)


def test_total_charge_and_node_volumes():
    g = _grid()
    gen = np.random.default_rng(3)
    pos = _positions(gen, g, 500, 9.0)
    pos[1, :60] *= 0.05
    qw = gen.uniform(0.5, 1.5, 500)
    rho = oracle.rho_q(g, pos, qw)
    V = 2 * np.pi * np.arange(g.n2 + 1) * g.dr ** 2 * g.dz
    V[0] = np.pi * (g.dr / 2) ** 2 * g.dz
    assert abs((rho[0].real * V[:, None]).sum() - qw.sum()) < 1e-11 * qw.sum()
    assert np.abs(rho[0].imag).max() == 0.0


def test_uniform_density_away_from_axis():
    """Weights proportional to r load a uniform density n: rho_0 = n on rows
    that the shapes reach from both sides (the spline's second moment makes the
    r-weighted sum exact for a uniform continuum)."""
    g = _grid(n1=16, n2=24, M=1)
    n0, per = 1.3, 64
    zs, rs, ths = [], [], []
    for i in range(g.n1):
        for j in range(18):
            for a in range(per):
                # midpoint rule in r on a fine sub-lattice of each cell
                zs.append((i + (a % 8 + 0.5) / 8) * g.dz)
                rs.append((j + (a // 8 + 0.5) / 8) * g.dr)
                ths.append(2 * np.pi * a / per)
    z, r, th = map(np.array, (zs, rs, ths))
    qw = n0 * 2 * np.pi * r * g.dr * g.dz / per
    rho = oracle.rho_q(g, np.stack([z, r * np.cos(th), r * np.sin(th)]), qw)
    np.testing.assert_allclose(rho[0, 3:15].real, n0, rtol=2e-3)


def _div(g, J):
    """Divergence of the Gauss residual, real space, FD along z: rows 1..n2-1
    for every mode, the axis (4 Jr_0/dr) for m = 0 only."""
    M = J.shape[0]
    D = np.zeros((M, g.n2 + 1, g.n1), complex)
    for m in range(M):
        Jz, Jr, Jt = J[m]
        dzJ = (Jz - np.roll(Jz, 1, axis=1)) / g.dz
        for j in range(1, g.n2):
            D[m, j] = (dzJ[j] + ((j + 0.5) * Jr[j] - (j - 0.5) * Jr[j - 1]) / (j * g.dr)
                       + 1j * m / (j * g.dr) * Jt[j])
        if m == 0:
            D[m, 0] = dzJ[0] + 4 * Jr[0] / g.dr
    return D


def _moves(gen, g, n, rmax_cells=5.0):
    pa = _positions(gen, g, n, rmax_cells)
    pa[1, : n // 5] *= 0.1
    pa[2, : n // 5] *= 0.1
    step = gen.uniform(-0.9, 0.9, (3, n)) * np.array([g.dz, g.dr / 1.5, g.dr / 1.5])[:, None]
    pb = pa + step
    return pa, pb


@pytest.mark.parametrize("M", [1, 3, 4])
def test_continuity_per_mode(M):
    g = _grid(M=M)
    gen = np.random.default_rng(10 + M)
    pa, pb = _moves(gen, g, 300)
    qw = gen.uniform(0.5, 1.5, 300)
    J = oracle.deposit_q(g, pa, pb, qw)
    pbw = pb.copy()
    pbw[0] = np.mod(pbw[0], g.n1 * g.dz)
    r0 = oracle.rho_q(g, pa, qw)
    r1 = oracle.rho_q(g, pbw, qw)
    res = r1 - r0 + g.dt * _div(g, J)
    scale = np.abs(r1).max()
    for m in range(M):
        rows = slice(0, g.n2) if m == 0 else slice(1, g.n2)
        assert np.abs(res[m, rows]).max() < 1e-12 * scale, (m, np.abs(res[m, rows]).max())


def test_m0_far_from_axis_is_cartesian_esirkepov():
    g = _grid(M=1)
    gen = np.random.default_rng(20)
    n = 60
    z0 = gen.uniform(0, g.n1 * g.dz, n)
    r0 = gen.uniform(5, 10, n) * g.dr
    z1 = z0 + gen.uniform(-0.9, 0.9, n) * g.dz
    r1 = r0 + gen.uniform(-0.9, 0.9, n) * g.dr
    th = gen.uniform(0, 2 * np.pi, n)  # same angle before and after: no azimuthal motion
    qw = gen.uniform(0.5, 1.5, n)
    pa = np.stack([z0, r0 * np.cos(th), r0 * np.sin(th)])
    pb = np.stack([z1, r1 * np.cos(th), r1 * np.sin(th)])
    J = oracle.deposit_q(g, pa, pb, qw)[0]
    g2 = oracle.grid2(g.n1, g.n2 + 1, g.dz, g.dr, g.dt)
    J2 = oracle.deposit2(g2, z0 / g.dz, r0 / g.dr, z1 / g.dz, r1 / g.dr, np.zeros(n), qw)
    j = np.arange(g.n2 + 1)
    A = 2 * np.pi * j * g.dr ** 2
    A[0] = np.pi * g.dr ** 2 / 4
    Ar = 2 * np.pi * (j + 0.5) * g.dr * g.dz
    # the 2D deposit carries dx/dt per unit charge weight; the face areas divide
    np.testing.assert_allclose(J[0].real, J2[0] / (g.dz * A[:, None]) * 1.0, atol=1e-12)
    np.testing.assert_allclose(J[1].real, J2[1] / (g.dr * Ar[:, None]), atol=1e-12)
    assert np.abs(J.imag).max() == 0.0


def test_direct_azimuthal_current_matches_flux_form():
    """A slow pure rotation at r_p: the m = 1 azimuthal current (from
    continuity) is 2 q w W P th_dot / (2 pi dr dz) per node; the m = 0 direct
    one is q w W3 v_th / V_j with v_th = r_p th_dot, i.e. the same up to the
    factor r_p / r_j and the phase."""
    g = _grid(M=2)
    rp, th0, dth = 6.3 * g.dr, 0.4, 1e-5
    z = 3.37 * g.dz
    pa = np.array([[z], [rp * np.cos(th0)], [rp * np.sin(th0)]])
    pb = np.array([[z], [rp * np.cos(th0 + dth)], [rp * np.sin(th0 + dth)]])
    J = oracle.deposit_q(g, pa, pb, np.array([1.0]))
    Pm = np.exp(-1j * (th0 + dth / 2))
    j = np.arange(g.n2 + 1)
    rj = np.where(j > 0, j * g.dr, 1.0)
    lhs = J[0, 2].real * (rj / rp)[:, None]
    rhs = (J[1, 2] / (2 * Pm)).real
    assert np.abs(rhs).max() > 0
    np.testing.assert_allclose(lhs, rhs, atol=1e-6 * np.abs(rhs).max())
    assert np.abs(J[0, 2]).max() > 0


@pytest.mark.parametrize("N", [4, 5])
def test_ring_has_no_low_modes(N):
    g = _grid(M=4)
    th = 0.3 + 2 * np.pi * np.arange(N) / N
    r0, r1, z0, z1 = 3.2 * g.dr, 3.6 * g.dr, 5.1 * g.dz, 5.5 * g.dz
    pa = np.stack([np.full(N, z0), r0 * np.cos(th), r0 * np.sin(th)])
    pb = np.stack([np.full(N, z1), r1 * np.cos(th + 0.01), r1 * np.sin(th + 0.01)])
    qw = np.ones(N)
    J = oracle.deposit_q(g, pa, pb, qw)
    rho = oracle.rho_q(g, pa, qw)
    for m in range(1, min(N, 4)):
        assert np.abs(J[m]).max() < 1e-12 * np.abs(J[0]).max()
        assert np.abs(rho[m]).max() < 1e-12 * np.abs(rho[0]).max()


def test_background_current_is_drift_times_mean_density():
    g = _grid(M=1)
    gen = np.random.default_rng(30)
    pos = _positions(gen, g, 400, 8.0)
    pos[1, :50] *= 0.05
    qw = gen.uniform(0.5, 1.5, 400)
    uz = 3.0
    u = np.stack([np.full(400, uz), np.zeros(400), np.zeros(400)])
    jbg = oracle.jbg_q(g, pos, u, qw)
    vz = uz / np.sqrt(1 + uz ** 2)
    rho = oracle.rho_q(g, pos, qw)
    np.testing.assert_allclose(jbg, -vz * rho[0].real.mean(axis=1), atol=1e-12)


def test_gyration_in_uniform_bz():
    """A test particle (negligible charge) in uniform B_z turns by the Boris
    angle 2 atan(|q/m| dt B / (2 gamma)) per step at constant |u|."""
    g = _grid(n2=24, M=2, dt=0.04)
    Bz, qm = 2.0, -1.0
    E = np.zeros((2, 3, g.n2 + 1, g.n1), complex)
    B = E.copy()
    B[0, 0] = Bz
    u0 = np.array([[0.1], [0.6], [0.0]])
    pos = np.array([[1.0], [2.0], [1.5]])
    st = oracle.StateQ(g, qm, pos, u0, np.array([1e-12]), E, B)
    n = 50
    st.step(n)
    gam = np.sqrt(1 + (u0 ** 2).sum())
    ang = 2 * np.arctan(abs(qm) * g.dt * Bz / (2 * gam))
    # du/dt = (q/m) v x B turns (ux, uy) clockwise when (q/m) Bz > 0
    turn = -np.sign(qm * Bz) * ang * n
    ux, uy = u0[1, 0], u0[2, 0]
    np.testing.assert_allclose(np.hypot(st.u[1, 0], st.u[2, 0]), np.hypot(ux, uy), rtol=1e-12)
    got = np.arctan2(st.u[2, 0], st.u[1, 0]) - np.arctan2(uy, ux)
    assert abs(np.angle(np.exp(1j * (got - turn)))) < 1e-9
    assert abs(st.u[0, 0] - 0.1) < 1e-12


def _thermal_plasma(gen, g, ppc_r=2, ppc_z=2, ppc_t=4, rcells=6, uth=0.05, drift=0.0):
    zs, rs, ths = [], [], []
    for i in range(g.n1):
        for j in range(rcells):
            for a in range(ppc_z):
                for b in range(ppc_r):
                    ph = gen.uniform(0, 2 * np.pi)
                    for t in range(ppc_t):
                        zs.append((i + (a + 0.5) / ppc_z) * g.dz)
                        rs.append((j + (b + 0.5) / ppc_r) * g.dr)
                        ths.append(ph + 2 * np.pi * t / ppc_t)
    z, r, th = map(np.array, (zs, rs, ths))
    n = len(z)
    ppc = ppc_r * ppc_z * ppc_t
    qw = 2 * np.pi * r * g.dr * g.dz / ppc
    u = gen.normal(0, uth, (3, n))
    u[0] += drift
    return np.stack([z, r * np.cos(th), r * np.sin(th)]), u, qw


def _gauss_rows(g, R):
    out = []
    for m in range(g.nmodes):
        rows = slice(0, g.n2 - 1) if m == 0 else slice(1, g.n2 - 1)
        out.append(R[m, rows])
    return out


@pytest.mark.parametrize("kmod", [0, 1])
def test_gauss_kept_over_steps_with_particles(kmod):
    g = _grid(n1=32, n2=12, M=3, dt=0.04, alpha=0.5, kmod=kmod)
    gen = np.random.default_rng(40)
    pos, u, qw = _thermal_plasma(gen, g)
    st = oracle.StateQ(g, -1.0, pos, u, -qw)  # electrons (charge -1) of weight qw
    rho_bg = -st.rho()
    R0 = oracle.gauss_q(g, st.E, st.rho() + rho_bg)
    st.step(6)
    R = oracle.gauss_q(g, st.E, st.rho() + rho_bg)
    scale = max(np.abs(st.E).max() / g.dr, 1e-30)
    assert np.abs(st.E).max() > 1e-6
    for a, b in zip(_gauss_rows(g, R), _gauss_rows(g, R0)):
        assert np.abs(a - b).max() < 1e-11 * scale, np.abs(a - b).max() / scale


def test_gauss_broken_without_correction():
    g = _grid(n1=32, n2=12, M=3, dt=0.04, alpha=1.0, correct=0)
    gen = np.random.default_rng(41)
    pos, u, qw = _thermal_plasma(gen, g, uth=0.2)
    st = oracle.StateQ(g, -1.0, pos, u, -qw)
    rho_bg = -st.rho()
    st.step(4)
    R = oracle.gauss_q(g, st.E, st.rho() + rho_bg)
    scale = np.abs(st.E).max() / g.dr
    assert max(np.abs(a).max() for a in _gauss_rows(g, R)) > 1e-6 * scale


def test_direct_azimuthal_current_moment_near_axis():
    """m = 0 azimuthal current of one particle, stencil across the axis: its
    moment sum_j r_j V_j Jth_0 is q w v_th (r_a + r_b)/2 (the spline's first
    moment), the far side of the cloud counting with the reversed direction."""
    g = _grid(M=1)
    gen = np.random.default_rng(50)
    for _ in range(20):
        ra = gen.uniform(0.05, 1.2) * g.dr
        th = gen.uniform(0, 2 * np.pi)
        dth = gen.uniform(-0.2, 0.2)
        rb = ra + gen.uniform(0.0, 0.2) * g.dr
        z = gen.uniform(0, g.n1 * g.dz)
        pa = np.array([[z], [ra * np.cos(th)], [ra * np.sin(th)]])
        pb = np.array([[z], [rb * np.cos(th + dth)], [rb * np.sin(th + dth)]])
        J = oracle.deposit_q(g, pa, pb, np.array([1.3]))
        xm, ym = 0.5 * (pa[1, 0] + pb[1, 0]), 0.5 * (pa[2, 0] + pb[2, 0])
        vx, vy = (pb[1, 0] - pa[1, 0]) / g.dt, (pb[2, 0] - pa[2, 0]) / g.dt
        vth = (xm * vy - ym * vx) / np.hypot(xm, ym)
        j = np.arange(g.n2 + 1)
        V = 2 * np.pi * j * g.dr ** 2 * g.dz
        moment = (J[0, 2].real * (j * g.dr * V)[:, None]).sum()
        assert abs(moment - 1.3 * vth * 0.5 * (ra + rb)) < 1e-12 * abs(1.3 * vth * ra) + 1e-15


def test_m1_axis_current_of_translating_ring():
    """A small ring around the axis translating along x carries the uniform
    current J_x = rho v near the axis, whose m = 1 azimuthal part on the axis
    node is i J_x: Jth_1[axis] = i v rho_0[axis] to first order in the move."""
    g = _grid(M=2)
    N, rho_r, v = 16, 0.3 * g.dr, 0.5
    th = 0.1 + 2 * np.pi * np.arange(N) / N
    z = np.full(N, 7.3 * g.dz)
    pa = np.stack([z, rho_r * np.cos(th), rho_r * np.sin(th)])
    pb = pa.copy()
    pb[1] += v * g.dt * 1e-3  # slow move: v * 1e-3
    J = oracle.deposit_q(g, pa, pb, np.ones(N))
    rho = oracle.rho_q(g, pa, np.ones(N))
    want = 1j * v * 1e-3 * rho[0, 0]
    np.testing.assert_allclose(J[1, 2, 0], want, atol=2e-3 * np.abs(want).max())
