"""Pins of the cubic particle shape of the 2D oracle (Sec. 4 names cubic shapes
as the cure of the (+-1, +-2) NCI modes that survive with quadratic ones;
Appendix A: the form factors of order l).  What fixes it:

* the cubic B-spline is the quadratic one smoothed by a one-cell box:
  S3(x) = integral of S2 over [x - 1/2, x + 1/2] (checked against the pinned
  quadratic gather of a single node by quadrature);
* partition of unity, linear data reproduced, and quadratic data x^2 turned
  into x^2 + 1/3 (the cubic spline's second moment);
* node-by-node continuity of the cubic Esirkepov deposit, total current
  q w v, and the out-of-plane current q w v3;
* the energy-conserving variant with the cubic shape (quadratic along the
  staggered directions) satisfies the work identity J.E = q v E along a move;
* Gauss's law is kept over whole steps with the correction.
"""
import numpy as np
import pytest

import oracle


def _unit_node_gather(shape, x1, x2, i0=8, j0=8, n=16):
    g = oracle.grid2(n, n, 0.2, 0.2, 0.05, shape=shape)
    E = np.zeros((3, n, n))
    E[2, j0, i0] = 1.0
    Ep, _ = oracle.gather2(g, E, np.zeros_like(E), np.atleast_1d(x1), np.atleast_1d(x2))
    return Ep[2]


def test_cubic_is_the_box_smoothed_quadratic():
    gen = np.random.default_rng(1)
    t, wq = np.polynomial.legendre.leggauss(12)
    for _ in range(20):
        x = 8 + gen.uniform(-2.2, 2.2)
        y = 8.3
        s3 = _unit_node_gather(3, x, y)[0] / _unit_node_gather(3, 8.0, y)[0] * (2.0 / 3.0)
        # integral over [x - 1/2, x + 1/2] of S2, piecewise polynomial: split at
        # the quadratic spline's break points (half-integers and +-3/2 around 8)
        br = np.array([x - 0.5] + [8 + k for k in (-1.5, -0.5, 0.5, 1.5) if x - 0.5 < 8 + k < x + 0.5]
                      + [x + 0.5])
        acc = 0.0
        for a, b in zip(br[:-1], br[1:]):
            pts = 0.5 * (b - a) * t + 0.5 * (a + b)
            vals = _unit_node_gather(2, pts, np.full_like(pts, y)) / _unit_node_gather(2, 8.0, y)[0] * 0.75
            acc += 0.5 * (b - a) * np.sum(wq * vals)
        assert abs(s3 - acc) < 1e-13, (x, s3, acc)


def test_cubic_gather_moments():
    n = 16
    g = oracle.grid2(n, n, 0.2, 0.2, 0.05, shape=3)
    gen = np.random.default_rng(2)
    xi = np.stack([gen.uniform(4, 12, 60), gen.uniform(4, 12, 60)])
    ii = np.arange(n)
    E = np.zeros((3, n, n))
    B = np.zeros((3, n, n))
    E[2] = 1.7
    Ep, _ = oracle.gather2(g, E, B, xi[0], xi[1])
    np.testing.assert_allclose(Ep[2], 1.7, rtol=1e-14)
    E[2] = np.ones(n)[:, None] * (3.0 * ii - 1.0)[None, :]
    Ep, _ = oracle.gather2(g, E, B, xi[0], xi[1])
    np.testing.assert_allclose(Ep[2], 3.0 * xi[0] - 1.0, rtol=1e-13)
    E[2] = np.ones(n)[:, None] * (ii ** 2.0)[None, :]
    Ep, _ = oracle.gather2(g, E, B, xi[0], xi[1])
    np.testing.assert_allclose(Ep[2], xi[0] ** 2 + 1.0 / 3.0, rtol=1e-13)
    # a half-node (staggered) component: nodes at i + 1/2
    E[:] = 0
    E[0] = np.ones(n)[:, None] * ((ii + 0.5) ** 2)[None, :]
    Ep, _ = oracle.gather2(g, E, B, xi[0], xi[1])
    np.testing.assert_allclose(Ep[0], xi[0] ** 2 + 1.0 / 3.0, rtol=1e-13)


def _moves(gen, n, count):
    xa = np.stack([gen.uniform(0, n[0], count), gen.uniform(0, n[1], count)])
    xb = xa + gen.uniform(-0.95, 0.95, (2, count))
    return xa, xb


def test_cubic_deposit_continuity_and_totals():
    n = (16, 12)
    g = oracle.grid2(*n, 0.2, 0.25, 0.05, shape=3)
    gen = np.random.default_rng(3)
    xa, xb = _moves(gen, n, 50)
    qw = gen.uniform(0.5, 1.5, 50)
    v3 = gen.uniform(-0.5, 0.5, 50)
    J = oracle.deposit2(g, xa[0], xa[1], xb[0], xb[1], v3, qw)
    xbw = np.stack([np.mod(xb[0], n[0]), np.mod(xb[1], n[1])])
    r0 = oracle.rho2(g, xa[0], xa[1], qw)
    r1 = oracle.rho2(g, xbw[0], xbw[1], qw)
    div = ((J[0] - np.roll(J[0], 1, axis=1)) / 0.2 + (J[1] - np.roll(J[1], 1, axis=0)) / 0.25)
    res = r1 - r0 + 0.05 * div
    assert np.abs(res).max() < 1e-13 * np.abs(r1).max()
    # totals: sum j = q w v (cells of unit volume in these units)
    v = (xb - xa) * np.array([[0.2], [0.25]]) / 0.05
    np.testing.assert_allclose(J[0].sum(), (qw * v[0]).sum(), rtol=1e-12)
    np.testing.assert_allclose(J[1].sum(), (qw * v[1]).sum(), rtol=1e-12)
    np.testing.assert_allclose(J[2].sum(), (qw * v3).sum(), rtol=1e-12)
    # the cubic stencil is wider than the quadratic one
    gq = oracle.grid2(*n, 0.2, 0.25, 0.05, shape=2)
    Jq = oracle.deposit2(gq, xa[0], xa[1], xb[0], xb[1], v3, qw)
    assert (np.abs(J[2]) > 0).sum() > (np.abs(Jq[2]) > 0).sum()


def _path_integral(values_at, a, b, breaks):
    lo, hi = min(a, b), max(a, b)
    pts = np.array([lo] + [p for p in breaks if lo < p < hi] + [hi])
    t, w = np.polynomial.legendre.leggauss(6)
    acc = 0.0
    for u, v in zip(pts[:-1], pts[1:]):
        q = 0.5 * (v - u) * t + 0.5 * (u + v)
        acc += 0.5 * (v - u) * np.sum(w * values_at(q))
    return acc if b >= a else -acc


@pytest.mark.parametrize("comp", [0, 1])
def test_cubic_energy_conserving_work_identity(comp):
    n1, n2, dx1, dx2, dt = 16, 12, 0.2, 0.25, 0.05
    g = oracle.grid2(n1, n2, dx1, dx2, dt, interp=1, shape=3)
    gen = np.random.default_rng(7 + comp)
    E = gen.standard_normal((3, n2, n1))
    B = np.zeros_like(E)
    lhs = rhs = 0.0
    breaks = [k + 0.5 * s for k in range(-2, 20) for s in (0, 1)]
    for _ in range(30):
        xa = np.array([gen.uniform(0, n1), gen.uniform(0, n2)])
        xb = xa.copy()
        xb[comp] += gen.uniform(-0.95, 0.95)
        qw = gen.uniform(0.5, 1.5)
        J = oracle.deposit2(g, [xa[0]], [xa[1]], [xb[0]], [xb[1]], [0.0], [qw])
        lhs += (J[comp] * E[comp]).sum()

        def field(s):
            pos = np.repeat(xa[:, None], len(s), axis=1)
            pos[comp] = s
            Ep, _ = oracle.gather2(g, E, B, pos[0], pos[1])
            return Ep[comp]

        rhs += qw * ((dx1, dx2)[comp] / dt) * _path_integral(field, xa[comp], xb[comp], breaks)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1.0)


def test_cubic_gauss_kept_over_steps():
    n1, n2, dx, dt = 32, 16, 0.2, 0.05
    gen = np.random.default_rng(9)
    npart = 4 * n1 * n2
    xi = np.stack([gen.uniform(0, n1, npart), gen.uniform(0, n2, npart)])
    u = gen.normal(0, 0.2, (3, npart))
    qw = -np.ones(npart) / 4
    g = oracle.grid2(n1, n2, dx, dx, dt, alpha=0.5, shape=3)
    st = oracle.State2(g, -1.0, xi[0], xi[1], u, qw)
    rho_bg = -oracle.rho2(g, xi[0], xi[1], qw)
    st.step(10)
    rho = oracle.rho2(g, st.xi1, st.xi2, qw) + rho_bg
    R = oracle.gauss2(g, st.E, rho)
    ref = np.abs(np.fft.rfft(rho, axis=1)).max()
    assert np.abs(st.E).max() > 1e-6
    assert np.abs(R).max() < 1e-11 * max(ref, 1e-30) * n1
