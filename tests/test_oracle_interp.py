"""Pins of the energy-conserving gather of the oracle (Appendix A, second
variant: the order of the shape drops by one along each staggered direction of
a component).  What fixes it: with that gather, the work done on a particle
over a straight move along one axis equals J.E of its Esirkepov current,

    sum_nodes J_c E_c dV = q w (dx_c/dt) * integral of E_c(x(t)) along the move,

exactly (the derivative of the quadratic spline is a difference of linear
ones), in 2D, 3D and for the m = 0 mode of the quasi-3D geometry; the
momentum-conserving gather breaks the identity.  The order along each
direction is pinned by quadratic data: a staggered direction interpolates the
chord, an integer-node direction gives x^2 + 1/4."""
import numpy as np
import pytest

import oracle


def _path_integral(values_at, a, b):
    """Exact integral of a function that is linear between half-integer
    points (cell units), from the function's values at the break points."""
    lo, hi = min(a, b), max(a, b)
    pts = [lo] + [k + 0.5 for k in range(int(np.floor(lo - 0.5)) + 1, int(np.floor(hi - 0.5)) + 1)
                  if lo < k + 0.5 < hi] + [hi]
    pts = np.array(pts)
    v = values_at(pts)
    integ = np.sum(0.5 * (v[1:] + v[:-1]) * np.diff(pts))
    return integ if b >= a else -integ


def _work_2d(interp, comp):
    n1, n2, dx1, dx2, dt = 16, 12, 0.2, 0.25, 0.05
    g = oracle.grid2(n1, n2, dx1, dx2, dt, interp=interp)
    gen = np.random.default_rng(3 + comp)
    E = gen.standard_normal((3, n2, n1))
    B = np.zeros_like(E)
    lhs = rhs = 0.0
    for _ in range(40):
        xa = np.array([gen.uniform(0, n1), gen.uniform(0, n2)])
        d = gen.uniform(-0.95, 0.95)
        xb = xa.copy()
        xb[comp] += d
        qw = gen.uniform(0.5, 1.5)
        J = oracle.deposit2(g, [xa[0]], [xa[1]], [xb[0]], [xb[1]], [0.0], [qw])
        lhs += (J[comp] * E[comp]).sum()

        def field(s):
            pos = np.repeat(xa[:, None], len(s), axis=1)
            pos[comp] = s
            Ep, _ = oracle.gather2(g, E, B, pos[0], pos[1])
            return Ep[comp]

        dxc = (dx1, dx2)[comp]
        rhs += qw * (dxc / dt) * _path_integral(field, xa[comp], xb[comp])
    return lhs, rhs


@pytest.mark.parametrize("comp", [0, 1])
def test_work_identity_2d(comp):
    lhs, rhs = _work_2d(1, comp)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1.0)
    lhs0, rhs0 = _work_2d(0, comp)  # the momentum-conserving gather breaks it
    assert abs(lhs0 - rhs0) > 1e-4 * abs(rhs0)


def test_work_identity_3d():
    n, dx, dt = (8, 8, 8), (0.2, 0.25, 0.3), 0.04
    g = oracle.grid3(*n, *dx, dt, interp=1)
    gen = np.random.default_rng(11)
    E = gen.standard_normal((3,) + n[::-1])
    B = np.zeros_like(E)
    for comp in range(3):
        lhs = rhs = 0.0
        for _ in range(15):
            xa = np.array([gen.uniform(0, n[d]) for d in range(3)])
            xb = xa.copy()
            xb[comp] += gen.uniform(-0.95, 0.95)
            qw = gen.uniform(0.5, 1.5)
            J = oracle.deposit3(g, xa[:, None], xb[:, None], np.array([qw]))
            lhs += (J[comp] * E[comp]).sum()

            def field(s):
                pos = np.repeat(xa[:, None], len(s), axis=1)
                pos[comp] = s
                Ep, _ = oracle.gather3(g, E, B, pos)
                return Ep[comp]

            rhs += qw * (dx[comp] / dt) * _path_integral(field, xa[comp], xb[comp])
        assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1.0), comp


def test_work_identity_q3d_m0():
    """m = 0 of the quasi-3D geometry, moves along z, stencils across the axis
    included: sum_nodes Jz Ez V_j = q w (dz/dt) * integral of Ez along the move."""
    n1, n2, M, dz, dr, dt = 16, 12, 2, 0.2, 0.25, 0.04
    g = oracle.gridq(n1, n2, M, dz, dr, dt, interp=1)
    gen = np.random.default_rng(12)
    E = np.zeros((M, 3, n2 + 1, n1), complex)
    E[0, 0] = gen.standard_normal((n2 + 1, n1))
    E[0, 0, n2] = 0
    B = np.zeros_like(E)
    j = np.arange(n2 + 1)
    V = 2 * np.pi * j * dr * dr * dz
    V[0] = np.pi * (dr / 2) ** 2 * dz
    lhs = rhs = 0.0
    for k in range(30):
        r = gen.uniform(0.0, 1.5 if k < 10 else 6.0) * dr
        th = gen.uniform(0, 2 * np.pi)
        z0 = gen.uniform(0, n1 * dz)
        d = gen.uniform(-0.95, 0.95) * dz
        pa = np.array([[z0], [r * np.cos(th)], [r * np.sin(th)]])
        pb = pa.copy()
        pb[0] += d
        qw = gen.uniform(0.5, 1.5)
        J = oracle.deposit_q(g, pa, pb, np.array([qw]))
        lhs += (J[0, 0].real * E[0, 0].real * V[:, None]).sum()

        def field(s):
            pos = np.repeat(pa, len(s), axis=1)
            pos[0] = s * dz
            Ep, _ = oracle.gather_q(g, E, B, pos)
            return Ep[0]

        rhs += qw * (dz / dt) * _path_integral(field, z0 / dz, (z0 + d) / dz)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1.0)


def test_orders_on_quadratic_data():
    """B1 (staggered in x2) on data x2^2: the chord between half nodes; E3
    (integer nodes in-plane) on x1^2: the quadratic spline's x^2 + 1/4; B3
    (staggered in both): the product of chords."""
    n1, n2 = 16, 16
    g = oracle.grid2(n1, n2, 0.2, 0.2, 0.05, interp=1)
    gen = np.random.default_rng(5)
    xi = np.stack([gen.uniform(4, 12, 50), gen.uniform(4, 12, 50)])
    ih, jh = np.arange(n1) + 0.5, np.arange(n2) + 0.5
    ii, jj = np.arange(n1), np.arange(n2)
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    B[0] = (jh ** 2)[:, None] * np.ones(n1)[None, :]
    E[2] = np.ones(n2)[:, None] * (ii ** 2)[None, :]
    B[2] = (jh ** 2)[:, None] * (ih ** 2)[None, :]
    Ep, Bp = oracle.gather2(g, E, B, xi[0], xi[1])

    def chord(x):
        lo = np.floor(x - 0.5) + 0.5
        t = x - lo
        return (1 - t) * lo ** 2 + t * (lo + 1) ** 2

    np.testing.assert_allclose(Bp[0], chord(xi[1]), rtol=1e-13)
    np.testing.assert_allclose(Ep[2], xi[0] ** 2 + 0.25, rtol=1e-13)
    np.testing.assert_allclose(Bp[2], chord(xi[0]) * chord(xi[1]), rtol=1e-13)
