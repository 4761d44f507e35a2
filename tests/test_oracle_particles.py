"""Pins of the oracle's field gather and Boris push.

Gather (momentum-conserving quadratic interpolation at the Yee nodes of
Eqs. (1)-(6)): the quadratic B-spline reproduces constants and linear
functions exactly and gives x^2 + 1/4 for x^2 (its variance is 1/4).  A linear
field therefore interpolates to its value at the particle, which fails if any
component is gathered from the wrong staggered position.

Boris (relativistic, textbook form): in a pure magnetic field |u| is kept
exactly and u turns by 2 atan(|t|) per step, t = (q/m)(dt/2) B / gamma; in a
pure electric field u changes by (q/m) dt E per step; with E perpendicular to
B and |E| < |B| the mean velocity is the E x B drift.
"""
import numpy as np
import pytest

import oracle

STAG_E = [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0)]
STAG_B = [(0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]


def _node_positions(n1, n2, s1, s2):
    i1 = np.arange(n1) + s1
    i2 = np.arange(n2) + s2
    return np.meshgrid(i1, i2)  # X1[i2][i1], X2[i2][i1]


@pytest.mark.parametrize("poly", ["const", "lin1", "lin2", "quad1", "quad2"])
def test_gather_reproduces_polynomials(poly):
    n1, n2 = 32, 16
    g = oracle.grid2(n1, n2, 0.3, 0.7, 0.05)
    gen = np.random.default_rng(3)
    # keep particles away from the periodic seam so the polynomial is smooth
    xi1 = gen.uniform(4, n1 - 4, 200)
    xi2 = gen.uniform(4, n2 - 4, 200)

    def f(x1, x2):
        return {"const": 2.5 + 0 * x1, "lin1": 1.0 + 0.37 * x1, "lin2": -2.0 + 0.61 * x2,
                "quad1": x1 * x1, "quad2": x2 * x2}[poly]

    def expect(x1, x2):
        e = f(x1, x2)
        if poly == "quad1":
            e = x1 * x1 + 0.25
        if poly == "quad2":
            e = x2 * x2 + 0.25
        return e

    E = np.stack([f(*_node_positions(n1, n2, *s)) for s in STAG_E])
    B = np.stack([f(*_node_positions(n1, n2, *s)) for s in STAG_B])
    Ep, Bp = oracle.gather2(g, E, B, xi1, xi2)
    for c in range(3):
        assert np.abs(Ep[c] - expect(xi1, xi2)).max() < 1e-12
        assert np.abs(Bp[c] - expect(xi1, xi2)).max() < 1e-12


def test_gather_wraps_periodically():
    n1, n2 = 16, 8
    g = oracle.grid2(n1, n2, 0.2, 0.2, 0.05)
    gen = np.random.default_rng(4)
    E = gen.standard_normal((3, n2, n1))
    B = gen.standard_normal((3, n2, n1))
    xi1 = np.array([0.1, 15.9, 0.49, 7.0])
    xi2 = np.array([0.2, 7.95, 3.3, 0.0])
    Ep, Bp = oracle.gather2(g, E, B, xi1, xi2)
    # shifting the grid by whole cells and the particles with it changes nothing
    Ep2, Bp2 = oracle.gather2(g, np.roll(E, (3, 5), axis=(1, 2)), np.roll(B, (3, 5), axis=(1, 2)),
                              np.mod(xi1 + 5, n1), np.mod(xi2 + 3, n2))
    assert np.abs(Ep - Ep2).max() < 1e-13 and np.abs(Bp - Bp2).max() < 1e-13


def test_boris_pure_magnetic_rotation():
    gen = np.random.default_rng(5)
    n = 50
    u = gen.standard_normal((3, n)) * 10
    B = gen.standard_normal((3, n))
    E = np.zeros((3, n))
    qm, dt = -1.0, 0.05
    u1 = oracle.boris(qm, dt, E, B, u)
    gam = np.sqrt(1 + (u * u).sum(0))
    assert np.abs(np.linalg.norm(u1, axis=0) / np.linalg.norm(u, axis=0) - 1).max() < 1e-14
    t = 0.5 * qm * dt * np.linalg.norm(B, axis=0) / gam
    angle_expect = 2 * np.arctan(np.abs(t))
    # angle of the rotation about B of the perpendicular component
    bh = B / np.linalg.norm(B, axis=0)
    up0 = u - (u * bh).sum(0) * bh
    up1 = u1 - (u1 * bh).sum(0) * bh
    cosang = (up0 * up1).sum(0) / (np.linalg.norm(up0, axis=0) * np.linalg.norm(up1, axis=0))
    assert np.abs(np.arccos(np.clip(cosang, -1, 1)) - angle_expect).max() < 1e-7
    # the parallel component is untouched
    assert np.abs((u * bh).sum(0) - (u1 * bh).sum(0)).max() < 1e-12


def test_boris_pure_electric_kick():
    gen = np.random.default_rng(6)
    n = 20
    u = gen.standard_normal((3, n))
    E = gen.standard_normal((3, n))
    u1 = oracle.boris(-1.0, 0.1, E, np.zeros((3, n)), u)
    assert np.abs(u1 - (u - 0.1 * E)).max() < 1e-14


def test_boris_exb_drift():
    # E = 0.01 e2, B = e3: drift velocity E x B / B^2 = 0.01 e1 (relativistically
    # exact for uniform crossed fields with |E| < |B|)
    qm, dt = -1.0, 0.05
    E = np.array([[0.0], [0.01], [0.0]])
    B = np.array([[0.0], [0.0], [1.0]])
    u = np.zeros((3, 1))
    steps = 20000
    x1 = 0.0
    for _ in range(steps):
        u = oracle.boris(qm, dt, E, B, u)
        gam = np.sqrt(1 + (u * u).sum())
        x1 += dt * u[0, 0] / gam
    assert abs(x1 / (steps * dt) - 0.01) < 2e-4
