"""Pins of the oracle's charge-conserving deposit.

FP64 Esirkepov deposit (the local charge-conserving deposit of Sec. 2.3):
  * the discrete continuity equation (23) holds node by node to round-off,
    with rho from the plain quadratic-spline charge deposit;
  * the first moment of the current is exact: summed over the nodes, j = q w v
    (the quadratic B-spline has its centroid at the particle);
  * a particle at rest deposits j1 = j2 = 0 and j3 = q w v3 S x S;
  * reversing the motion negates j1 and j2.

Fixed-point deposit in the kernel's precision:
  * 2 (rho_new - rho_old) = div J holds exactly in the 64-bit integers;
  * converted to physical units it agrees with the FP64 deposit within the
    2^-P shape quantisation.
"""
import numpy as np
import pytest

import oracle


def _random_moves(n1, n2, npart, maxstep, seed):
    gen = np.random.default_rng(seed)
    xa1 = gen.uniform(0, n1, npart)
    xa2 = gen.uniform(0, n2, npart)
    xb1 = xa1 + gen.uniform(-maxstep, maxstep, npart)
    xb2 = xa2 + gen.uniform(-maxstep, maxstep, npart)
    v3 = gen.uniform(-0.9, 0.9, npart)
    qw = gen.uniform(-2.0, 1.0, npart)
    return xa1, xa2, xb1, xb2, v3, qw


def _div(J, dx1, dx2):
    """Backward-difference divergence of a staggered current (Eq. (23))."""
    return (J[0] - np.roll(J[0], 1, axis=1)) / dx1 + (J[1] - np.roll(J[1], 1, axis=0)) / dx2


@pytest.mark.parametrize("maxstep", [0.05, 0.45, 0.99])
def test_fp64_continuity(maxstep):
    n1, n2, dx1, dx2, dt = 16, 12, 0.1, 0.2, 0.045
    g = oracle.grid2(n1, n2, dx1, dx2, dt)
    xa1, xa2, xb1, xb2, v3, qw = _random_moves(n1, n2, 300, maxstep, 11)
    J = oracle.deposit2(g, xa1, xa2, xb1, xb2, v3, qw)
    ra = oracle.rho2(g, xa1, xa2, qw)
    rb = oracle.rho2(g, np.mod(xb1, n1), np.mod(xb2, n2), qw)
    res = (rb - ra) / dt + _div(J, dx1, dx2)
    scale = np.abs(rb - ra).max() / dt
    assert np.abs(res).max() <= 1e-13 * scale


def test_fp64_first_moment_and_rest():
    n1, n2, dx1, dx2, dt = 16, 12, 0.1, 0.2, 0.05
    g = oracle.grid2(n1, n2, dx1, dx2, dt)
    xa1, xa2, xb1, xb2, v3, qw = _random_moves(n1, n2, 50, 0.8, 12)
    for p in range(50):
        sl = slice(p, p + 1)
        J = oracle.deposit2(g, xa1[sl], xa2[sl], xb1[sl], xb2[sl], v3[sl], qw[sl])
        v1 = (xb1[p] - xa1[p]) * dx1 / dt
        v2 = (xb2[p] - xa2[p]) * dx2 / dt
        assert abs(J[0].sum() - qw[p] * v1) < 1e-12 * (1 + abs(qw[p] * v1))
        assert abs(J[1].sum() - qw[p] * v2) < 1e-12 * (1 + abs(qw[p] * v2))
        assert abs(J[2].sum() - qw[p] * v3[p]) < 1e-13
    # at rest: no in-plane current, and j3 = q w v3 times the charge shape
    J = oracle.deposit2(g, xa1, xa2, xa1, xa2, v3, qw)
    assert np.abs(J[:2]).max() == 0.0
    assert np.abs(J[2] - oracle.rho2(g, xa1, xa2, qw * v3)).max() < 1e-13


def test_fp64_time_reversal():
    n1, n2 = 16, 12
    g = oracle.grid2(n1, n2, 0.1, 0.2, 0.05)
    xa1, xa2, xb1, xb2, v3, qw = _random_moves(n1, n2, 100, 0.7, 13)
    Jf = oracle.deposit2(g, xa1, xa2, xb1, xb2, v3, qw)
    Jr = oracle.deposit2(g, xb1, xb2, xa1, xa2, v3, qw)
    assert np.abs(Jf[:2] + Jr[:2]).max() < 1e-12
    assert np.abs(Jf[2] - Jr[2]).max() < 1e-13


def test_fp64_rejects_long_moves():
    g = oracle.grid2(8, 8, 0.1, 0.1, 0.05)
    with pytest.raises(ValueError):
        oracle.deposit2(g, [1.0], [1.0], [2.0], [1.0], [0.0], [1.0])


# ------------------------------------------------------------- fixed point
P_BITS = 20


def _split(xi):
    """Cell index and FP32 offset of a position in cell units."""
    c = np.floor(xi).astype(np.int64)
    f = (xi - c).astype(np.float32)
    over = f >= np.float32(1.0)
    c[over] += 1
    f[over] = 0.0
    return c.astype(np.int32), f


def _fixed_case(n1, n2, npart, maxstep, seed, edge=False):
    xa1, xa2, xb1, xb2, v3, qw = _random_moves(n1, n2, npart, maxstep, seed)
    if edge:
        # offsets on and next to the node-switch point, cell edges and the seam
        special = np.array([0.0, 0.5, np.nextafter(0.5, 0), np.nextafter(0.5, 1), 0.25, 0.75,
                            np.nextafter(1.0, 0), 1e-9])
        k = len(special)
        xa1[:k] = 3 + special
        xb1[:k] = 3 + special[::-1] + 0.4
        xa2[k:2 * k] = (n2 - 1) + special
        xb2[k:2 * k] = (n2 - 1) + special + 0.3
    ca1, fa1 = _split(np.mod(xa1, n1))
    ca2, fa2 = _split(np.mod(xa2, n2))
    cb1, fb1 = _split(np.mod(xb1, n1))
    cb2, fb2 = _split(np.mod(xb2, n2))
    return ca1, ca2, fa1, fa2, cb1, cb2, fb1, fb2, v3.astype(np.float32), qw.astype(np.float32)


@pytest.mark.parametrize("seed,maxstep,edge", [(21, 0.45, False), (22, 0.99, False),
                                               (23, 0.45, True)])
def test_fixed_integer_continuity_exact(seed, maxstep, edge):
    n1, n2 = 16, 8
    ca1, ca2, fa1, fa2, cb1, cb2, fb1, fb2, v3, qw = _fixed_case(n1, n2, 400, maxstep, seed, edge)
    qmax = np.abs(qw).max()
    inv_wunit = np.float32(2.0 ** 15 / qmax)
    c3 = np.float32(2.0 ** (30 - 15 - 2 * P_BITS) / 6.0)
    J = oracle.deposit2_fixed(n1, n2, P_BITS, inv_wunit, c3, ca1, ca2, fa1, fa2, cb1, cb2, fb1,
                              fb2, v3, qw)
    ra = oracle.rho2_fixed(n1, n2, P_BITS, inv_wunit, ca1, ca2, fa1, fa2, qw)
    rb = oracle.rho2_fixed(n1, n2, P_BITS, inv_wunit, cb1, cb2, fb1, fb2, qw)
    div = (J[0] - np.roll(J[0], 1, axis=1)) + (J[1] - np.roll(J[1], 1, axis=0))
    assert np.array_equal(2 * (rb - ra), div)
    # total charge is an exact integer invariant
    assert ra.sum() == rb.sum()


def test_fixed_matches_fp64_within_quantisation():
    n1, n2, dx1, dx2, dt = 16, 8, 0.1, 0.2, 0.045
    ca1, ca2, fa1, fa2, cb1, cb2, fb1, fb2, v3, qw = _fixed_case(n1, n2, 400, 0.45, 24)
    # weights on the 2^-15 grid of the largest, so the integer charge is exact
    qmax = np.float32(np.abs(qw).max())
    qw = (np.round(qw / qmax * 2 ** 15) * qmax / 2 ** 15).astype(np.float32)
    inv_wunit = np.float32(2.0 ** 15 / qmax)
    c3 = np.float32(2.0 ** (30 - 15 - 2 * P_BITS) / 6.0)
    Ji = oracle.deposit2_fixed(n1, n2, P_BITS, inv_wunit, c3, ca1, ca2, fa1, fa2, cb1, cb2, fb1,
                               fb2, v3, qw)
    wunit = 1.0 / float(inv_wunit)
    j1 = -(dx1 / dt) * wunit * Ji[0] / 2.0 ** (2 * P_BITS + 1)
    j2 = -(dx2 / dt) * wunit * Ji[1] / 2.0 ** (2 * P_BITS + 1)
    j3 = Ji[2] / (float(inv_wunit) * float(c3) * 6.0 * 2.0 ** (2 * P_BITS))
    # the same motion in FP64 (unwrapped new position = old + wrapped difference)
    d1 = np.mod(cb1 - ca1 + n1 // 2, n1) - n1 // 2
    d2 = np.mod(cb2 - ca2 + n2 // 2, n2) - n2 // 2
    xa1 = ca1 + fa1.astype(np.float64)
    xa2 = ca2 + fa2.astype(np.float64)
    xb1 = ca1 + d1 + fb1.astype(np.float64)
    xb2 = ca2 + d2 + fb2.astype(np.float64)
    g = oracle.grid2(n1, n2, dx1, dx2, dt)
    J = oracle.deposit2(g, xa1, xa2, xb1, xb2, v3.astype(np.float64), qw.astype(np.float64))
    # each particle touches a node with shape errors of at most ~2^-P per factor
    per = 4 * 2.0 ** -P_BITS * np.abs(qw).max()
    count = 400
    assert np.abs(j1 - J[0]).max() <= per * (dx1 / dt) * count ** 0.5 * 4
    assert np.abs(j2 - J[1]).max() <= per * (dx2 / dt) * count ** 0.5 * 4
    assert np.abs(j3 - J[2]).max() <= per * count ** 0.5 * 4
    # and the relative L2 difference is at the level of the quantisation
    for a, b in ((j1, J[0]), (j2, J[1]), (j3, J[2])):
        assert np.linalg.norm(a - b) <= 2e-5 * np.linalg.norm(b)


def test_fixed_shape_factors_round_to_nearest():
    """The quantised shape factors are the quadratic B-spline weights times 2^P
    rounded to integers: each is within one unit of 2^P S (half a unit from
    quantising the offset, half from the final rounding) and the errors are
    unbiased.  Column sums of the integer density of isolated unit-charge
    particles give s1 times 2^P exactly, since the x2 factors sum to 2^P."""
    npart, spacing = 20000, 4
    n1, n2 = npart * spacing, 4
    gen = np.random.default_rng(31)
    f1 = gen.random(npart).astype(np.float32)
    c1 = (np.arange(npart) * spacing + 1).astype(np.int32)
    c2 = np.ones(npart, dtype=np.int32)
    f2 = gen.random(npart).astype(np.float32)
    qw = np.ones(npart, dtype=np.float32)
    rho = oracle.rho2_fixed(n1, n2, P_BITS, np.float32(1.0), c1, c2, f1, f2, qw)
    col = rho.sum(axis=0).reshape(npart, spacing) / 2.0 ** P_BITS   # integers s1 per node
    assert np.array_equal(col, np.round(col))
    xi = c1 + f1.astype(np.float64)
    nodes = np.arange(n1).reshape(npart, spacing)
    delta = xi[:, None] - nodes
    a = np.abs(delta)
    exact = np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    err = col - exact * 2.0 ** P_BITS
    side = (a >= 0.5) & (a < 1.5)
    assert np.abs(err[side]).max() <= 1.0 + 1e-9
    assert abs(err[side].mean()) < 0.02
    assert np.array_equal(col.sum(axis=1), np.full(npart, 2.0 ** P_BITS))


@pytest.mark.parametrize("seed,maxstep", [(41, 0.45), (42, 0.99)])
def test_fp64_matches_column_sum_of_3d_deposit(seed, maxstep):
    """The 2D current of a move with out-of-plane velocity v3 is the 3D
    Esirkepov current of the same move, with x3 advanced by v3 dt, summed over
    a periodic x3 column (both are q w v S with w the density weight).  The 3D
    deposit is pinned independently by 3D continuity, which fixes all three of
    its weights; summed over x3 its W3 bracket gives the 2D out-of-plane weight
    1/3 S0 S0 + 1/6 S1 S0 + 1/6 S0 S1 + 1/3 S1 S1 (Sec. 2.3, Esirkepov's
    decomposition), and its W1, W2 the in-plane weights.  A wrong 2D W3 such
    as (S0 S0 + S1 S1)/2 or the midpoint product fails this, where the moment
    and time-reversal pins above do not."""
    n1, n2, n3 = 16, 12, 8
    dx1, dx2, dx3, dt = 0.1, 0.2, 0.25, 0.05
    xa1, xa2, xb1, xb2, v3, qw = _random_moves(n1, n2, 300, maxstep, seed)
    g2 = oracle.grid2(n1, n2, dx1, dx2, dt)
    J2 = oracle.deposit2(g2, xa1, xa2, xb1, xb2, v3, qw)
    gen = np.random.default_rng(seed + 100)
    xa3 = gen.uniform(0, n3, xa1.size)
    xb3 = xa3 + v3 * dt / dx3
    assert np.abs(xb3 - xa3).max() < 1
    g3 = oracle.grid3(n1, n2, n3, dx1, dx2, dx3, dt)
    J3 = oracle.deposit3(g3, np.stack([xa1, xa2, xa3]), np.stack([xb1, xb2, xb3]), qw)
    col = J3.sum(axis=1)
    scale = np.abs(J2).max()
    for c in range(3):
        assert np.abs(col[c] - J2[c]).max() <= 1e-13 * scale


@pytest.mark.parametrize("unit_charge", [True, False])
def test_fixed_matches_fp64_per_node(unit_charge):
    """The kernel-precision deposit against the FP64 Esirkepov deposit of the
    same FP32 positions, node by node: every node's difference is within the
    sum over the particles reaching it of their shape-quantisation and FP32
    rounding bounds (tests/deposit_bound.py derives them), and the bound is
    tight enough to matter: a few 1e-6 of the gross current |q w| v reaching
    the node with equal charges, 1e-4 with charges rounded to 15 bits."""
    from tests.deposit_bound import covered_sum, node_bounds
    n1, n2, dx1, dx2, dt = 16, 8, 0.1, 0.2, 0.045
    ca1, ca2, fa1, fa2, cb1, cb2, fb1, fb2, v3, qw = _fixed_case(n1, n2, 3000, 0.45, 25, True)
    if unit_charge:
        qw = np.full_like(qw, -0.75)
    qmax = np.float32(np.abs(qw).max())
    qbits = 0 if unit_charge else 15
    P = 22 if unit_charge else 20
    inv_wunit = np.float32(2.0 ** qbits / qmax)
    c3 = np.float32(2.0 ** (30 - qbits - 2 * P) / 6.0)
    Ji = oracle.deposit2_fixed(n1, n2, P, inv_wunit, c3, ca1, ca2, fa1, fa2, cb1, cb2, fb1,
                               fb2, v3, qw)
    wunit = 1.0 / float(inv_wunit)
    jf = np.stack([-(dx1 / dt) * wunit * Ji[0] / 2.0 ** (2 * P + 1),
                   -(dx2 / dt) * wunit * Ji[1] / 2.0 ** (2 * P + 1),
                   Ji[2] / (float(inv_wunit) * float(c3) * 6.0 * 2.0 ** (2 * P))])
    d1 = np.mod(cb1 - ca1 + n1 // 2, n1) - n1 // 2
    d2 = np.mod(cb2 - ca2 + n2 // 2, n2) - n2 // 2
    xa = np.stack([ca1 + fa1.astype(np.float64), ca2 + fa2.astype(np.float64)])
    xb = np.stack([ca1 + d1 + fb1.astype(np.float64), ca2 + d2 + fb2.astype(np.float64)])
    g = oracle.grid2(n1, n2, dx1, dx2, dt)
    J = oracle.deposit2(g, xa[0], xa[1], xb[0], xb[1], v3.astype(np.float64),
                        qw.astype(np.float64))
    bound = node_bounds(n1, n2, dx1, dx2, dt, xa, xb, qw, v3, P, inv_wunit, c3, unit_charge)
    aq = np.abs(qw.astype(np.float64))
    gross = [covered_sum(n1, n2, xa, xb, aq) * dx1 / dt, covered_sum(n1, n2, xa, xb, aq) * dx2 / dt,
             covered_sum(n1, n2, xa, xb, aq * np.abs(v3))]
    for c in range(3):
        assert np.all(np.abs(jf[c] - J[c]) <= bound[c])
        assert np.all(bound[c] <= (4e-6 if unit_charge else 1e-4) * gross[c])
