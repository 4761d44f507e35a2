"""Per-node error bound of the 64-bit fixed-point deposit against the plain
FP64 Esirkepov deposit of the same moves (Sec. 2.3).

The fixed-point deposit quantises each quadratic shape factor to an integer
multiple of 2^-P: the two outer factors of a particle's three are within one
unit of 2^P S, the middle one takes the remainder so that the three sum to 2^P
exactly, so every factor is within eps = 2 units.  For one particle and one
node (a = position in the x1 window):

* j1 weight W1 = C1 A2 / 2 with C1 the running sum of S1 - S0 along x1
  (|C1| <= 1; its error is at most min(a + 1, 3 - a) 2 eps <= 4 eps, counting
  the sum from either end, since both shape sums are exact) and A2 = S0 + S1
  along x2 (<= 1.5, error <= 2 eps): |dW1| <= 4 eps 0.75 + 2 eps / 2 = 4 eps,
  i.e. 8 units, times |q w| dx1/dt.  j2 alike with dx2/dt.  Unequal charges
  add the rounding of the integer charge, half a unit of wunit.
* j3 weight W3 = (S0x S0y + S1x S1y)/3 + (S1x S0y + S0x S1y)/6: each product of
  factors <= 0.75 moves by <= 1.5 eps, so |dW3| <= 1.5 eps = 3 units, times
  |q w v3|; the FP32 evaluation (charge scale, h = q w v3 c3, two products, one
  fused multiply-add, all terms of one sign) adds 8 ulp relative, and the
  final rounding to an integer half a unit of the j3 scale.

A node's bound is the sum of these over the particles whose 4 x 4 window
(first node min(nearest node before, after) - 1 along each axis) covers it.
"""
import numpy as np


def window_origin(x):
    """First node of the 4-node deposit window along one axis for moves
    x[0] -> x[1] (cell units, x[1] unwrapped)."""
    na = np.floor(x[0] + 0.5).astype(np.int64)
    nb = np.floor(x[1] + 0.5).astype(np.int64)
    return np.minimum(na, nb) - 1


def covered_sum(n1, n2, xa, xb, weight):
    """sum over particles of weight[p] at every node of the particle's 4 x 4
    window, on the periodic n2 x n1 grid."""
    b1 = window_origin((xa[0], xb[0]))
    b2 = window_origin((xa[1], xb[1]))
    out = np.zeros(n1 * n2)
    for j in range(4):
        r = np.mod(b2 + j, n2) * n1
        for i in range(4):
            out += np.bincount(r + np.mod(b1 + i, n1), weights=weight, minlength=n1 * n2)
    return out.reshape(n2, n1)


def node_bounds(n1, n2, dx1, dx2, dt, xa, xb, qw, v3, P, inv_wunit, c3, unit_charge):
    """Bounds [3][n2][n1] of |j_fixed - j_fp64| per node and component."""
    unit = 2.0 ** -P
    wunit = 1.0 / float(inv_wunit)
    aq = np.abs(qw.astype(np.float64))
    qround = 0.0 if unit_charge else 0.5 * wunit
    per12 = 8 * unit * aq + qround
    j3_unit = 1.0 / (float(inv_wunit) * float(c3) * 6.0 * 2.0 ** (2 * P))
    per3 = aq * np.abs(v3.astype(np.float64)) * (3 * unit + 8 * 2.0 ** -24) + 0.5 * j3_unit
    return np.stack([covered_sum(n1, n2, xa, xb, per12) * (dx1 / dt),
                     covered_sum(n1, n2, xa, xb, per12) * (dx2 / dt),
                     covered_sum(n1, n2, xa, xb, per3)])
