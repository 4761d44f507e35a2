"""The Lorentz-boosted laser wakefield set-up of Table 2 (Sec. 6) at full size
(8192 x 512 cells, gamma_b = 14, 16 777 216 particles, the laser launched by
the moving antenna), FP32 form, and the n1 = 8192 row transforms it needs:

* n1 = 8192 against the oracle (plasma and a moving antenna, a few steps);
* the full run to t' = 3955 (6400 steps) with the k1 filter: the antenna's
  laser has the boosted-frame amplitude a0 omega' on axis, a wake of the
  expected order forms behind it, and the plasma ahead of the laser stays
  quiet (no numerical Cherenkov noise, Sec. 6 reports none);
* the same run without the filter fills that region with NCI noise (seeded
  by the plasma's 1e-4 momentum spread, not by round-off).

The paper's comparisons (UPIC-EMMA, OSIRIS lab frame) are not available, so
the levels are parity unpinned: the thresholds are wide margins around the
measured values (laser amplitude within 5% of the closed form, wake between
0.03 and 0.2, quiet region below 1e-3 against above 1e-2 without the filter).
"""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("fp64", 1e-9)])
def test_n1_8192_with_antenna_matches_oracle(hpic, prec, tol):
    """Rows of 8192 points are transformed one component per block."""
    d = W.drift2d(8192, 8, 0.2, 0.2, 0.05, sub=(2, 1), gamma=5.0, sigma_u=0.1, jitter=True,
                  seed=77)
    ant = dict(x0=700.0, v=-0.8, t0=0.0, T=4.0, K0=1.0, omega=3.0, x2c=0.8, waist=0.5)
    sim = hpic.from_workload(d, prec)
    sim.set_antenna(0, **ant)
    g = oracle.grid2(8192, 8, 0.2, 0.2, 0.05, alpha=d["alpha"], jbg=d["jbg"])
    if prec == "fp32":
        raw = sim.particles_raw(0)
        o = np.argsort(raw["id"])
        xa = raw["cell"][:, o] + raw["off"][:, o].astype(np.float64)
        st = oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"][:, o], raw["qw"][o],
                           antenna=oracle.antenna(**ant))
    else:
        p = sim.particles(0)
        o = np.argsort(p["id"])
        st = oracle.State2(g, d["qm"], p["x"][0, o] / 0.2, p["x"][1, o] / 0.2, p["u"][:, o],
                           d["q"] * p["w"][o], antenna=oracle.antenna(**ant))
    sim.step(8)
    st.step(8)
    E, B = sim.fields(0)
    assert np.abs(st.E[2]).max() > 0.01  # the antenna's field is there
    assert np.abs(E - st.E).max() <= tol * np.abs(st.E).max()
    assert np.abs(B - st.B).max() <= tol * np.abs(st.B).max()
    dg = sim.diagnostics(0)
    assert dg["gauss_l2"] <= (3e-5 if prec == "fp32" else 1e-11) * dg["gauss_ref_l2"]
    sim.close()


@pytest.fixture(scope="module")
def lwfa_runs(hpic):
    d = W.lwfa_boosted()
    out = {}
    for alpha in (0.5, 1.0):
        sim = hpic.from_workload(d, "fp32", alpha=alpha)
        sim.use_graphs(True)
        sim.step(d["steps"])
        E, _ = sim.fields(0)
        out[alpha] = dict(E1=E[0, d["n"][1] // 2].copy(), E3=E[2, d["n"][1] // 2].copy(),
                          diag=sim.diagnostics(0))
        sim.close()
    return d, out


def test_lwfa_laser_and_wake(lwfa_runs):
    d, out = lwfa_runs
    r = out[0.5]
    lz = d["laser"]
    assert abs(np.abs(r["E3"]).max() / (lz["a0"] * lz["omega"]) - 1.0) < 0.05
    i3 = int(np.argmax(np.abs(r["E3"])))
    i1 = int(np.argmax(np.abs(r["E1"])))
    assert 0.03 < np.abs(r["E1"]).max() < 0.2
    # the wake trails the laser (both well inside the box)
    assert i1 < i3
    assert r["diag"]["gauss_l2"] < 1e-4 * r["diag"]["gauss_ref_l2"]


def test_lwfa_filter_keeps_the_plasma_quiet(lwfa_runs):
    _, out = lwfa_runs
    quiet = slice(2000, 7000)  # cells ahead of the laser, never reached by it
    assert np.abs(out[0.5]["E1"][quiet]).max() < 1e-3
    assert np.abs(out[1.0]["E1"][quiet]).max() > 1e-2
