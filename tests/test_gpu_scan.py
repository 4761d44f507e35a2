"""The batched parameter scan: many independent runs of uneven grid sizes
advanced together, one launch per stage, replayed as HIP graphs.

Small version (grids divided by 8): every run of the batch equals the same run
advanced alone bit for bit, a few runs follow the oracle's FP64 step, and the
integer continuity residual of every run is exactly zero.  Full size (64 runs,
about 1.6e8 particles): one step in the launch configuration of the benchmark,
with the deposit of the smallest runs compared bit for bit with the oracle's
fixed-point deposit and exact continuity in every run.
"""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _v3_float32(u):
    u = u.astype(np.float32)
    s = np.float32(1) + u[0] * u[0]
    s = s + u[1] * u[1]
    s = s + u[2] * u[2]
    return u[2] * (np.float32(1) / np.sqrt(s))


def _fields_by_id(sim, r):
    E, B = sim.fields(r)
    return E, B, sim.current_fixed(r)


def test_scan_small_batch_equals_single_runs(hpic):
    ds = W.scan2d(nruns=16, shrink=8)
    sim = hpic.from_workloads(ds, "fp32")
    sim.step(39)
    for r in range(len(ds)):
        sim.diagnostics(r)
    sim.step(1)
    for r in range(len(ds)):
        assert sim.diagnostics(r)["cont_int"] == 0
    for r in (0, 5, 11, 15):
        one = hpic.from_workload(ds[r], "fp32")
        one.step(40)
        a, b = _fields_by_id(sim, r), _fields_by_id(one, 0)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), r
        one.close()
    sim.close()


@pytest.mark.parametrize("run", [2, 9])
def test_scan_small_runs_follow_oracle(hpic, run):
    ds = W.scan2d(nruns=16, shrink=8)
    sim = hpic.from_workloads(ds, "fp32")
    d = ds[run]
    raw = sim.particles_raw(run)
    o = np.argsort(raw["id"])
    raw = {k: v[..., o] for k, v in raw.items()}
    g = oracle.grid2(d["n"][0], d["n"][1], d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                     jbg=d["jbg"])
    xa = raw["cell"] + raw["off"].astype(np.float64)
    st = oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"], raw["qw"])
    sim.step(10)
    st.step(10)
    E1, B1 = sim.fields(run)
    scale = max(np.abs(st.E).max(), np.abs(st.B).max())
    assert np.abs(E1 - st.E).max() <= 1e-4 * scale
    assert np.abs(B1 - st.B).max() <= 1e-4 * scale
    sim.close()


def test_scan_full_size_one_step(hpic):
    params = W.scan2d_params()
    ds = [W.scan2d_run(p) for p in params]
    sim = hpic.from_workloads(ds, "fp32")
    small = sorted(range(len(ds)), key=lambda r: ds[r]["w"].size)[:2]
    before = {r: sim.particles_raw(r) for r in small}
    fp = {r: sim.fixed_params(r) for r in small}
    for r in range(len(ds)):
        sim.diagnostics(r)
    sim.step(1)
    for r in range(len(ds)):
        assert sim.diagnostics(r)["cont_int"] == 0, r
    for r in small:
        n1, n2 = ds[r]["n"][0], ds[r]["n"][1]
        b, a = before[r], sim.particles_raw(r)
        assert np.array_equal(b["id"], a["id"])
        Jo = oracle.deposit2_fixed(n1, n2, fp[r]["P"], fp[r]["inv_wunit"], fp[r]["c3"],
                                   b["cell"][0], b["cell"][1], b["off"][0], b["off"][1],
                                   a["cell"][0], a["cell"][1], a["off"][0], a["off"][1],
                                   _v3_float32(a["u"]), b["qw"])
        assert np.array_equal(sim.current_fixed(r), Jo), r
    # a few more steps through the captured graphs stay exact
    sim.step(31)
    for r in range(len(ds)):
        sim.diagnostics(r)
    sim.step(1)
    for r in range(len(ds)):
        assert sim.diagnostics(r)["cont_int"] == 0, r
    sim.close()
