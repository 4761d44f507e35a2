"""Tile shape, sort interval and the autotuner change only the speed: the FP32
form's fields, 64-bit current and particles are bit-identical for every
setting (integer deposit), including tiles whose particles do not fit the LDS
budget (global-memory fallback of the push)."""
import numpy as np
import pytest

from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _workload():
    laser = dict(a0=2.0, waist=2.0, length=1.5, k0=10.0, x1c=0.6 * 128 * 0.1, x2c=0.5 * 40 * 0.2)
    return W.drift2d(128, 40, 0.1, 0.2, 0.045, sub=(4, 2), gamma=20.0, sigma_u=0.05, jitter=True,
                     seed=W.SEED0 + 55, laser=laser, name="tiling")


def _state(sim):
    E, B = sim.fields(0)
    raw = sim.particles_raw(0)
    o = np.argsort(raw["id"])
    return [E, B, sim.current_fixed(0)] + [v[..., o] for _, v in sorted(raw.items())]


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.fixture(scope="module")
def reference(hpic):
    d = _workload()
    sim = hpic.from_workload(d, "fp32")
    sim.step(24)
    ref = _state(sim)
    sim.close()
    return d, ref


@pytest.mark.parametrize("t1,t2,K", [(64, 4, 8), (16, 16, 2), (7, 3, 5), (128, 2, 1),
                                     (1, 1, 4), (128, 40, 6)])
def test_tiling_invariance(hpic, reference, t1, t2, K):
    d, ref = reference
    sim = hpic.from_workload(d, "fp32")
    sim.set_tiling(t1, t2, K)
    t = sim.tiling()
    assert t["tile"] == (t1, t2) and t["sort_interval"] == K
    sim.step(24)
    _same(_state(sim), ref)
    if (t1, t2) == (128, 40):
        # the whole grid as one tile exceeds the LDS budget: global fallback
        assert sim.push_stats()["fallback_tiles"] > 0
    sim.close()


def test_autotune_advances_exactly(hpic, reference):
    d, ref = reference
    sim = hpic.from_workload(d, "fp32")
    tune = sim.autotune(24)
    assert tune["steps"] == 24 and tune["candidates"] >= 1
    assert tune["sort_interval"] >= 1 and tune["lds_bytes"] >= 16384
    assert sim.diagnostics(0)["step"] == 24
    _same(_state(sim), ref)
    sim.close()


def test_autotune_then_steps(hpic):
    """A full tuning pass (all candidates) on a batch of scan runs, then more
    steps with the chosen setting, equals plain steps."""
    ds = W.scan2d(nruns=6, shrink=8)
    a = hpic.from_workloads(ds, "fp32")
    b = hpic.from_workloads(ds, "fp32")
    tune = a.autotune(600)
    assert tune["candidates"] >= 4
    a.step(10)
    b.step(610)
    for r in range(len(ds)):
        Ea, Ba = a.fields(r)
        Eb, Bb = b.fields(r)
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
        assert np.array_equal(a.current_fixed(r), b.current_fixed(r))
    a.close()
    b.close()


def test_set_tiling_rejects_bad_values(hpic):
    sim = hpic.from_workload(_workload(), "fp32")
    for bad in [(0, 8, 16), (32, 0, 16), (32, 8, 0), (5000, 8, 16), (32, 8, 2000)]:
        with pytest.raises(hpic.HpError):
            sim.set_tiling(*bad)
    sim.close()
