"""The step replayed as captured HIP graphs gives the same results as the
same kernels launched one by one.

Each graph holds one particle sort and sort_interval steps.  The FP32 form is
deterministic (integer deposit), so the fields, the 64-bit current and every
particle must agree bit for bit after each replay; eager work (diagnostics,
field reads, extra single steps) runs between the replays.
"""
import numpy as np
import pytest

from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _state(sim, run=0):
    E, B = sim.fields(run)
    raw = sim.particles_raw(run)
    o = np.argsort(raw["id"])
    return E, B, sim.current_fixed(run), {k: v[..., o] for k, v in raw.items()}


def _same(a, b):
    Ea, Ba, Ja, Pa = a
    Eb, Bb, Jb, Pb = b
    assert np.array_equal(Ea, Eb)
    assert np.array_equal(Ba, Bb)
    assert np.array_equal(Ja, Jb)
    for k in Pa:
        assert np.array_equal(Pa[k], Pb[k]), k


@pytest.mark.parametrize("interval", [2, 4])
def test_graph_replays_equal_eager(hpic, interval):
    laser = dict(a0=2.0, waist=2.0, length=1.5, k0=10.0, x1c=0.6 * 128 * 0.1, x2c=0.5 * 32 * 0.2)
    d = W.drift2d(128, 32, 0.1, 0.2, 0.045, sub=(4, 2), gamma=20.0, sigma_u=0.05, jitter=True,
                  seed=W.SEED0 + 77, laser=laser, name="graph")
    g = hpic.from_workload(d, "fp32", sort_interval=interval)
    e = hpic.from_workload(d, "fp32", sort_interval=interval)
    e.use_graphs(False)
    # chunks: whole blocks (replays), ragged remainders (eager), more blocks
    for n in [interval, 3 * interval, 1, interval + 1, 2 * interval, 5, 4 * interval]:
        g.step(n)
        e.step(n)
        _same(_state(g), _state(e))
        # one more single step between replays, with its continuity residual
        for sim in (g, e):
            sim.diagnostics(0)
            sim.step(1)
        dg, de = g.diagnostics(0), e.diagnostics(0)
        assert dg["cont_int"] == 0 and de["cont_int"] == 0
        assert dg["step"] == de["step"]
    g.close()
    e.close()


def test_graph_batched_runs_and_reload(hpic):
    """Two runs in one handle; reloading particles (new work lists) drops the
    captured graphs and the next replays use the new lists."""
    a = W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=5.0, sigma_u=0.1, jitter=True, seed=5)
    b = W.drift2d(32, 24, 0.2, 0.2, 0.05, sub=(3, 1), gamma=50.0, sigma_u=0.1, jitter=True,
                  seed=6)

    def make(graphs):
        cfgs = [hpic.config(64, 16, 0.2, 0.2, 0.05, sort_interval=2),
                hpic.config(32, 24, 0.2, 0.2, 0.05, sort_interval=2)]
        sim = hpic.Sim(cfgs)
        sim.use_graphs(graphs)
        for r, w in enumerate((a, b)):
            sim.set_particles(r, w["xi"] * 0.2, w["u"], w["w"], w["qm"], w["q"])
        return sim

    g, e = make(True), make(False)
    for sim in (g, e):
        sim.step(6)
    for r in (0, 1):
        _same(_state(g, r), _state(e, r))
    # reload run 1 with fewer particles: work lists change size
    for sim in (g, e):
        pr = sim.particles(1)
        keep = np.argsort(pr["id"])[: pr["id"].size // 3]
        sim.set_particles(1, pr["x"][:, keep], pr["u"][:, keep], pr["w"][keep], b["qm"], b["q"])
        sim.step(8)
    for r in (0, 1):
        _same(_state(g, r), _state(e, r))
    g.close()
    e.close()
