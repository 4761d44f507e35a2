"""The moving antenna (hp_set_antenna) on the GPU against the oracle's
(pinned by the jump conditions of a moving current sheet): a plasma run with
a moving, Gaussian-profiled antenna in both forms, identical results for
eager and graph-replayed steps (the antenna's time comes from a device step
counter), a checkpoint resumed with the antenna set again, and the argument
checks."""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu

ANT = dict(x0=9.0, v=-0.6, t0=0.2, T=6.0, K0=0.7, omega=4.0, phase=0.3, x2c=1.5, waist=0.9)


def _setup(hpic, prec, seed=41, graphs=False):
    d = W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=3.0, sigma_u=0.1, jitter=True,
                  seed=seed)
    sim = hpic.from_workload(d, prec)
    sim.use_graphs(graphs)
    sim.set_antenna(0, **ANT)
    return d, sim


def _oracle(d, sim, prec):
    g = oracle.grid2(64, 16, 0.2, 0.2, 0.05, alpha=d["alpha"], jbg=d["jbg"])
    a = oracle.antenna(**ANT)
    if prec == "fp32":
        raw = sim.particles_raw(0)
        o = np.argsort(raw["id"])
        xa = raw["cell"][:, o] + raw["off"][:, o].astype(np.float64)
        return oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"][:, o], raw["qw"][o], antenna=a)
    p = sim.particles(0)
    o = np.argsort(p["id"])
    return oracle.State2(g, d["qm"], p["x"][0, o] / 0.2, p["x"][1, o] / 0.2, p["u"][:, o],
                         d["q"] * p["w"][o], antenna=a)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("fp64", 1e-9)])
def test_antenna_run_matches_oracle(hpic, prec, tol):
    d, sim = _setup(hpic, prec)
    st = _oracle(d, sim, prec)
    sim.step(120)
    st.step(120)
    E, B = sim.fields(0)
    assert np.abs(st.E[2]).max() > 0.05  # the antenna's wave is there
    scale = np.abs(st.E).max()
    assert np.abs(E - st.E).max() <= tol * scale
    assert np.abs(B - st.B).max() <= tol * max(np.abs(st.B).max(), 1e-3)
    if prec == "fp64":
        j3 = sim.current(0, 2) - d["jbg"][2]
        assert np.abs(j3 - st.J[2]).max() <= 1e-9 * np.abs(st.J[2]).max() + 1e-14
    sim.close()


def test_antenna_graphs_equal_eager(hpic):
    out = []
    for graphs in (False, True):
        _, sim = _setup(hpic, "fp32", graphs=graphs)
        sim.step(48)
        out.append(sim.fields(0)[0])
        sim.close()
    assert np.array_equal(out[0], out[1])


def test_antenna_checkpoint_resume(hpic):
    _, a = _setup(hpic, "fp32", graphs=True)
    a.step(30)
    blob = a.get_state()
    a.step(34)
    Ea = a.fields(0)[0]
    _, b = _setup(hpic, "fp32", graphs=True)
    b.set_state(blob)
    b.set_antenna(0, **ANT)
    b.step(34)
    assert np.array_equal(Ea, b.fields(0)[0])
    # removing the antenna changes the result from then on
    _, c = _setup(hpic, "fp32")
    c.set_state(blob)
    c.set_antenna(0, None)
    c.step(34)
    assert not np.array_equal(Ea, c.fields(0)[0])
    a.close()
    b.close()
    c.close()


def test_antenna_arguments(hpic):
    _, sim = _setup(hpic, "fp32")
    for bad in (dict(v=1.0), dict(v=-1.5), dict(T=0.0), dict(K0=float("nan"))):
        kw = dict(ANT)
        kw.update(bad)
        with pytest.raises(hpic.HpError):
            sim.set_antenna(0, **kw)
    sim.close()
    s3 = hpic.Sim([hpic.config(16, 8, 0.2, 0.2, 0.05, n3=8, dx3=0.2)])
    with pytest.raises(hpic.HpError):
        s3.set_antenna(0, **ANT)
    s3.close()
    sq = hpic.Sim([hpic.config(16, 8, 0.2, 0.2, 0.05, modes=2)])
    with pytest.raises(hpic.HpError):
        sq.set_antenna(0, **ANT)
    sq.close()
