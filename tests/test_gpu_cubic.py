"""The cubic particle shape (2D, hp_config.shape_order = 3) on the GPU against
the oracle's cubic step (pinned by the spline moments, continuity and the work
identity): both forms over whole steps, with the energy-conserving gather,
the Gauss residual kept, results independent of the sort interval (the FP32
accumulation is order-independent), and the 2048 x 512 laser workload at full
size (sampled particles against the oracle's gather and push)."""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _small(seed=31):
    return W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=5.0, sigma_u=0.1, jitter=True,
                     seed=seed)


def _oracle_state(sim, d, prec, interp=0):
    g = oracle.grid2(d["n"][0], d["n"][1], d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                     jbg=d["jbg"], interp=interp, shape=3)
    if prec == "fp32":
        raw = sim.particles_raw(0)
        o = np.argsort(raw["id"])
        xa = raw["cell"][:, o] + raw["off"][:, o].astype(np.float64)
        return oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"][:, o], raw["qw"][o])
    p = sim.particles(0)
    o = np.argsort(p["id"])
    return oracle.State2(g, d["qm"], p["x"][0, o] / d["dx"][0], p["x"][1, o] / d["dx"][1],
                         p["u"][:, o], d["q"] * p["w"][o])


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("fp64", 1e-9)])
@pytest.mark.parametrize("interp", [0, 1])
def test_cubic_steps_match_oracle(hpic, prec, tol, interp):
    d = _small()
    sim = hpic.from_workload(d, prec, shape=3, interp=interp)
    st = _oracle_state(sim, d, prec, interp)
    sim.step(20)
    st.step(20)
    E1, B1 = sim.fields(0)
    scale = max(np.abs(st.E).max(), 1e-3)
    assert np.abs(E1 - st.E).max() <= tol * scale
    assert np.abs(B1 - st.B).max() <= tol * max(np.abs(st.B).max(), 1e-3)
    p = sim.particles(0)
    o = np.argsort(p["id"])
    assert np.abs(p["u"][:, o] - st.u).max() <= tol * max(1.0, np.abs(st.u).max())
    if prec == "fp64":
        for c in range(3):
            jc = sim.current(0, c) - d["jbg"][c]
            assert np.abs(jc - st.J[c]).max() <= 1e-9 * (np.abs(st.J[c]).max() + 1e-30) + 1e-14
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 3e-5), ("fp64", 1e-11)])
def test_cubic_gauss_and_continuity(hpic, prec, tol):
    d = _small(seed=32)
    sim = hpic.from_workload(d, prec, shape=3)
    sim.step(30)
    dg = sim.diagnostics(0)
    assert dg["gauss_ref_l2"] > 0
    assert dg["gauss_l2"] <= tol * dg["gauss_ref_l2"]
    sim.step(1)
    dc = sim.diagnostics(0)
    if prec == "fp32":
        # integer weights with exact sums: continuity holds exactly in the integers
        assert dc["cont_int"] == 0
    else:
        assert 0 <= dc["cont_linf"] <= 1e-10
    sim.close()


def test_cubic_independent_of_sort_interval(hpic):
    d = _small(seed=33)
    out = []
    for k in (4, 16):
        sim = hpic.from_workload(d, "fp32", shape=3, sort_interval=k)
        sim.step(24)
        out.append((sim.fields(0)[0], sim.current_fixed(0)))
        sim.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_cubic_full_size_sampled(hpic):
    d = W.drift2d_laser()
    sim = hpic.from_workload(d, "fp32", shape=3)
    E0, B0 = sim.fields(0)
    raw = sim.particles_raw(0)
    gen = np.random.default_rng(3)
    idx = gen.choice(raw["qw"].size, 500, replace=False)
    xa = raw["cell"][:, idx] + raw["off"][:, idx].astype(np.float64)
    g = oracle.grid2(d["n"][0], d["n"][1], d["dx"][0], d["dx"][1], d["dt"], shape=3)
    Ep, Bp = oracle.gather2(g, E0, B0, xa[0], xa[1])
    u1, u2, u3 = (np.ascontiguousarray(raw["u"][c, idx].astype(np.float64)) for c in range(3))
    oracle.lib().or_boris(len(idx), d["qm"], d["dt"], oracle._p(np.ascontiguousarray(Ep)),
                          oracle._p(np.ascontiguousarray(Bp)), oracle._p(u1), oracle._p(u2),
                          oracle._p(u3))
    ids = raw["id"][idx]
    sim.step(1)
    raw1 = sim.particles_raw(0)
    pos = {int(v): k for k, v in enumerate(raw1["id"])}
    k1 = np.array([pos[int(v)] for v in ids])
    uo = np.stack([u1, u2, u3])
    assert np.abs(raw1["u"][:, k1] - uo).max() <= 2e-5 * np.abs(uo).max()
    d0 = sim.diagnostics(0)
    sim.step(5)
    d1 = sim.diagnostics(0)
    assert d1["gauss_l2"] <= 1e-4 * max(d1["gauss_ref_l2"], 1e-30) + d0["gauss_l2"]
    sim.close()


def test_cubic_state_resume_bitexact(hpic):
    """Checkpoint and resume of a cubic-shape run (FP32 form): the same bits
    as the uninterrupted run, diagnostics included."""
    d = _small(seed=34)
    a = hpic.from_workload(d, "fp32", shape=3)
    a.step(3)
    blob = a.get_state()
    a.step(4)
    Ea, Ba = a.fields(0)
    ja = a.current_fixed(0)
    b = hpic.from_workload(d, "fp32", shape=3)
    b.set_state(blob)
    b.step(4)
    Eb, Bb = b.fields(0)
    assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
    assert np.array_equal(ja, b.current_fixed(0))
    da, db = a.diagnostics(0), b.diagnostics(0)
    assert da["gauss_l2"] == db["gauss_l2"] and da["charge_total"] == db["charge_total"]
    a.close()
    b.close()
