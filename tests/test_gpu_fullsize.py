"""GPU parity at the benchmark size and on edge cases.

Full size: the 2048 x 512 laser workload (8 388 608 particles) in the launch
configuration bench.py times.  One step: the 64-bit deposit of every particle
is compared bit for bit with the oracle's fixed-point deposit of the same
moves; a random sample of particles is pushed by the oracle (FP64 gather and
Boris from the GPU's fields); the field update is compared with the oracle's
FP64 update of the same fields and current; integer continuity holds exactly.

Edge cases: an empty run batched with a loaded one, grids whose size is not a
multiple of the particle tile, the largest (n1 = 4096) and smallest (n1 = 8)
x1 transforms, particles on cell edges and periodic seams.
"""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W
from tests.deposit_bound import node_bounds

pytestmark = pytest.mark.gpu


def _v3_float32(u):
    u = u.astype(np.float32)
    s = np.float32(1) + u[0] * u[0]
    s = s + u[1] * u[1]
    s = s + u[2] * u[2]
    return u[2] * (np.float32(1) / np.sqrt(s))


def test_full_size_one_step(hpic):
    d = W.drift2d_laser()
    n1, n2 = d["n"][0], d["n"][1]
    sim = hpic.from_workload(d, "fp32")
    before = sim.particles_raw(0)
    E0, B0 = sim.fields(0)
    fp = sim.fixed_params(0)
    sim.diagnostics(0)
    sim.step(1)
    dg = sim.diagnostics(0)
    assert dg["cont_int"] == 0
    after = sim.particles_raw(0)
    E1, B1 = sim.fields(0)
    Jg = sim.current_fixed(0)
    assert np.array_equal(before["id"], after["id"])
    v3 = _v3_float32(after["u"])
    Jo = oracle.deposit2_fixed(n1, n2, fp["P"], fp["inv_wunit"], fp["c3"], before["cell"][0],
                               before["cell"][1], before["off"][0], before["off"][1],
                               after["cell"][0], after["cell"][1], after["off"][0],
                               after["off"][1], v3, before["qw"])
    assert np.array_equal(Jg, Jo)
    # sampled push
    gen = np.random.default_rng(77)
    idx = gen.choice(before["qw"].size, 20000, replace=False)
    xa = before["cell"][:, idx] + before["off"][:, idx].astype(np.float64)
    g = oracle.grid2(n1, n2, d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"], jbg=d["jbg"])
    Ep, Bp = oracle.gather2(g, E0, B0, xa[0], xa[1])
    u = oracle.boris(d["qm"], d["dt"], Ep, Bp, before["u"][:, idx].astype(np.float64))
    assert np.abs(after["u"][:, idx] - u).max() <= 8e-6 * (1 + np.abs(u).max())
    # field update with the FP64 Esirkepov current of the GPU's moves
    step = after["cell"] - before["cell"]
    step[0] = (step[0] + n1 // 2) % n1 - n1 // 2
    step[1] = (step[1] + n2 // 2) % n2 - n2 // 2
    xall = before["cell"] + before["off"].astype(np.float64)
    xb = before["cell"] + step + after["off"].astype(np.float64)
    J64 = oracle.deposit2(g, xall[0], xall[1], xb[0], xb[1], v3.astype(np.float64),
                          before["qw"].astype(np.float64))
    # the GPU current against that FP64 current, node by node, within the
    # shape quantisation and FP32 rounding of the particles reaching the node
    bound = node_bounds(n1, n2, d["dx"][0], d["dx"][1], d["dt"], xall, xb, before["qw"], v3,
                        fp["P"], fp["inv_wunit"], fp["c3"], fp["Q"] == 0)
    for c in range(3):
        assert np.all(np.abs(sim.current(0, c) - d["jbg"][c] - J64[c]) <= bound[c])
    Eo, Bo = oracle.field_update2(g, E0, B0, J64)
    scale = max(np.abs(Eo).max(), np.abs(Bo).max())
    assert np.abs(E1 - Eo).max() <= 2e-5 * scale
    assert np.abs(B1 - Bo).max() <= 2e-5 * scale
    sim.close()


def test_empty_run_in_batch(hpic):
    w = W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=10.0, sigma_u=1e-2, seed=31)
    cfgs = [hpic.config(64, 16, 0.2, 0.2, 0.05), hpic.config(32, 8, 0.2, 0.2, 0.05)]
    sim = hpic.Sim(cfgs)
    sim.set_particles(0, w["xi"] * 0.2, w["u"], w["w"], w["qm"], w["q"])
    sim.set_particles(1, np.zeros((2, 0)), np.zeros((3, 0)), np.zeros(0))
    E = np.zeros((3, 8, 32))
    E[2] = np.cos(2 * np.pi * np.arange(32) / 32)[None, :]
    sim.set_fields(1, E, np.zeros_like(E))
    sim.step(5)
    assert sim.count(1) == 0
    assert np.abs(sim.current_fixed(1)).max() == 0
    one = hpic.from_workload(w, "fp32", background=False)
    one.step(5)
    assert np.array_equal(one.current_fixed(0), sim.current_fixed(0))
    sim.close()
    one.close()


@pytest.mark.parametrize("n1,n2", [(64, 20), (8, 12), (128, 7)])
def test_ragged_tiles_match_oracle(hpic, n1, n2):
    """Grids that are not a multiple of the 32 x 8 particle tile."""
    d = W.drift2d(n1, n2, 0.2, 0.2, 0.05, sub=(2, 2), gamma=3.0, sigma_u=0.2, jitter=True,
                  seed=W.SEED0 + n1 + n2)
    sim = hpic.from_workload(d, "fp32")
    raw = sim.particles_raw(0)
    o = np.argsort(raw["id"])
    raw = {k: v[..., o] for k, v in raw.items()}
    g = oracle.grid2(n1, n2, 0.2, 0.2, 0.05, alpha=d["alpha"], jbg=d["jbg"])
    xa = raw["cell"] + raw["off"].astype(np.float64)
    st = oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"], raw["qw"])
    sim.step(6)
    st.step(6)
    E1, B1 = sim.fields(0)
    scale = max(np.abs(st.E).max(), 1e-3)
    assert np.abs(E1 - st.E).max() <= 1e-4 * scale
    sim.close()


@pytest.mark.parametrize("n1", [8, 4096])
def test_smallest_and_largest_transform(hpic, n1):
    n2, dx1, dx2 = 8, 0.1, 0.2
    dt = 0.9 * oracle.courant_limit2(dx1, dx2)
    sim = hpic.Sim([hpic.config(n1, n2, dx1, dx2, dt, alpha=1.0)])
    k1i = n1 // 4 - 1
    X1, X2 = np.meshgrid(np.arange(n1), np.arange(n2))
    E = np.zeros((3, n2, n1))
    E[2] = np.cos(2 * np.pi * (k1i * X1 / n1 + X2 / n2))
    sim.set_fields(0, E, np.zeros_like(E))
    sim.step(40)
    k1 = 2 * np.pi * k1i / (n1 * dx1)
    kk2 = np.sin(np.pi / n2) / (dx2 / 2)
    theta = 2 * np.arcsin(0.5 * dt * np.hypot(k1, kk2))
    assert np.abs(sim.field(0, 2) - np.cos(40 * theta) * E[2]).max() < 5e-5
    sim.close()


def test_cell_edges_and_seams(hpic):
    """Particles exactly on cell edges, on node-switch points and across the
    periodic seams move and deposit like the oracle's fixed-point definition."""
    n1, n2 = 32, 8
    sim = hpic.Sim([hpic.config(n1, n2, 0.1, 0.2, 0.045)])
    special = np.array([0.0, 0.5, 0.25, np.nextafter(np.float32(1.0), 0), 1e-7, 0.999])
    xs = []
    for c1 in (0, n1 - 1, 7):
        for c2 in (0, n2 - 1):
            for f in special:
                xs.append((c1 + f, c2 + special[::-1][len(xs) % len(special)]))
    xi = np.array(xs).T
    npart = xi.shape[1]
    gen = np.random.default_rng(3)
    u = np.stack([gen.choice([-5.0, 5.0], npart), gen.choice([-2.0, 2.0], npart),
                  gen.standard_normal(npart)])
    sim.set_particles(0, xi * np.array([[0.1], [0.2]]), u, np.full(npart, 0.125))
    before = sim.particles_raw(0)
    fp = sim.fixed_params(0)
    sim.step(1)
    after = sim.particles_raw(0)
    o1, o2 = np.argsort(before["id"]), np.argsort(after["id"])
    b = {k: v[..., o1] for k, v in before.items()}
    a = {k: v[..., o2] for k, v in after.items()}
    Jo = oracle.deposit2_fixed(n1, n2, fp["P"], fp["inv_wunit"], fp["c3"], b["cell"][0],
                               b["cell"][1], b["off"][0], b["off"][1], a["cell"][0], a["cell"][1],
                               a["off"][0], a["off"][1], _v3_float32(a["u"]), b["qw"])
    assert np.array_equal(sim.current_fixed(0), Jo)
    assert np.all((a["off"] >= 0) & (a["off"] < 1))
    sim.close()
