"""GPU parity: the HIP path against the FP64 CPU oracle on identical seeded inputs.

Tolerances (FP32 form) follow from the arithmetic: FP32 rounds each operation
to 2^-24 ~ 6e-8 relative; a quadratic gather sums 9 terms, Boris takes ~20
dependent operations, so momenta agree to ~1e-6 relative and positions to
~1e-6 cells per step; a radix-4 FP32 FFT of length 2^k adds ~k eps relative
error per transform, so a field update (forward + inverse) agrees to ~1e-5 of
the field magnitude.  The fixed-point deposit is bit-exact against the oracle's
fixed-point definition (same integers), and the FP64 form agrees with the
oracle to ~1e-10 after 100 steps.
"""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W
from tests.deposit_bound import node_bounds

pytestmark = pytest.mark.gpu


def _oracle_grid(sim, run=0, jbg=(0.0, 0.0, 0.0), **kw):
    c = sim.cfgs[run]
    return oracle.grid2(c.n[0], c.n[1], c.dx[0], c.dx[1], c.dt, alpha=c.filter_frac,
                        deriv1=c.deriv1, correct=c.correct, jbg=jbg, **kw)


def _v3_float32(u):
    """Out-of-plane velocity in FP32 with the kernel's operation order:
    g = sqrt(((1 + u1 u1) + u2 u2) + u3 u3), v3 = u3 * (1/g), each op rounded once."""
    u = u.astype(np.float32)
    s = np.float32(1) + u[0] * u[0]
    s = s + u[1] * u[1]
    s = s + u[2] * u[2]
    return u[2] * (np.float32(1) / np.sqrt(s))


def _moves(n1, n2, npart, seed, edge=True):
    gen = np.random.default_rng(seed)
    c0 = np.stack([gen.integers(0, n1, npart), gen.integers(0, n2, npart)]).astype(np.int32)
    o0 = gen.random((2, npart)).astype(np.float32)
    step = gen.uniform(-0.99, 0.99, (2, npart))
    xi1 = c0 + o0.astype(np.float64) + step
    if edge:
        special = np.array([0.0, 0.5, np.nextafter(np.float32(0.5), 0), np.nextafter(np.float32(0.5), 1),
                            0.25, 0.75, np.nextafter(np.float32(1), 0), 1e-9], dtype=np.float32)
        k = len(special)
        o0[0, :k] = special
        o0[1, k:2 * k] = special
        xi1[:, :2 * k] = c0[:, :2 * k] + o0[:, :2 * k] + 0.3
    c1 = np.floor(xi1).astype(np.int64)
    o1 = (xi1 - c1).astype(np.float32)
    over = o1 >= 1
    c1[over] += 1
    o1[over] = 0
    c1[0] %= n1
    c1[1] %= n2
    v3 = gen.uniform(-0.95, 0.95, npart).astype(np.float32)
    qw = gen.uniform(-1.0, -0.5, npart).astype(np.float32)
    return c0, o0, c1.astype(np.int32), o1, v3, qw


@pytest.mark.parametrize("n1,n2,npart", [(64, 32, 20000), (256, 16, 100000)])
def test_debug_deposit_bitexact(hpic, n1, n2, npart):
    sim = hpic.Sim([hpic.config(n1, n2, 0.1, 0.2, 0.045)])
    c0, o0, c1, o1, v3, qw = _moves(n1, n2, npart, 100 + n1)
    # charges from a non-uniform set: the run's fixed-point unit comes from them
    gen = np.random.default_rng(5)
    xi = np.stack([gen.uniform(0, n1, 1000), gen.uniform(0, n2, 1000)])
    sim.set_particles(0, xi * np.array([[0.1], [0.2]]), np.zeros((3, 1000)),
                      gen.uniform(0.5, 1.0, 1000), -1.0, -1.0)
    fp = sim.fixed_params(0)
    assert fp["Q"] > 0
    Jg = sim.debug_deposit(0, c0, o0, c1, o1, v3, qw)
    Jo = oracle.deposit2_fixed(n1, n2, fp["P"], fp["inv_wunit"], fp["c3"], c0[0], c0[1], o0[0],
                               o0[1], c1[0], c1[1], o1[0], o1[1], v3, qw)
    assert np.array_equal(Jg, Jo)
    sim.close()


def _small_laser(seed=W.SEED0 + 201, n1=256, n2=64):
    dx1, dx2 = 0.1, 0.2
    L1, L2 = n1 * dx1, n2 * dx2
    laser = dict(a0=2.0, waist=3.0, length=2.0, k0=10.0, x1c=0.6 * L1, x2c=0.5 * L2)
    return W.drift2d(n1, n2, dx1, dx2, 0.045, sub=(4, 2), gamma=20.0, sigma_u=0.0, jitter=True,
                     seed=seed, laser=laser, name="laser_small")


def test_fp32_one_step_matches_oracle(hpic):
    d = _small_laser()
    sim = hpic.from_workload(d, "fp32")
    n1, n2 = d["n"][0], d["n"][1]
    before = sim.particles_raw(0)
    E0, B0 = sim.fields(0)
    fp = sim.fixed_params(0)
    sim.step(1)
    after = sim.particles_raw(0)
    E1, B1 = sim.fields(0)
    assert np.array_equal(before["id"], after["id"])
    xa = before["cell"] + before["off"].astype(np.float64)
    g = _oracle_grid(sim, jbg=d["jbg"])
    # push: gather + Boris in FP64 from the GPU's own FP32 inputs
    Ep, Bp = oracle.gather2(g, E0, B0, xa[0], xa[1])
    u = oracle.boris(d["qm"], d["dt"], Ep, Bp, before["u"].astype(np.float64))
    assert np.abs(after["u"] - u).max() <= 1e-6 * (1 + np.abs(u).max()) * 8
    gam = np.sqrt(1 + (u * u).sum(0))
    xb = xa + d["dt"] * (u[:2] / gam) / np.array([[d["dx"][0]], [d["dx"][1]]])
    step = after["cell"] - before["cell"]
    step[0] = (step[0] + n1 // 2) % n1 - n1 // 2
    step[1] = (step[1] + n2 // 2) % n2 - n2 // 2
    xg = before["cell"] + step + after["off"].astype(np.float64)
    assert np.abs(xg - xb).max() <= 2e-6
    # deposit: bit-exact against the fixed-point definition on the GPU's moves
    Jg = sim.current_fixed(0)
    v3 = _v3_float32(after["u"])
    Jo = oracle.deposit2_fixed(n1, n2, fp["P"], fp["inv_wunit"], fp["c3"], before["cell"][0],
                               before["cell"][1], before["off"][0], before["off"][1],
                               after["cell"][0], after["cell"][1], after["off"][0],
                               after["off"][1], v3, before["qw"])
    assert np.array_equal(Jg, Jo)
    # and, node by node, within the shape quantisation and FP32 rounding of the
    # plain FP64 Esirkepov current of the same moves (bound per node: the sum
    # over the particles reaching it, tests/deposit_bound.py)
    J64 = oracle.deposit2(g, xa[0], xa[1], xg[0], xg[1], v3.astype(np.float64),
                          before["qw"].astype(np.float64))
    bound = node_bounds(n1, n2, d["dx"][0], d["dx"][1], d["dt"], xa, xg, before["qw"], v3,
                        fp["P"], fp["inv_wunit"], fp["c3"], fp["Q"] == 0)
    for c in range(3):
        jc = sim.current(0, c) - d["jbg"][c]
        assert np.all(np.abs(jc - J64[c]) <= bound[c])
    # field update: FP64 hybrid update of the GPU's fields with that current
    Eo, Bo = oracle.field_update2(g, E0, B0, J64)
    scale = max(np.abs(Eo).max(), np.abs(Bo).max())
    assert np.abs(E1 - Eo).max() <= 2e-5 * scale
    assert np.abs(B1 - Bo).max() <= 2e-5 * scale
    sim.close()


def _by_id(p):
    """Particle arrays reordered by load index (the GPU sorts particles by tile)."""
    o = np.argsort(p["id"])
    return {k: (v[..., o] if isinstance(v, np.ndarray) else v) for k, v in p.items()}


def test_fp32_ten_steps_track_oracle(hpic):
    d = _small_laser(seed=W.SEED0 + 202)
    sim = hpic.from_workload(d, "fp32")
    raw = _by_id(sim.particles_raw(0))
    E0, B0 = sim.fields(0)
    g = _oracle_grid(sim, jbg=d["jbg"])
    xa = raw["cell"] + raw["off"].astype(np.float64)
    st = oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"], raw["qw"], E=E0, B=B0)
    sim.step(10)
    st.step(10)
    E1, B1 = sim.fields(0)
    # the oracle starts from the FP32 state: what remains is the FP32 push,
    # gather and fields over 10 steps (measured relative L2 1.4e-7 (E) and
    # 1.5e-7 (B), momenta 7.5e-7)
    for a, b in ((E1, st.E), (B1, st.B)):
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b)
    p = _by_id(sim.particles(0))
    assert np.abs(p["u"] - st.u).max() <= 3e-6 * (1 + np.abs(st.u).max())
    sim.close()


def test_fp64_form_matches_oracle_configs0(hpic):
    """64 x 32, gamma = 50, 100 steps in FP64 on the GPU and in the oracle."""
    d = W.drift2d_small()
    sim = hpic.from_workload(d, "fp64")
    p0 = _by_id(sim.particles(0))
    xi = p0["x"] / np.array([[d["dx"][0]], [d["dx"][1]]])
    g = _oracle_grid(sim, jbg=d["jbg"])
    qw = d["q"] * p0["w"]
    st = oracle.State2(g, d["qm"], xi[0], xi[1], p0["u"], qw)
    sim.step(d["steps"])
    st.step(d["steps"])
    E1, B1 = sim.fields(0)
    scale = max(np.abs(st.E).max(), np.abs(st.B).max())
    assert np.abs(E1 - st.E).max() <= 1e-9 * scale
    assert np.abs(B1 - st.B).max() <= 1e-9 * scale
    p = _by_id(sim.particles(0))
    assert np.abs(p["u"] - st.u).max() <= 1e-9 * np.abs(st.u).max()
    for c in range(3):
        jc = sim.current(0, c) - d["jbg"][c]
        assert np.abs(jc - st.J[c]).max() <= 1e-9 * (np.abs(st.J[c]).max() + 1e-30) + 1e-14
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 3e-5), ("fp64", 1e-11)])
@pytest.mark.parametrize("deriv1", [0, 1])
def test_vacuum_dispersion_gpu(hpic, prec, tol, deriv1):
    n1, n2, dx1, dx2 = 64, 32, 0.2, 0.3
    dt = 0.9 * oracle.courant_limit2(dx1, dx2)
    sim = hpic.Sim([hpic.config(n1, n2, dx1, dx2, dt, alpha=1.0, deriv1=deriv1, precision=prec)])
    k1i, k2i = 7, 5
    k1 = 2 * np.pi * k1i / (n1 * dx1)
    k2 = 2 * np.pi * k2i / (n2 * dx2)
    kk1 = np.sin(k1 * dx1 / 2) / (dx1 / 2) if deriv1 else k1
    kk2 = np.sin(k2 * dx2 / 2) / (dx2 / 2)
    theta = 2 * np.arcsin(0.5 * dt * np.hypot(kk1, kk2))
    X1, X2 = np.meshgrid(np.arange(n1), np.arange(n2))
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    E[2] = np.cos(2 * np.pi * (k1i * X1 / n1 + k2i * X2 / n2))
    sim.set_fields(0, E, B)
    steps = 60
    sim.step(steps)
    assert np.abs(sim.field(0, 2) - np.cos(steps * theta) * E[2]).max() < tol
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("fp64", 1e-10)])
def test_vacuum_eigenmode_1000_steps(hpic, prec, tol):
    """One discrete eigenmode carried 1000 steps: the phase follows the closed
    form (Eqs. (10), (19)) to FP32 rounding of the real-space output, i.e. the
    FP32 form does not accumulate a phase drift."""
    n1, n2, dx1, dx2, dt = 256, 16, 0.1, 0.2, 0.045
    sim = hpic.Sim([hpic.config(n1, n2, dx1, dx2, dt, alpha=1.0, precision=prec)])
    k1i, k2i = 41, 1
    k1 = 2 * np.pi * k1i / (n1 * dx1)
    kk2 = np.sin(np.pi * k2i / n2) / (dx2 / 2)
    theta = 2 * np.arcsin(0.5 * dt * np.hypot(k1, kk2))
    X1, X2 = np.meshgrid(np.arange(n1), np.arange(n2))
    E = np.zeros((3, n2, n1))
    E[2] = np.cos(2 * np.pi * (k1i * X1 / n1 + k2i * X2 / n2))
    sim.set_fields(0, E, np.zeros_like(E))
    sim.step(1000)
    assert np.abs(sim.field(0, 2) - np.cos(1000 * theta) * E[2]).max() < tol
    sim.close()


def test_fp32_laser_vacuum_1000_steps_matches_oracle(hpic):
    """The Gaussian laser pulse of the benchmark workload (k0 = 10, moving
    -x1) on a 256 x 32 grid without plasma, 1000 steps: relative L2 error of E
    and B of the FP32 form against the oracle's FP64 update at most 1e-5."""
    n1, n2, dx1, dx2, dt = 256, 32, 0.1, 0.2, 0.045
    laser = dict(a0=2.0, waist=1.5, length=2.0, k0=10.0, x1c=0.5 * n1 * dx1, x2c=0.5 * n2 * dx2)
    E0, B0 = W.laser_2d(n1, n2, dx1, dx2, **laser)
    sim = hpic.Sim([hpic.config(n1, n2, dx1, dx2, dt)])
    sim.set_fields(0, E0, B0)
    sim.step(1000)
    E1, B1 = sim.fields(0)
    g = oracle.grid2(n1, n2, dx1, dx2, dt, alpha=0.5)
    Eo, Bo = E0, B0
    J = np.zeros_like(E0)
    for _ in range(1000):
        Eo, Bo = oracle.field_update2(g, Eo, Bo, J)
    err = np.linalg.norm(np.concatenate([(E1 - Eo).ravel(), (B1 - Bo).ravel()])) / \
        np.linalg.norm(np.concatenate([Eo.ravel(), Bo.ravel()]))
    assert err <= 1e-5, err
    sim.close()


@pytest.mark.parametrize("n2", [16, 13, 4])
def test_fd_mode_matches_oracle_yee(hpic, n2):
    """deriv1 = 1 turns the hybrid kernels into the Yee scheme (end of Sec. 2.1).
    Row counts that are not a multiple of the update kernel's row strip (13)
    or smaller than one strip (4) take its partial-strip path."""
    n1 = 32
    gen = np.random.default_rng(9)
    E = gen.standard_normal((3, n2, n1))
    B = gen.standard_normal((3, n2, n1))
    sim = hpic.Sim([hpic.config(n1, n2, 0.15, 0.25, 0.05, alpha=1.0, deriv1=1, precision="fp64")])
    sim.set_fields(0, E, B)
    sim.step(1)
    g = oracle.grid2(n1, n2, 0.15, 0.25, 0.05, alpha=1.0, deriv1=1)
    Ey, By = oracle.yee_update2(g, E, B, np.zeros_like(E))
    E1, B1 = sim.fields(0)
    assert np.abs(E1 - Ey).max() < 1e-12 and np.abs(B1 - By).max() < 1e-12
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_gauss_and_continuity_gpu(hpic, prec):
    d = W.drift2d(64, 32, 0.2, 0.2, 0.05, sub=(2, 2), gamma=3.0, sigma_u=0.3, jitter=True,
                  alpha=0.5, seed=W.SEED0 + 301)
    sim = hpic.from_workload(d, prec)
    d0 = sim.diagnostics(0)
    assert d0["gauss_l2"] <= 1e-12 * max(d0["gauss_ref_l2"], 1.0)
    sim.step(20)
    sim.diagnostics(0)
    sim.step(1)
    d1 = sim.diagnostics(0)
    ref = max(d1["gauss_ref_l2"], 1e-3)
    if prec == "fp32":
        assert d1["cont_int"] == 0
        assert d1["gauss_l2"] <= 1e-4 * ref
    else:
        assert d1["cont_linf"] <= 1e-10
        assert d1["gauss_l2"] <= 1e-11 * ref
    # ablation: no current correction -> the Gauss residual grows
    sim2 = hpic.from_workload(d, prec, correct=0)
    sim2.step(21)
    d2 = sim2.diagnostics(0)
    assert d2["gauss_l2"] > 100 * d1["gauss_l2"]
    sim.close()
    sim2.close()


def test_state_resume_bitexact(hpic):
    d = _small_laser(seed=W.SEED0 + 203, n1=128, n2=32)
    a = hpic.from_workload(d, "fp32")
    a.step(3)
    blob = a.get_state()
    a.step(4)
    Ea, Ba = a.fields(0)
    ra = _by_id(a.particles_raw(0))
    b = hpic.from_workload(d, "fp32")
    b.set_state(blob)
    b.step(4)
    Eb, Bb = b.fields(0)
    rb = _by_id(b.particles_raw(0))
    assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
    for k in ("cell", "off", "u"):
        assert np.array_equal(ra[k], rb[k])
    a.close()
    b.close()


def test_batched_runs_equal_single_runs(hpic):
    """Runs of different sizes advanced in one batched launch give the same
    bits as each run alone."""
    ws = [W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=5.0, sigma_u=1e-2, seed=11),
          W.drift2d(128, 8, 0.2, 0.2, 0.05, sub=(2, 1), gamma=30.0, sigma_u=1e-3, seed=12,
                    density=2.0)]
    cfgs = [hpic.config(w["n"][0], w["n"][1], 0.2, 0.2, 0.05) for w in ws]
    batch = hpic.Sim(cfgs)
    for i, w in enumerate(ws):
        batch.set_particles(i, w["xi"] * 0.2, w["u"], w["w"], w["qm"], w["q"])
        batch.set_background(i, True, w["jbg"])
    batch.step(5)
    for i, w in enumerate(ws):
        one = hpic.from_workload(w, "fp32")
        one.step(5)
        assert np.array_equal(np.stack(one.fields(0)), np.stack(batch.fields(i)))
        assert np.array_equal(one.current_fixed(0), batch.current_fixed(i))
        one.close()
    batch.close()


def test_results_independent_of_sort_interval(hpic):
    """The fixed-point deposit is order-independent, so the tile sort cadence
    (which reorders particles) leaves fields and every particle bit-identical."""
    d = _small_laser(seed=W.SEED0 + 204, n1=256, n2=64)
    outs = []
    for k in (1, 7, 100000):
        sim = hpic.from_workload(d, "fp32", sort_interval=k)
        sim.profile(True)
        sim.step(12)
        E, B = sim.fields(0)
        raw = sim.particles_raw(0)
        order = np.argsort(raw["id"])
        st = sim.push_stats()
        assert st["tiles"] > 0 and st["fallback_tiles"] == 0
        outs.append((E, B, raw["cell"][:, order], raw["off"][:, order], raw["u"][:, order],
                     sim.current_fixed(0)))
        sim.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,tol", [("fp32", 5e-6), ("fp64", 1e-10)])
def test_kmod_dispersion_gpu(hpic, prec, tol):
    """Eq. (29) on the GPU: a mode inside the bump (k1/kg1 = 0.215) follows the
    closed form with [k]1 = k1 + dk_mod, coefficients of Sec. 4."""
    from tests.golden import load
    c = load("dkmod_table1.txt")
    n1, n2, dx1, dx2 = 256, 8, 0.2, 0.2
    dt = 0.9 * oracle.courant_limit2(dx1, dx2)
    k1i = 55
    k1 = 2 * np.pi * k1i / (n1 * dx1)
    kg = 2 * np.pi / dx1
    kl, ku = c["k1l_over_kg1"] * kg, c["k1u_over_kg1"] * kg
    km = 0.5 * (kl + ku)
    dk = c["dkmax_over_kg1"] * kg * np.cos((k1 - km) / (kl - km) * np.pi / 2) ** 2
    kk2 = np.sin(np.pi / n2) / (dx2 / 2)
    theta = 2 * np.arcsin(0.5 * dt * np.hypot(k1 + dk, kk2))
    sim = hpic.Sim([hpic.config(n1, n2, dx1, dx2, dt, alpha=1.0, precision=prec, kmod=1)])
    X1, X2 = np.meshgrid(np.arange(n1), np.arange(n2))
    E = np.zeros((3, n2, n1))
    E[2] = np.cos(2 * np.pi * (k1i * X1 / n1 + X2 / n2))
    sim.set_fields(0, E, np.zeros_like(E))
    sim.step(200)
    assert np.abs(sim.field(0, 2) - np.cos(200 * theta) * E[2]).max() < tol
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_kmod_gauss_and_oracle_gpu(hpic, prec):
    """With the Eq. (29) symbol the GPU step follows the oracle and keeps the
    Gauss residual (the correction is [k]1,FD/[k]1,mod)."""
    d = W.drift2d(64, 16, 0.2, 0.2, 0.05, sub=(2, 2), gamma=5.0, sigma_u=0.1, jitter=True, seed=22)
    sim = hpic.from_workload(d, prec, kmod=1)
    g = oracle.grid2(64, 16, 0.2, 0.2, 0.05, alpha=d["alpha"], jbg=d["jbg"], kmod=1)
    if prec == "fp32":
        raw = sim.particles_raw(0)
        o = np.argsort(raw["id"])
        xa = raw["cell"][:, o] + raw["off"][:, o].astype(np.float64)
        st = oracle.State2(g, d["qm"], xa[0], xa[1], raw["u"][:, o], raw["qw"][o])
    else:
        p = sim.particles(0)
        o = np.argsort(p["id"])
        st = oracle.State2(g, d["qm"], p["x"][0, o] / 0.2, p["x"][1, o] / 0.2, p["u"][:, o],
                           d["q"] * p["w"][o])
    sim.step(20)
    st.step(20)
    E1, _ = sim.fields(0)
    scale = max(np.abs(st.E).max(), 1e-3)
    assert np.abs(E1 - st.E).max() <= (1e-4 if prec == "fp32" else 1e-9) * scale
    dg = sim.diagnostics(0)
    assert dg["gauss_l2"] <= (2e-5 if prec == "fp32" else 1e-11) * dg["gauss_ref_l2"]
    sim.close()
