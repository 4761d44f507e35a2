"""Quasi-3D particle side on the GPU (gather from the modes, Boris push,
per-mode charge-conserving deposit, current transform, correction, filter and
the per-mode update) against the oracle: one step and many steps on small
grids in both forms, Gauss's law per mode kept with particles, the co-drifting
background current, error paths, and the 4096 x 256 three-mode workload (sampled
particles against the oracle's gather and push, Gauss's law at full size)."""
import numpy as np
import pytest

import oracle
from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _plasma(gen, n1, n2, dz, dr, rcells, ppc=(2, 2, 4), uth=0.05, drift=0.0, near_axis=True):
    zs, rs, ths = [], [], []
    for i in range(n1):
        for j in range(rcells):
            ph = gen.uniform(0, 2 * np.pi)
            for a in range(ppc[0]):
                for b in range(ppc[1]):
                    for t in range(ppc[2]):
                        zs.append((i + (a + gen.uniform(0.1, 0.9)) / ppc[0]) * dz)
                        rs.append((j + (b + gen.uniform(0.1, 0.9)) / ppc[1]) * dr)
                        ths.append(ph + 2 * np.pi * t / ppc[2])
    z, r, th = map(np.array, (zs, rs, ths))
    if near_axis:
        r[: len(r) // 10] *= 0.1
    n = z.size
    w = 2 * np.pi * r * dr * dz / np.prod(ppc)
    u = gen.normal(0, uth, (3, n))
    u[0] += drift
    return np.stack([z, r * np.cos(th), r * np.sin(th)]), u, w


def _random_fields(gen, M, n1, n2, scale):
    F = scale * (gen.standard_normal((M, 3, n2 + 1, n1)) + 1j * gen.standard_normal((M, 3, n2 + 1, n1)))
    F[:, :, n2] = 0
    for m in range(M):
        if m != 1:
            F[m, 2, 0] = 0
        if m != 0:
            F[m, 0, 0] = 0
    F[0] = F[0].real
    return F


def _read_fields(sim, M, run=0):
    E = np.stack([np.stack([sim.field_mode(run, c, m) for c in range(3)]) for m in range(M)])
    B = np.stack([np.stack([sim.field_mode(run, c, m) for c in range(3, 6)]) for m in range(M)])
    return E, B


def _setup(hpic, prec, n1=32, n2=16, M=3, dz=0.2, dr=0.25, dt=0.04, alpha=0.5, seed=0, fields=0.3,
           uth=0.05, kmod=0):
    gen = np.random.default_rng(seed)
    x, u, w = _plasma(gen, n1, n2, dz, dr, n2 - 6, uth=uth)
    E = _random_fields(gen, M, n1, n2, fields)
    B = _random_fields(gen, M, n1, n2, fields)
    B[:, 1, 0] = 0
    if M > 1:
        B[1, 1, 0] = fields * gen.standard_normal(n1)
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=alpha, precision=prec, modes=M, kmod=kmod)])
    for m in range(M):
        sim.set_fields_mode(0, m, E[m], B[m])
    sim.set_particles(0, x, u, w, q_over_m=-1.0, q=-1.0)
    g = oracle.gridq(n1, n2, M, dz, dr, dt, alpha=alpha, kmod=kmod)
    st = oracle.StateQ(g, -1.0, x, u, -w, E, B)
    return sim, st, g


def _particles(sim):
    p = sim.particles(0)
    order = np.argsort(p["id"])
    return p["x"][:, order], p["u"][:, order]


def _by_id(p):
    o = np.argsort(p["id"])
    return {k: v[..., o] for k, v in p.items()}


def _zdiff(a, b, L):
    return (a - b + 0.5 * L) % L - 0.5 * L


# M = 2 and 3 take the push kernels with the mode loops unrolled, 1 and 4 the
# general one
@pytest.mark.parametrize("M", [1, 2, 3, 4])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 3e-5)])
def test_one_step_matches_oracle(hpic, prec, tol, M):
    sim, st, g = _setup(hpic, prec, M=M)
    assert g.nmodes == M
    sim.step(1)
    st.step(1)
    x, u = _particles(sim)
    L = g.n1 * g.dz
    assert np.abs(_zdiff(x[0], st.pos[0], L)).max() <= tol * 10 * g.dz
    assert np.abs(x[1:] - np.stack(st.pos[1:])).max() <= tol * 10 * g.n2 * g.dr
    assert np.abs(u - st.u).max() <= tol * max(1.0, np.abs(st.u).max())
    Jscale = np.abs(st.J).max()
    for m in range(M):
        for c in range(3):
            Jg = sim.current_mode(0, c, m)
            err = np.abs(Jg - st.J[m, c]).max()
            assert err <= tol * 10 * Jscale, (m, c, err / Jscale)
    E, B = _read_fields(sim, M)
    scale = max(np.abs(st.E).max(), np.abs(st.B).max())
    assert np.abs(E - st.E).max() <= tol * 10 * scale
    assert np.abs(B - st.B).max() <= tol * 10 * scale
    sim.close()


# FP32: the oracle starts from the exact inputs, so the error is the FP32
# rounding of the particle state and the fields (a few units of 6e-8)
# carried over 20 steps; measured 1.1e-7 and 1.2e-7 of the field scale, and
# 2.2e-6 in the momenta (the FP32 mode gather with its FP32 phase factors)
@pytest.mark.parametrize("prec,tol,tol_u", [("fp64", 1e-9, 1e-9), ("fp32", 1e-6, 1e-5)])
@pytest.mark.parametrize("kmod", [0, 1])
def test_many_steps_match_oracle(hpic, prec, tol, tol_u, kmod):
    sim, st, g = _setup(hpic, prec, seed=1, kmod=kmod)
    M = g.nmodes
    sim.step(20)
    st.step(20)
    E, B = _read_fields(sim, M)
    scale = max(np.abs(st.E).max(), np.abs(st.B).max())
    assert np.abs(E - st.E).max() <= tol * scale
    assert np.abs(B - st.B).max() <= tol * scale
    x, u = _particles(sim)
    assert np.abs(u - st.u).max() <= tol_u * max(1.0, np.abs(st.u).max())
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 3e-5)])
def test_gauss_kept_with_particles(hpic, prec, tol):
    """E = B = 0 at the start and rho_bg = -rho_e(0): the residual of every mode
    starts at zero and stays at round-off (charge-conserving deposit plus the
    Eq. (11) correction of jz)."""
    n1, n2, M, dz, dr, dt = 32, 16, 3, 0.2, 0.25, 0.04
    gen = np.random.default_rng(5)
    x, u, w = _plasma(gen, n1, n2, dz, dr, n2 - 6, uth=0.1)
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=0.5, precision=prec, modes=M)])
    sim.set_particles(0, x, u, w, q_over_m=-1.0, q=-1.0)
    sim.set_background(0, 1)
    d0 = sim.diagnostics(0)
    assert d0["gauss_l2"] <= 1e-12 * max(d0["gauss_ref_l2"], 1.0)
    sim.step(30)
    d = sim.diagnostics(0)
    We = sum(d["W_E"])
    assert We > 0
    # scale: the norm of D.E itself is of the order of the filtered density change
    assert d["gauss_l2"] <= tol * max(d["gauss_ref_l2"], 1e-30), (d["gauss_l2"], d["gauss_ref_l2"])
    sim.close()


def test_background_current_matches_oracle(hpic):
    """A cold column drifting along z with the co-drifting background: the
    GPU's background profile (through the fields it drives) equals the
    oracle's."""
    n1, n2, M, dz, dr, dt = 32, 16, 2, 0.2, 0.25, 0.04
    gen = np.random.default_rng(6)
    x, u, w = _plasma(gen, n1, n2, dz, dr, n2 - 6, uth=0.0, drift=3.0)
    u[1:] += 1e-3 * gen.standard_normal((2, u.shape[1]))
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=0.5, precision="fp64", modes=M)])
    sim.set_particles(0, x, u, w, q_over_m=-1.0, q=-1.0)
    sim.set_background(0, 2)
    g = oracle.gridq(n1, n2, M, dz, dr, dt, alpha=0.5)
    jbg = oracle.jbg_q(g, x, u, -w)
    st = oracle.StateQ(g, -1.0, x, u, -w, jbg=jbg)
    sim.step(10)
    st.step(10)
    E, B = _read_fields(sim, M)
    scale = max(np.abs(st.E).max(), np.abs(st.B).max())
    assert np.abs(E - st.E).max() <= 1e-9 * scale
    # without the background the z-average of the m = 0 E_z grows from the net
    # current: the background really cancels it
    st2 = oracle.StateQ(g, -1.0, x, u, -w)
    st2.step(10)
    mean_with = np.abs(st.E[0, 0].mean(axis=1)).max()
    mean_without = np.abs(st2.E[0, 0].mean(axis=1)).max()
    assert mean_without > 100 * mean_with
    sim.close()


def test_particle_limits(hpic):
    n1, n2, M, dz, dr, dt = 16, 8, 2, 0.2, 0.25, 0.04
    sim = hpic.Sim([hpic.config(n1, n2, dz, dr, dt, alpha=0.5, precision="fp32", modes=M)])
    x = np.array([[0.1], [(n2 - 3) * dr + 1e-3], [0.0]])
    with pytest.raises(hpic.HpError):
        sim.set_particles(0, x, np.zeros((3, 1)), np.ones(1))
    # a particle pushed outward across r = (n2 - 3) dr stops the run with HP_ERANGE
    x = np.array([[0.1], [(n2 - 3) * dr - 0.01], [0.0]])
    u = np.array([[0.0], [50.0], [0.0]])
    sim.set_particles(0, x, u, np.ones(1))
    with pytest.raises(hpic.HpError):
        sim.step(1)
        sim.synchronize()
    sim.close()


def _full(hpic, prec):
    d = W.drift_q3d()
    n1, n2 = d["n"]
    sim = hpic.Sim([hpic.config(n1, n2, d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                                precision=prec, modes=d["modes"])])
    for m in range(d["modes"]):
        sim.set_fields_mode(0, m, d["E"][m], d["B"][m])
    sim.set_particles(0, d["x"], d["u"], d["w"], q_over_m=d["qm"], q=d["q"])
    sim.set_background(0, 2)
    return sim, d


def test_full_size_sampled_push_and_gauss(hpic):
    """4096 x 256, three modes, 8 192 000 particles (FP32 form): sampled
    particles after one step agree with the oracle's gather and Boris push in
    the GPU's fields, and the Gauss residual (non-zero from the seed pulse,
    whose divergence is not zero) keeps its norm over 5 steps to single
    precision."""
    sim, d = _full(hpic, "fp32")
    n1, n2 = d["n"]
    M = d["modes"]
    E0, B0 = _read_fields(sim, M)
    x0, u0 = _particles(sim)
    gen = np.random.default_rng(7)
    idx = np.concatenate([gen.choice(x0.shape[1], 400, replace=False),
                          np.arange(0, 2 * 4 * 8)])  # and some near the axis
    r0 = np.hypot(x0[1], x0[2])
    idx = np.concatenate([idx, np.nonzero(r0 < 0.3)[0][:50]])
    g = oracle.gridq(n1, n2, M, d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"])
    Ep, Bp = oracle.gather_q(g, E0, B0, x0[:, idx])
    uz, ux, uy = (np.ascontiguousarray(u0[c, idx]) for c in range(3))
    lib = oracle.lib()
    _p = oracle._p
    lib.or_boris(len(idx), d["qm"], d["dt"], _p(np.ascontiguousarray(Ep)),
                 _p(np.ascontiguousarray(Bp)), _p(uz), _p(ux), _p(uy))
    sim.step(1)
    x1, u1 = _particles(sim)
    uo = np.stack([uz, ux, uy])
    assert np.abs(u1[:, idx] - uo).max() <= 2e-5 * np.abs(uo).max()
    d0 = sim.diagnostics(0)
    sim.step(4)
    d1 = sim.diagnostics(0)
    assert abs(d1["gauss_l2"] - d0["gauss_l2"]) <= 1e-4 * d0["gauss_l2"]
    sim.close()


def test_full_size_fp64_gauss(hpic):
    """The same workload in the FP64 form: the residual's norm is unchanged to
    double-precision round-off after 3 steps (charge conservation per mode at
    full size)."""
    sim, d = _full(hpic, "fp64")
    d0 = sim.diagnostics(0)
    sim.step(3)
    d1 = sim.diagnostics(0)
    assert d1["gauss_ref_l2"] > 0
    assert abs(d1["gauss_l2"] - d0["gauss_l2"]) <= 1e-9 * d0["gauss_l2"]
    sim.close()


def test_fp32_drift_stays_near_fp64_level(hpic):
    """Continuity of the FP32 deposit to 2^-41 of a particle's charge: on a
    quasi-3D drift of gamma = 50, n = 100 (256 x 64, modes 0 and 1, dt = 0.08,
    filter and the Eq. (29) symbol) the E_r energy of the FP32 form stays
    within a decade of the FP64 form's over 4000 steps (a deposit with FP32
    weights and a 2^28 scale grew four decades here)."""
    d = W.drift_q3d(n1=256, n2=64, dz=0.2, dr=0.2, dt=0.08, modes=2, sub=(2, 1, 4), gamma=50.0,
                    sigma_u=1e-4, density=100.0, a0=0.0, seed=W.SEED0 + 12)
    top = {}
    for prec in ("fp64", "fp32"):
        sim = hpic.Sim([hpic.config(256, 64, 0.2, 0.2, 0.08, alpha=0.5, precision=prec, modes=2,
                                    kmod=1)])
        sim.set_particles(0, d["x"], d["u"], d["w"], q_over_m=d["qm"], q=d["q"])
        sim.set_background(0, 2)
        logw = []
        for _ in range(10):
            sim.step(400)
            logw.append(np.log10(sim.diagnostics(0)["W_E"][1]))
        sim.close()
        top[prec] = max(logw)
    assert top["fp32"] < top["fp64"] + 1.5, top


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_state_resume_bitexact(hpic, prec):
    """Checkpoint of a quasi-3D handle (particles, fields of every mode, the
    FP64 master, the last deposit, the background): the current read right
    after the restore is the checkpointed handle's, and a fresh handle restored
    from it and advanced takes the same steps, bit for bit in the FP32 form
    (64-bit integer deposit).  The FP64 form accumulates its deposit with FP64
    atomics, whose order varies from run to run, so there the resumed run
    agrees to rounding; so does the Gauss residual in both forms, whose charge
    density is deposited with FP64 atomics."""
    a, _, g = _setup(hpic, prec, seed=21)
    a.set_background(0, 2)
    a.step(3)
    blob = a.get_state()
    j_before = [a.current_mode(0, c, m) for m in range(g.nmodes) for c in range(3)]
    a.step(4)
    b, _, _ = _setup(hpic, prec, seed=22)
    b.set_state(blob)
    for want, m_c in zip(j_before, [(m, c) for m in range(g.nmodes) for c in range(3)]):
        assert np.array_equal(b.current_mode(0, m_c[1], m_c[0]), want)
    b.step(4)
    Ea, Ba = _read_fields(a, g.nmodes)
    Eb, Bb = _read_fields(b, g.nmodes)
    pa, pb = _by_id(a.particles(0)), _by_id(b.particles(0))
    if prec == "fp32":
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k
        # the Gauss diagnostic's charge density is an FP64 atomic deposit
        ga, gb = a.diagnostics(0)["gauss_l2"], b.diagnostics(0)["gauss_l2"]
        assert abs(ga - gb) <= 1e-12 * abs(ga)
    else:
        scale = max(np.abs(Ea).max(), np.abs(Ba).max())
        assert max(np.abs(Ea - Eb).max(), np.abs(Ba - Bb).max()) <= 1e-12 * scale
        assert np.array_equal(pa["id"], pb["id"])
        for k in ("x", "u"):
            assert np.abs(pa[k] - pb[k]).max() <= 1e-12 * (1 + np.abs(pa[k]).max())
    # a blob of the other precision or a truncated one is refused
    with pytest.raises(hpic.HpError):
        b.set_state(blob[: len(blob) // 2])
    other, _, _ = _setup(hpic, "fp32" if prec == "fp64" else "fp64", seed=23)
    with pytest.raises(hpic.HpError):
        other.set_state(blob)
    for s in (a, b, other):
        s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sort_leaves_the_steps_unchanged(hpic, prec):
    """The periodic counting sort of the particles by (z column, radial row)
    bin only permutes their storage: sorting every step and never sorting give
    the same fields and particles, bit for bit in the FP32 form (integer
    deposit), to rounding in the FP64 form (FP64 atomics)."""
    a, _, g = _setup(hpic, prec, seed=31, uth=0.2)
    b, _, _ = _setup(hpic, prec, seed=31, uth=0.2)
    a.set_tiling(2, 4, 1)
    b.set_tiling(2, 4, 1024)
    assert tuple(a.tiling()["tile"]) == (2, 4) and a.tiling()["sort_interval"] == 1
    a.step(30)
    b.step(30)
    Ea, Ba = _read_fields(a, g.nmodes)
    Eb, Bb = _read_fields(b, g.nmodes)
    ra, rb = a.particles(0), b.particles(0)
    assert not np.array_equal(ra["id"], rb["id"])  # the sort did reorder
    pa, pb = _by_id(ra), _by_id(rb)
    if prec == "fp32":
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k
    else:
        scale = max(np.abs(Ea).max(), np.abs(Ba).max())
        assert max(np.abs(Ea - Eb).max(), np.abs(Ba - Bb).max()) <= 1e-12 * scale
        assert np.abs(pa["u"] - pb["u"]).max() <= 1e-12 * (1 + np.abs(pa["u"]).max())
    for sim in (a, b):
        with pytest.raises(hpic.HpError):
            sim.set_tiling(0, 4, 8)
        sim.close()


def test_sort_of_batched_runs(hpic):
    """Two quasi-3D runs of different sizes in one handle: the sort works per
    run (its bins per run's grid), and the FP32 results equal those of the
    same runs never sorted, bit for bit."""
    cfgs = [hpic.config(32, 16, 0.2, 0.25, 0.04, precision="fp32", modes=3),
            hpic.config(64, 12, 0.1, 0.2, 0.04, precision="fp32", modes=2)]
    gen = np.random.default_rng(41)
    loads = []
    for (n1, n2, dz, dr, M) in ((32, 16, 0.2, 0.25, 3), (64, 12, 0.1, 0.2, 2)):
        x, u, w = _plasma(gen, n1, n2, dz, dr, n2 - 6, uth=0.2)
        E = _random_fields(gen, M, n1, n2, 0.3)
        B = _random_fields(gen, M, n1, n2, 0.3)
        B[:, 1, 0] = 0
        loads.append((x, u, w, E, B, M))
    out = []
    for K in (1, 1024):
        sim = hpic.Sim(cfgs)
        for run, (x, u, w, E, B, M) in enumerate(loads):
            for m in range(M):
                sim.set_fields_mode(run, m, E[m], B[m])
            sim.set_particles(run, x, u, w, q_over_m=-1.0, q=-1.0)
        sim.set_tiling(4, 2, K)
        sim.step(25)
        res = []
        for run, (_, _, _, _, _, M) in enumerate(loads):
            res.append((_read_fields(sim, M, run), _by_id(sim.particles(run))))
        out.append(res)
        sim.close()
    for (fa, pa), (fb, pb) in zip(out[0], out[1]):
        for a, b in zip(fa, fb):
            assert np.array_equal(a, b)
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k
