"""Device-buffer entry points of the C ABI (the scheme's particle input and
field/particle output, Sec. 2, with caller-owned device memory):
hp_set_particles_device loads from FP64 device tensors with the same
conversion as the host loader, so the run's state is the same bit for bit and
so are the fields after steps (the FP32 form; the FP64 form's atomics make
them equal to rounding); hp_get_field_device, hp_get_particles_device and
hp_get_current_device return what the host reads return; host pointers,
quasi-3D handles and non-finite input are rejected without changing the
run."""
import ctypes

import numpy as np
import pytest

from paper_1502_01376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _by_id(p):
    o = np.argsort(p["id"])
    return {k: v[..., o] for k, v in p.items()}


def _laser(seed=W.SEED0 + 401):
    laser = dict(a0=2.0, waist=2.0, length=1.5, k0=10.0, x1c=0.6 * 12.8, x2c=0.5 * 6.4)
    return W.drift2d(128, 32, 0.1, 0.2, 0.045, sub=(4, 2), gamma=20.0, sigma_u=1e-2, jitter=True,
                     seed=seed, laser=laser, name="io")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_device_load_equals_host_load(hpic, precision):
    import torch
    d = _laser()
    a = hpic.from_workload(d, precision)
    b = hpic.from_workload(d, precision)
    x = np.stack([d["xi"][k] * d["dx"][k] for k in range(2)])
    dev = torch.device("cuda")
    b.set_particles_device(0, torch.tensor(x, device=dev), torch.tensor(d["u"], device=dev),
                           torch.tensor(d["w"], device=dev), d["qm"], d["q"])
    b.set_background(0, True, d["jbg"])
    if precision == "fp32":
        assert a.fixed_params(0) == b.fixed_params(0)
        pa, pb = _by_id(a.particles_raw(0)), _by_id(b.particles_raw(0))
    else:
        pa, pb = _by_id(a.particles(0)), _by_id(b.particles(0))
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    a.step(5)
    b.step(5)
    Ea, Ba = a.fields(0)
    Eb, Bb = b.fields(0)
    if precision == "fp32":
        # integer deposit: independent of the order of the atomics
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
    else:
        # FP64 atomics: the same to rounding
        scale = max(np.abs(Ea).max(), np.abs(Ba).max())
        assert max(np.abs(Ea - Eb).max(), np.abs(Ba - Bb).max()) <= 1e-12 * scale
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_device_reads_equal_host_reads(hpic, precision):
    import torch
    d = _laser(W.SEED0 + 402)
    sim = hpic.from_workload(d, precision)
    sim.step(3)
    rt = torch.float32 if precision == "fp32" else torch.float64
    n, dev = sim.count(0), torch.device("cuda")
    F = torch.empty((6,) + sim.shape(0), dtype=rt, device=dev)
    for c in range(6):
        sim.field_device(0, c, F[c])
    cell = torch.empty((2, n), dtype=torch.int32, device=dev)
    off = torch.empty((2, n), dtype=rt, device=dev)
    u = torch.empty((3, n), dtype=rt, device=dev)
    qw = torch.empty(n, dtype=rt, device=dev)
    pid = torch.empty(n, dtype=torch.int32, device=dev)
    sim.particles_device(0, cell, off, u, qw, pid)
    sim.synchronize()
    E, B = sim.fields(0)
    assert np.array_equal(F.cpu().numpy().astype(np.float64), np.concatenate([E, B]))
    for corrected in (False, True):
        J = torch.empty((3,) + sim.shape(0), dtype=torch.float64, device=dev)
        for c in range(3):
            sim.current_device(0, c, J[c], corrected=corrected)
        sim.synchronize()
        want = np.stack([sim.current(0, c, corrected=corrected) for c in range(3)])
        assert np.array_equal(J.cpu().numpy(), want), corrected
    if precision == "fp32":
        raw = sim.particles_raw(0)
        for k, t in (("cell", cell), ("off", off), ("u", u), ("qw", qw), ("id", pid)):
            assert np.array_equal(raw[k], t.cpu().numpy()), k
    else:
        p = sim.particles(0)
        x = (cell.cpu().numpy() + off.cpu().numpy()) * np.array([[d["dx"][0]], [d["dx"][1]]])
        assert np.abs(x - p["x"]).max() < 1e-12
        assert np.array_equal(u.cpu().numpy(), p["u"])
        assert np.array_equal(pid.cpu().numpy(), p["id"].astype(np.int32))
    sim.close()


def test_device_entry_points_reject_bad_input(hpic):
    import torch
    d = _laser(W.SEED0 + 403)
    sim = hpic.from_workload(d, "fp32")
    before = _by_id(sim.particles_raw(0))
    n, dev = d["w"].size, torch.device("cuda")
    x = torch.tensor(np.stack([d["xi"][k] * d["dx"][k] for k in range(2)]), device=dev)
    u = torch.tensor(d["u"], device=dev)
    w = torch.tensor(d["w"], device=dev)
    # host memory where device memory is required
    xh = np.ascontiguousarray(x.cpu().numpy())
    rc = hpic.lib().hp_set_particles_device(sim.h, 0, 0, n, xh.ctypes.data_as(ctypes.c_void_p),
                                            ctypes.c_void_p(u.data_ptr()),
                                            ctypes.c_void_p(w.data_ptr()), -1.0, -1.0)
    assert rc == hpic.HP_EINVAL
    out = np.empty(sim.shape(0), dtype=np.float32)
    assert hpic.lib().hp_get_field_device(sim.h, 0, 0, out.ctypes.data_as(ctypes.c_void_p),
                                          out.size) == hpic.HP_EINVAL
    out64 = np.empty(sim.shape(0))
    assert hpic.lib().hp_get_current_device(sim.h, 0, 0, 0, out64.ctypes.data_as(ctypes.c_void_p),
                                            out64.size) == hpic.HP_EINVAL
    # a non-finite input leaves the run as it was
    u_bad = u.clone()
    u_bad[1, n // 2] = float("nan")
    with pytest.raises(hpic.HpError):
        sim.set_particles_device(0, x, u_bad, w, d["qm"], d["q"])
    after = _by_id(sim.particles_raw(0))
    for k in before:
        assert np.array_equal(before[k], after[k])
    sim.close()
    q = hpic.Sim([hpic.config(64, 16, 0.1, 0.2, 0.04, modes=2)])
    with pytest.raises(hpic.HpError):
        q.set_particles_device(0, torch.zeros((3, 4), dtype=torch.float64, device=dev),
                               torch.zeros((3, 4), dtype=torch.float64, device=dev),
                               torch.ones(4, dtype=torch.float64, device=dev))
    q.close()
