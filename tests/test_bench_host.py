"""Host-side behaviour of bench.py (no GPU): more than one GPU is refused with
a message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


class _FakeSim:
    """Stand-in handle: fields are a fixed function of the loaded particles and
    the step count, with an offset per precision, so the comparison logic of
    the precision runs can be checked on the host."""

    def __init__(self, ds, precision):
        import numpy as np
        self.ds, self.prec, self.steps = ds, precision, 0
        self.np = np

    def step(self, n):
        self.steps += n

    def _base(self, r):
        d = self.ds[r]
        s = float(self.np.sum(d["xi"])) + 1e-3 * self.steps
        return s + (1e-6 if self.prec == "fp32" else 0.0)

    def fields(self, r):
        v = self._base(r)
        return self.np.full((3, 2, 4), v), self.np.full((3, 2, 4), 2 * v)

    def current(self, r, c):
        return self.np.full((2, 4), self._base(r) + c)

    def particles(self, r):
        d = self.ds[r]
        x = self.np.stack([d["xi"][k] * d["dx"][k] for k in range(d["xi"].shape[0])])
        return dict(x=x.astype(self.np.float32).astype(float), u=d["u"], w=d["w"],
                    id=self.np.arange(x.shape[1]))

    def diagnostics(self, r):
        return dict(gauss_l2=1e-9, gauss_ref_l2=1.0)

    def close(self):
        pass


def test_precision_runs_bookkeeping():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench

    class H:
        @staticmethod
        def from_workloads(ds, precision):
            return _FakeSim(ds, precision)

    gen = np.random.default_rng(5)
    ds = [dict(xi=gen.uniform(0, 8, (2, 16)), dx=(0.1, 0.2, 1.0), u=gen.normal(size=(3, 16)),
               w=np.ones(16)) for _ in range(3)]
    cps, hist, diag = bench.precision_cartesian(H, ds, 50, (10, 30, 100))
    assert cps == [10, 30, 50]
    assert set(hist) == set(bench.CONTROLS) and len(diag) == 3
    for k in bench.CONTROLS:
        assert len(hist[k]) == 3 and all(len(h) == 3 for h in hist[k])
    # the FP32 stand-in is off by 1e-6 in every value; the ulp control by the
    # one-ulp position change only
    for h in hist["fp32"]:
        for r in range(3):
            assert 0 < h[r]["E"] < 1e-6
    assert max(h[r]["E"] for h in hist["fp64_ulp"] for r in range(3)) < 1e-12
    tab = bench._single_run_table(cps, {k: [[h[0]] for h in hist[k]] for k in hist}, diag)
    assert tab["checkpoints"] == cps and len(tab["fp32"]["E"]) == 3
    assert tab["gauss_rel_l2_fp32"] == 1e-9


class _FakeCartSim(_FakeSim):
    """Enough of hpic.Sim for bench.py's legs: steps, tiling, profiling,
    reads (shapes of the workload), diagnostics."""

    def __init__(self, ds, precision, **kw):
        super().__init__(ds, precision)
        self.tile = dict(tile=[16, 16], sort_interval=8, lds_bytes=1024, ms_per_step=0.1,
                         candidates=0, steps=0)

    def set_tiling(self, t1, t2, k):
        self.tile = dict(self.tile, tile=[t1, t2], sort_interval=k)

    def tiling(self):
        return dict(self.tile)

    def autotune(self, n):
        self.steps += n
        return dict(self.tile, candidates=3, steps=n)

    def synchronize(self):
        pass

    def profile(self, on):
        pass

    def kernel_times(self):
        return {k: (0.1 * 5, 5) for k in ("push_deposit", "fft_j", "kupdate", "ifft_eb", "sort")}

    def push_stats(self):
        return dict(fallback_tiles=0, tiles=10)

    def diagnostics(self, r):
        return dict(gauss_l2=1e-9, gauss_ref_l2=1.0, cont_linf=0.0, charge_total=-1.0, step=self.steps,
                    kinetic=1.0, W_E=[1.0, 1.0, 1.0], W_B=[1.0, 1.0, 1.0])

    def fields(self, r):
        import numpy as np
        n = self.ds[r]["n"]
        v = self._base(r)
        return np.full((3,) + tuple(n[::-1]), v), np.full((3,) + tuple(n[::-1]), 2 * v)

    def current(self, r, c):
        import numpy as np
        return np.full(tuple(self.ds[r]["n"][::-1]), self._base(r) + c)


def _fake_env():
    import numpy as np
    import types
    sys.path.insert(0, ROOT)
    import bench

    def cart(n, seed):
        g = np.random.default_rng(seed)
        npart = 32
        xi = g.uniform(0, 4, (len(n), npart))
        return dict(n=tuple(n) + (1,) * (3 - len(n)), dx=(0.1, 0.2, 0.2), xi=xi,
                    u=g.normal(size=(3, npart)), w=np.ones(npart), name="fake", dt=0.05)

    class FakeQ(_FakeCartSim):
        def __init__(self, cfgs, stream=None):
            super().__init__([dict(xi=np.zeros((3, 4)), n=(8, 4, 1), dx=(0.1, 0.2, 1.0))], cfgs[0]["p"])

        def set_fields_mode(self, *a):
            pass

        def set_particles(self, run, x, u, w, q_over_m, q):
            self.ds = [dict(self.ds[0], xi=x.copy())]

        def set_background(self, *a):
            pass

        def particles(self, r):
            d = self.ds[r]
            return dict(x=d["xi"].astype(np.float32).astype(float), u=np.zeros((3, 4)),
                        w=np.ones(4), id=np.arange(4))

        def field_mode(self, r, c, m):
            return np.full((5, 8), self._base(r) + c + 1j * m)

        def current_mode(self, r, c, m):
            return np.full((5, 8), self._base(r) + c + 0j)

    hp = types.SimpleNamespace(
        from_workloads=lambda ds, precision, stream=None, **kw: _FakeCartSim(ds, precision),
        Sim=FakeQ, config=lambda *a, precision="fp32", **kw: {"p": precision})
    torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None,
                                                           current_stream=lambda: None))
    W = types.SimpleNamespace(
        scan2d=lambda: [cart((8, 4), 1), cart((16, 4), 2)],
        scan2d_params=lambda: [dict(n1=8, n2=4, ppc=4, gamma=5.0, density=1.0),
                               dict(n1=16, n2=4, ppc=8, gamma=50.0, density=2.0)],
        drift3d=lambda: cart((8, 4, 4), 3),
        drift_q3d=lambda: dict(n=(8, 4), dx=(0.1, 0.2), dt=0.04, alpha=0.5, modes=2, name="q",
                               E=[0, 0], B=[0, 0], x=np.ones((3, 4)), u=np.zeros((3, 4)),
                               w=np.ones(4), qm=-1.0, q=-1.0))
    return bench, hp, torch, W


def test_bench_legs_run_on_a_stand_in_library():
    """The scan, 3D and quasi-3D legs of bench.py (timing, precision runs,
    fixed or tuned tilings) run end to end on a stand-in library, so that a
    mistake in their Python shows here rather than on the GPU."""
    bench, hp, torch, W = _fake_env()
    s = bench.scan_leg(hp, torch, W, 20, 10, True)
    assert s["precision"]["checkpoints"] == [10, 20] and len(s["precision"]["per_run"]) == 2
    for fixed in (None, [8, 4, 16]):
        d3 = bench.d3_leg(hp, torch, W, 20, 10, True, fixed)
        assert d3["err_vs_fp64"]["checkpoints"] == [10, 20]
        assert d3["tiling"]["tile"] == ([8, 4] if fixed else [16, 16])
    q = bench.q3d_leg(hp, torch, W, 20, True)
    assert q["err_vs_fp64"]["checkpoints"] == [10, 20] and "push_deposit_frac" in q
