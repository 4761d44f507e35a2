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
