"""Command-line driver: advances one of the synthetic workloads through the
library and prints one JSON line with the wall time per step and the
per-kernel durations of a second, event-timed pass.  Used to run a single
workload under a profiler without the rest of the benchmark.

    python3 -m paper_1502_01376_amd.drive drift3d --precision fp32 --steps 500 --tiling 8,4,64
"""
import argparse
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1502_01376_amd import hpic  # noqa: E402
from paper_1502_01376_amd import workloads as W  # noqa: E402

WORKLOADS = ("drift2d_laser", "drift3d", "drift_q3d")


def make(name, precision, stream):
    if name == "drift_q3d":
        d = W.drift_q3d()
        n1, n2 = d["n"]
        sim = hpic.Sim([hpic.config(n1, n2, d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                                    precision=precision, modes=d["modes"])], stream=stream)
        for m in range(d["modes"]):
            sim.set_fields_mode(0, m, d["E"][m], d["B"][m])
        sim.set_particles(0, d["x"], d["u"], d["w"], q_over_m=d["qm"], q=d["q"])
        sim.set_background(0, 2)
        return sim, d["w"].size
    d = getattr(W, name)()
    return hpic.from_workload(d, precision, stream=stream), d["w"].size


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=WORKLOADS)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tiling", type=str, default="",
                    help="T1,T2,K: tile shape and sort interval (Cartesian workloads)")
    a = ap.parse_args(argv)
    import torch
    sim, npart = make(a.workload, a.precision, torch.cuda.current_stream())
    if a.tiling:
        sim.set_tiling(*[int(v) for v in a.tiling.split(",")])
    sim.step(a.warmup)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(a.steps)
    sim.synchronize()
    t = time.perf_counter() - t0
    sim.profile(True)
    sim.step(a.steps)
    sim.synchronize()
    kt = sim.kernel_times()
    sim.profile(False)
    print(json.dumps({"workload": a.workload, "precision": a.precision, "particles": npart,
                      "steps": a.steps, "ms_per_step": 1e3 * t / a.steps,
                      "kernels_us": {k: 1e3 * ms / n for k, (ms, n) in kt.items() if n}}), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
