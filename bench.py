"""Benchmark of the hybrid Yee-FFT PIC step on one MI355X.

Workload: the 2D drifting-plasma laser case, 2048 x 512 cells, dx = (0.1, 0.2),
dt = 0.045, 8 particles per cell (8 388 608), gamma = 20, Gaussian laser
a0 = 2 (synthetic, seeded).  One step is the whole hot path: gather + Boris +
charge-conserving deposit, FFT of j along x1 with the current correction and
the low-pass filter, hybrid Maxwell update, inverse FFT of E and B.

Prints one JSON line: particle-steps/s of the FP32 form (64-bit fixed-point
deposit) with the FP64 form measured beside it and the FP32-vs-FP64 field error,
the roofline of the push+deposit kernel from HIP-event timing, and the FP64 CPU
oracle timed on the host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic HBM bytes of one push+deposit launch: each particle's state is
# read once (cell 4 + offsets 8 + momenta 12 + charge 4 = 28 B) and written
# once (24 B); each cell's six FP32 field values are read once (24 B) and its
# three 64-bit current accumulators read and written once (48 B).
BYTES_PER_PARTICLE = 52
BYTES_PER_CELL = 72
# Quasi-3D push+deposit: 76 B per particle (read 40: cell, offsets, momenta,
# charge; write 36) and 144 B per node of each mode (48 B of complex FP32
# fields read, 96 B of complex int64 current read-modify-write).
Q3D_BYTES_PER_PARTICLE = 76
Q3D_BYTES_PER_MODE_NODE = 144
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=-1,
                    help="steps of the FP64 form timed beside the FP32 form (-1: as --steps, 0: skip)")
    ap.add_argument("--err-steps", type=int, default=1000,
                    help="steps over which the FP32 form of the benchmark workload is compared "
                         "with the FP64 form and its controls (0: skip)")
    ap.add_argument("--precision", type=int, default=1,
                    help="compare the FP32 form with the FP64 form and the FP64 controls on the "
                         "3D, quasi-3D and scan legs too, at their own step counts")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--tune-steps", type=int, default=1200,
                    help="steps advanced by the autotuner before the warm-up (0: default tiling)")
    ap.add_argument("--tiling", type=str, default="",
                    help="T1,T2,K: fixed tile shape and sort interval instead of the autotuner")
    ap.add_argument("--scan-steps", type=int, default=200,
                    help="steps of the 64-run parameter scan (0: skip)")
    ap.add_argument("--d3-steps", type=int, default=500,
                    help="steps of the 3D 512x128x128 drifting-plasma leg (0: skip)")
    ap.add_argument("--d3-tiling", type=str, default="",
                    help="T1,T2,K: fixed 3D tiling (T1 x T2 x T2 cells, sort interval K) instead "
                         "of the autotuner")
    ap.add_argument("--shape-steps", type=int, default=200,
                    help="steps of the benchmark workload with the energy-conserving gather "
                         "and with the cubic shape (0: skip)")
    ap.add_argument("--q3d-steps", type=int, default=500,
                    help="steps of the quasi-3D 4096x256 three-mode PIC leg (0: skip)")
    ap.add_argument("--lwfa-steps", type=int, default=6400,
                    help="steps of the Table 2 boosted-frame laser wakefield run (8192x512, "
                         "FP32, with and without the k1 filter; 0: skip)")
    ap.add_argument("--nci-steps", type=int, default=40000,
                    help="steps of the Table 1 NCI contrast (four 256x256 runs; 0: skip)")
    ap.add_argument("--n1", type=int, default=2048)
    ap.add_argument("--n2", type=int, default=512)
    return ap.parse_args()


def align_to_sort(sim):
    """Untimed steps after which the next step starts with a tile sort: a
    timed window of n steps then holds ceil(n / K) sorts for the sort interval
    K, however n compares with K (the sort's cost is counted, never skipped).
    Returns K (0 for handles without a tile sort)."""
    try:
        t = sim.tiling()
    except Exception:
        return 0
    K = int(t["sort_interval"])
    if K <= 0:
        return 0
    sim.set_tiling(t["tile"][0], t["tile"][1], K)  # sorts now
    # K steps reach the next sort; two more blocks of a sort and K steps
    # capture the step graphs of both particle buffers outside the window
    sim.step(3 * K)
    return K


def timed_steps(torch, sim, warmup, steps, align=True):
    """Wall time of `steps` steps after `warmup` untimed ones (and, with
    align, the steps that bring the next tile sort to the window's first
    step), synchronised on both sides."""
    sim.step(warmup)
    if align:
        align_to_sort(sim)
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.synchronize()
    return t1 - t0


def _as_tiling(t):
    """[T1, T2, K] of a tiling record (the FP64 form runs at the FP32 form's
    tiling: its own short autotuning picked tiles whose boxes outgrow the LDS
    budget later in a run)."""
    return [t["tile"][0], t["tile"][1], t["sort_interval"]]


def run_form(hpic, torch, ds, precision, warmup, steps, profile=False, tune_steps=0, tiling=None,
             **cfg_kw):
    """Untimed: the autotuner (tune_steps steps, picking tile shape and sort
    interval on the live runs) and `warmup` steps.  Timed region: `steps`
    steps with the captured-graph step (the library's default).  With
    `profile`, a second pass of the same length launches every kernel with HIP
    events around it on the library's stream for per-kernel durations."""
    sim = hpic.from_workloads(ds, precision, stream=torch.cuda.current_stream(), **cfg_kw)
    if tiling:
        sim.set_tiling(*tiling)
    # the autotuner's record: candidates tried, steps, the choice's timing
    sim.tuning = sim.autotune(tune_steps) if not tiling and tune_steps > 0 else sim.tiling()
    t = timed_steps(torch, sim, warmup, steps)
    kt = None
    if profile:
        sim.profile(True)
        tp = timed_steps(torch, sim, 0, steps)
        kt = sim.kernel_times()
        kt["push_stats"] = sim.push_stats()
        kt["profiled_wall_s"] = tp
        sim.profile(False)
    return sim, t, kt


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "push_deposit_drift2d_2048x512_hbm_traffic.txt")
PUSH_SOURCES = [os.path.join(ROOT, "paper_1502_01376_amd", "csrc", f)
                for f in ("push.hip", "hpic_internal.h")]


CSRC = os.path.join(ROOT, "paper_1502_01376_amd", "csrc")
D3_COUNTERS = os.path.join(ROOT, "profiles", "drift3d_512x128x128_counters.txt")
D3_SOURCES = [os.path.join(CSRC, f) for f in ("push3.hip", "hpic_internal.h")]
Q3D_COUNTERS = os.path.join(ROOT, "profiles", "drift_q3d_4096x256_counters.txt")
Q3D_SOURCES = [os.path.join(CSRC, f) for f in ("pushq.hip", "hpic_q3d.h", "hpic_internal.h")]


def source_hash(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in files or PUSH_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, sources=None, prefix=""):
    """HBM bytes per push+deposit launch from a committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    key = prefix + "hbm_bytes_per_launch"
    if vals.get(prefix + "source_hash") != source_hash(sources) or key not in vals:
        return None
    return float(vals[key])


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# Error of the FP32 form at the configurations' own lengths, beside two
# controls that separate round-off amplified by the dynamics from a defect:
# the FP64 form started from positions one FP64 ulp away (ulp64), and the
# FP64 form started from the FP32 form's initial state, i.e. the inputs
# rounded to FP32 offsets, momenta and charges (fp32_init).  All against the
# FP64 form from the exact inputs, at checkpoints along the run.
CONTROLS = ("fp32", "fp64_ulp", "fp64_fp32_init")


def _ulp_positions(d):
    return dict(d, xi=np.nextafter(d["xi"], np.inf))


def _fp32_init(sim, ds):
    out = []
    for r, d in enumerate(ds):
        p = sim.particles(r)
        xi = np.stack([p["x"][k] / d["dx"][k] for k in range(p["x"].shape[0])])
        out.append(dict(d, xi=xi, u=p["u"], w=p["w"]))
    return out


def _cart_state(sim, runs):
    out = []
    for r in range(runs):
        E, B = sim.fields(r)
        out.append((E, B, np.stack([sim.current(r, c) for c in range(3)])))
    return out


def _errs(st, ref):
    return [{k: rel_l2(a[i], b[i]) for i, k in enumerate("EBJ")} for a, b in zip(st, ref)]


def _checkpoint_loop(sims, read, steps, checkpoints):
    """Advance every handle of `sims` (fp64 is the reference) to each
    checkpoint and record the per-run errors of the others against it."""
    cps = sorted({c for c in checkpoints if 0 < c < steps} | {steps})
    hist = {k: [] for k in CONTROLS}
    done = 0
    for cp in cps:
        for sim in sims.values():
            sim.step(cp - done)
        done = cp
        ref = read(sims["fp64"])
        for k in CONTROLS:
            hist[k].append(_errs(read(sims[k]), ref))
    diag = [sims["fp32"].diagnostics(r) for r in range(len(hist["fp32"][-1]))]
    for sim in sims.values():
        sim.close()
    return cps, hist, diag


def _single_run_table(cps, hist, diag):
    """Error histories of a one-run handle: per control and component, the
    relative L2 error at each checkpoint; the FP32 form's Gauss residual."""
    out = {"checkpoints": cps}
    for k in CONTROLS:
        out[k] = {c: [float("%.4g" % h[0][c]) for h in hist[k]] for c in "EBJ"}
    out["gauss_rel_l2_fp32"] = diag[0]["gauss_l2"] / max(diag[0]["gauss_ref_l2"], 1e-300)
    return out


def precision_cartesian(hpic, ds, steps, checkpoints):
    """FP32 form and the two FP64 controls against the FP64 form on the
    Cartesian workloads `ds` (one handle each, all runs together)."""
    sims = {"fp32": hpic.from_workloads(ds, "fp32"), "fp64": hpic.from_workloads(ds, "fp64"),
            "fp64_ulp": hpic.from_workloads([_ulp_positions(d) for d in ds], "fp64")}
    sims["fp64_fp32_init"] = hpic.from_workloads(_fp32_init(sims["fp32"], ds), "fp64")
    return _checkpoint_loop(sims, lambda s: _cart_state(s, len(ds)), steps, checkpoints)


def _q3d_sim(hpic, d, prec, x, u, w):
    n1, n2 = d["n"]
    sim = hpic.Sim([hpic.config(n1, n2, d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                                precision=prec, modes=d["modes"])])
    for m in range(d["modes"]):
        sim.set_fields_mode(0, m, d["E"][m], d["B"][m])
    sim.set_particles(0, x, u, w, q_over_m=d["qm"], q=d["q"])
    sim.set_background(0, 2)
    return sim


def _q3d_state(sim, M):
    F = np.stack([np.stack([sim.field_mode(0, c, m) for c in range(6)]) for m in range(M)])
    J = np.stack([np.stack([sim.current_mode(0, c, m) for c in range(3)]) for m in range(M)])
    return [(F[:, :3], F[:, 3:], J)]


def precision_q3d(hpic, d, steps, checkpoints):
    """The same comparison for a quasi-3D handle (every mode's E, B and J)."""
    sims = {"fp32": _q3d_sim(hpic, d, "fp32", d["x"], d["u"], d["w"]),
            "fp64": _q3d_sim(hpic, d, "fp64", d["x"], d["u"], d["w"]),
            "fp64_ulp": _q3d_sim(hpic, d, "fp64", np.nextafter(d["x"], np.copysign(np.inf, d["x"])),
                                 d["u"], d["w"])}
    p = sims["fp32"].particles(0)
    sims["fp64_fp32_init"] = _q3d_sim(hpic, d, "fp64", p["x"], p["u"], p["w"])
    return _checkpoint_loop(sims, lambda s: _q3d_state(s, d["modes"]), steps, checkpoints)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, all_core_seconds=8.0, one_thread_steps=1):
    """FP64 oracle on the host, whole steps of the same workload: with every
    host core (OpenMP; its loops give the same bits for any thread count) for
    about all_core_seconds, then one thread for one_thread_steps."""
    import oracle
    g = oracle.grid2(d["n"][0], d["n"][1], d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                     jbg=d["jbg"])
    npart = d["w"].size
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(ncores, omp) if omp > 0 else ncores

    def run(nthreads, min_s, max_steps):
        oracle.set_threads(nthreads)
        st = oracle.State2(g, d["qm"], d["xi"][0], d["xi"][1], d["u"], d["q"] * d["w"],
                           E=d["E"], B=d["B"])
        steps, t0 = 0, time.perf_counter()
        while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_s):
            st.step(1)
            steps += 1
        return steps, time.perf_counter() - t0

    s_all, t_all = run(threads, all_core_seconds, 10)
    s_one, t_one = run(1, 0.0, one_thread_steps)
    oracle.set_threads(threads)
    return {"value": npart * s_all / t_all, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d full steps of the same workload (%d particles, %dx%d grid), FP64 C "
                      "with OpenMP on %d threads, %.1f s" % (s_all, npart, d["n"][0], d["n"][1],
                                                               threads, t_all),
            "single_thread": {"value": npart * s_one / t_one, "cores": 1,
                              "sample": "%d full step(s), one thread, %.1f s" % (s_one, t_one)},
            "host_cpus": ncores, "cpu_model": cpu_model()}


def scan_leg(hpic, torch, W, steps, tune_steps, precision=True):
    """The 64-run parameter scan in one handle: aggregate particle-steps/s of
    the FP32 form (graph-replayed) and of the FP64 form over `steps` steps;
    with `precision`, fresh handles over the same `steps` give each run's
    FP32-vs-FP64 relative L2 error of E, B and J beside the FP64 controls,
    with the run's gamma, particles per cell and grid."""
    t0 = time.perf_counter()
    ds = W.scan2d()
    params = W.scan2d_params()
    gen_s = time.perf_counter() - t0
    npart = sum(x["w"].size for x in ds)
    warm = 16
    a, t32, _ = run_form(hpic, torch, ds, "fp32", warm, steps, tune_steps=tune_steps)
    tiling = a.tuning
    a.close()
    b, t64, _ = run_form(hpic, torch, ds, "fp64", warm, steps, tiling=_as_tiling(tiling))
    b.close()
    v32 = npart * steps / t32
    v64 = npart * steps / t64
    out = {"workload": "scan2d_64runs", "runs": len(ds), "particles": npart,
           "cells": int(sum(x["n"][0] * x["n"][1] for x in ds)), "steps": steps,
           "value": v32, "unit": "particle-steps/s", "ms_per_step": 1e3 * t32 / steps,
           "fp64_form": {"value": v64, "ms_per_step": 1e3 * t64 / steps,
                         "fp32_speedup": v32 / v64},
           "generate_s": gen_s, "tiling": tiling,
           "note": "autotuner (%d steps) and warm-up (%d steps) before the timed region"
                   % (tune_steps, warm)}
    if precision:
        cps, hist, diag = precision_cartesian(hpic, ds, steps, (10, 30, 100))
        fin = {k: hist[k][-1] for k in CONTROLS}
        runs = []
        for r, p in enumerate(params):
            runs.append([p["n1"], p["n2"], p["ppc"], round(p["gamma"], 2), round(p["density"], 3)] +
                        [float("%.3g" % fin["fp32"][r][c]) for c in "EBJ"] +
                        [float("%.3g" % fin["fp64_ulp"][r]["E"]),
                         float("%.3g" % fin["fp64_fp32_init"][r]["E"]),
                         float("%.3g" % (diag[r]["gauss_l2"] / max(diag[r]["gauss_ref_l2"], 1e-300)))])
        e32 = np.array([fin["fp32"][r]["E"] for r in range(len(ds))])
        einit = np.array([fin["fp64_fp32_init"][r]["E"] for r in range(len(ds))])
        eulp = np.array([fin["fp64_ulp"][r]["E"] for r in range(len(ds))])
        med = {k: {c: [float("%.3g" % np.median([h[r][c] for r in range(len(ds))]))
                       for h in hist[k]] for c in "EBJ"} for k in CONTROLS}
        out["precision"] = {
            "steps": steps, "checkpoints": cps,
            "median_over_runs": med,
            "fp32_E": {"max": float(e32.max()), "median": float(np.median(e32))},
            "fp32_E_over_fp32_init_E": {"max": float((e32 / einit).max()),
                                        "median": float(np.median(e32 / einit))},
            "ulp64_E": {"max": float(eulp.max()), "median": float(np.median(eulp))},
            "per_run_columns": ["n1", "n2", "ppc", "gamma", "density", "E", "B", "J",
                                "E_fp64_ulp", "E_fp64_fp32_init", "gauss_rel_fp32"],
            "per_run": runs}
    return out


def d3_leg(hpic, torch, W, steps, tune_steps, precision=True, fixed_tiling=None):
    """3D Cartesian leg: 512 x 128 x 128 cells, 16.8M particles, gamma = 50,
    density +-5%.  Particle-steps/s of the FP32 form (graph-replayed) and the
    FP64 form over `steps` steps, the Gauss and continuity residuals of the
    FP32 form, and with `precision`, fresh handles over the same `steps` for
    the FP32-vs-FP64 errors of E, B and J beside the FP64 controls."""
    d = W.drift3d()
    npart = d["w"].size
    warm = 10
    tune = min(tune_steps, 400)
    a, t32, kt = run_form(hpic, torch, [d], "fp32", warm, steps, profile=True, tune_steps=tune,
                          tiling=fixed_tiling)
    kt.pop("profiled_wall_s")
    push_stats = kt.pop("push_stats")
    tiling = a.tuning
    a.diagnostics(0)
    a.step(1)
    da = a.diagnostics(0)
    a.close()
    b, t64, _ = run_form(hpic, torch, [d], "fp64", warm, steps,
                         tiling=fixed_tiling or _as_tiling(tiling))
    tiling64 = b.tuning
    b.close()
    v32 = npart * steps / t32
    pd_ms, pd_n = kt["push_deposit"]
    cells = int(np.prod(d["n"]))
    rho_scale = abs(da["charge_total"]) / (cells * float(np.prod(d["dx"])))
    out = {"workload": d["name"], "n": list(d["n"]), "particles": npart, "steps": steps,
           "value": v32, "unit": "particle-steps/s", "ms_per_step": 1e3 * t32 / steps,
           "fp64_form": {"value": npart * steps / t64, "ms_per_step": 1e3 * t64 / steps,
                         "fp32_speedup": t64 / t32, "tiling": tiling64},
           "kernels": {k: {"avg_us": 1e3 * ms / max(n, 1), "launches": n} for k, (ms, n) in kt.items()},
           "lds_fallback_tiles": push_stats["fallback_tiles"], "tiling": tiling,
           "residuals_fp32": {"after_steps": da["step"],
                              "gauss_rel_l2": da["gauss_l2"] / max(da["gauss_ref_l2"], 1e-300),
                              "continuity_linf_rel": da["cont_linf"] * d["dt"] / max(rho_scale, 1e-300)},
           "push_deposit_alg_GBps": (60 * npart + 72 * cells) / (pd_ms / max(pd_n, 1) * 1e-3) / 1e9}
    out["push_deposit_frac"] = out["push_deposit_alg_GBps"] / HBM_PEAK_GBS
    out["push_deposit_traffic"] = measured_traffic(D3_COUNTERS, D3_SOURCES, "push_deposit.")
    if precision:
        out["err_vs_fp64"] = _single_run_table(*precision_cartesian(hpic, [d], steps, (10, 30, 100, 300)))
    return out


def q3d_leg(hpic, torch, W, steps, precision=True):
    """Quasi-3D PIC step: 4096 (z) x 256 (r) cells, dz = 0.1, dr = 0.2, dt =
    0.04, azimuthal modes 0, 1, 2 advanced together (one launch per stage), a
    plasma column of 8 192 000 particles drifting at gamma = 20 over a
    co-drifting background, and an m = 1 seed pulse (synthetic, seeded).  Both
    forms over the same steps: particle-steps/s, per-kernel times, the
    push+deposit kernel's algorithmic GB/s, the change of the Gauss residual
    norm (constant in exact arithmetic); with `precision`, fresh handles over
    `steps` steps for the FP32-vs-FP64 errors of every mode's E, B and J beside
    the FP64 controls."""
    d = W.drift_q3d()
    n1, n2 = d["n"]
    M = d["modes"]
    npart = d["w"].size
    out = {"workload": d["name"], "n": [n1, n2], "modes": M, "particles": npart, "steps": steps}
    for prec in ("fp32", "fp64"):
        sim = hpic.Sim([hpic.config(n1, n2, d["dx"][0], d["dx"][1], d["dt"], alpha=d["alpha"],
                                    precision=prec, modes=M)], stream=torch.cuda.current_stream())
        for m in range(M):
            sim.set_fields_mode(0, m, d["E"][m], d["B"][m])
        sim.set_particles(0, d["x"], d["u"], d["w"], q_over_m=d["qm"], q=d["q"])
        sim.set_background(0, 2)
        g0 = sim.diagnostics(0)["gauss_l2"]
        t = timed_steps(torch, sim, 10, steps)
        sim.profile(True)
        sim.step(steps)
        kt = sim.kernel_times()
        sim.profile(False)
        dg = sim.diagnostics(0)
        sim.close()
        out[prec] = {"ms_per_step": 1e3 * t / steps,
                     "particle_steps_per_s": npart * steps / t,
                     "kernels": {k: {"avg_us": 1e3 * ms / n, "launches": n}
                                 for k, (ms, n) in kt.items() if n > 0},
                     "gauss_l2_change": abs(dg["gauss_l2"] - g0) / max(g0, 1e-300),
                     "kinetic": dg["kinetic"],
                     "field_energy": sum(dg["W_E"]) + sum(dg["W_B"])}
        if prec == "fp32":
            pd_ms, pd_n = kt["push_deposit"]
            alg = Q3D_BYTES_PER_PARTICLE * npart + Q3D_BYTES_PER_MODE_NODE * M * (n2 + 1) * n1
            out["push_deposit_alg_GBps"] = alg / (pd_ms / max(pd_n, 1) * 1e-3) / 1e9
            out["push_deposit_alg_bytes"] = alg
            out["push_deposit_frac"] = out["push_deposit_alg_GBps"] / HBM_PEAK_GBS
            out["push_deposit_traffic"] = measured_traffic(Q3D_COUNTERS, Q3D_SOURCES,
                                                           "push_deposit.")
    out["fp32_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"]
    if precision:
        out["err_vs_fp64"] = _single_run_table(*precision_q3d(hpic, d, steps, (10, 30, 100, 300)))
    return out


def nci_leg(steps):
    """The Table 1 drift (256x256, gamma = 50, n = 100, FP32 form) without the
    k1 filter, with it, with the Eq. (29) modification and with that and the
    cubic shape: log10 of the E2 energy at t = 160, 320 and the end, the
    wavenumber of the strongest E2 mode at the end, and the wall time."""
    import math
    from paper_1502_01376_amd import nci
    t0 = time.time()
    res = nci.run(tuple(nci.CASES), steps=steps, every=500)
    out = {"steps": steps, "t_end": steps * 0.08}
    for name, r in res.items():
        t = np.asarray(r["t"])
        lw = [math.log10(max(w, 1e-300)) for w in r["W_E2"]]
        pick = {"log10_W_E2_t%g" % tt: round(lw[int(np.argmin(np.abs(t - tt)))], 3)
                for tt in (160.0, 320.0) if tt <= t[-1]}
        out[name] = dict(pick, log10_W_E2_end=round(lw[-1], 3),
                         peak_k1_over_kg1=round(r["peak"]["k1_over_kg1"], 4),
                         peak_k2=round(r["peak"]["k2"], 4))
    # (0, 0) modes against the time step (filter on): growth rate and k1,
    # measured and from the Appendix A linear theory of the same scheme
    from paper_1502_01376_amd import nci_theory
    ratios = (0.25, 0.3, 0.35, 0.4, 0.45, 0.5)
    scan = nci.dt_scan(ratios=ratios, steps=30000)
    theory = nci_theory.dt_scan(ratios=ratios)
    out["dt_scan"] = []
    for r, th in zip(scan, theory):
        e = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()
             if k in ("ratio", "growth_rate", "k1_over_kg1")}
        e["theory_growth_rate"] = round(th["growth_rate"], 5)
        e["theory_k1_over_kg1"] = round(th["k1_over_kg1"], 4)
        out["dt_scan"].append(e)
    out["wall_s"] = round(time.time() - t0, 2)
    return out


def lwfa_leg(hpic, torch, W, steps):
    """The Table 2 boosted-frame laser wakefield run (8192x512, gamma_b = 14,
    16 777 216 particles, laser from the moving antenna), FP32 form, graph-
    replayed: particle-steps/s and per-kernel times of the filtered run, then on
    axis the laser amplitude against a0 omega', the wake's peak E1 and the
    largest E1 ahead of the laser (numerical Cherenkov noise), with the k1
    filter and without it."""
    d = W.lwfa_boosted()
    npart = d["w"].size
    lz = d["laser"]
    out = {"workload": d["name"], "n": list(d["n"][:2]), "particles": npart, "steps": steps,
           "t_end": steps * d["dt"]}
    for alpha in (0.5, 1.0):
        sim = hpic.from_workload(d, "fp32", alpha=alpha)
        sim.use_graphs(True)
        if alpha == 0.5:
            sim.step(20)
            sim.synchronize()
            sim.profile(True)
            sim.step(100)
            sim.synchronize()
            kt = sim.kernel_times()
            sim.profile(False)
            done = 120
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps - done)
            sim.synchronize()
            t = time.perf_counter() - t0
            out["ms_per_step"] = 1e3 * t / (steps - done)
            out["particle_steps_per_s"] = npart * (steps - done) / t
            out["kernels_us"] = {k: 1e3 * ms / max(n, 1) for k, (ms, n) in kt.items() if n > 0}
        else:
            sim.step(steps)
        E, _ = sim.fields(0)
        e1, e3 = E[0, d["n"][1] // 2], E[2, d["n"][1] // 2]
        key = "filter" if alpha == 0.5 else "no_filter"
        out[key] = {"laser_amplitude_over_a0_omega": float(np.abs(e3).max() / (lz["a0"] * lz["omega"])),
                    "wake_E1_max": float(np.abs(e1).max()),
                    "E1_max_ahead_of_laser": float(np.abs(e1[2000:7000]).max())}
        sim.close()
    return out


def shape_leg(hpic, torch, d, steps, tune_steps, tiling):
    """The benchmark workload (2048x512, 8 388 608 particles, FP32 form) with
    the energy-conserving gather and with the cubic shape, each over `steps`
    steps after the same warm-up: particle-steps/s and push+deposit time."""
    npart = d["w"].size
    out = {"steps": steps}
    for name, kw in (("energy_conserving", dict(interp=1)), ("cubic", dict(shape=3)),
                     ("cubic_energy_conserving", dict(shape=3, interp=1))):
        sim, t, kt = run_form(hpic, torch, [d], "fp32", 20, steps, profile=True,
                              tune_steps=tune_steps if "cubic" not in name else 0,
                              tiling=tiling, **kw)
        kt.pop("profiled_wall_s", None)
        pd_ms, pd_n = kt["push_deposit"]
        out[name] = {"particle_steps_per_s": npart * steps / t, "ms_per_step": 1e3 * t / steps,
                     "push_deposit_us": 1e3 * pd_ms / max(pd_n, 1)}
        sim.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1502_01376_amd import hpic
    from paper_1502_01376_amd import workloads as W

    d = W.drift2d_laser(n1=args.n1, n2=args.n2)
    npart = d["w"].size
    ncell = d["n"][0] * d["n"][1]

    tiling = [int(v) for v in args.tiling.split(",")] if args.tiling else None
    sim32, t32, kt = run_form(hpic, torch, [d], "fp32", args.warmup, args.steps, profile=True,
                              tune_steps=args.tune_steps, tiling=tiling)
    chosen = sim32.tuning
    profiled_wall = kt.pop("profiled_wall_s")
    value = npart * args.steps / t32
    ms_step = 1e3 * t32 / args.steps
    pd_ms, pd_n = kt["push_deposit"]
    pd_avg_s = pd_ms / max(pd_n, 1) * 1e-3
    alg_bytes = BYTES_PER_PARTICLE * npart + BYTES_PER_CELL * ncell
    achieved = alg_bytes / pd_avg_s / 1e9
    push_stats = kt.pop("push_stats")
    kernels = {k: {"avg_us": 1e3 * ms / max(n, 1), "launches": n} for k, (ms, n) in kt.items()}
    kernels["push_deposit"]["lds_fallback_tiles"] = push_stats["fallback_tiles"]
    kernels["push_deposit"]["tiles"] = push_stats["tiles"]
    sim32.close()

    out = {
        "metric": "particle-steps/sec (push+deposit+hybrid solve), FP32-batched vs FP64 at stated err",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": d["name"], "n1": d["n"][0], "n2": d["n"][1],
                   "dx": list(d["dx"][:2]), "dt": d["dt"], "particles": npart,
                   "particles_per_cell": 8, "gamma": 20.0, "laser_a0": 2.0,
                   "filter_frac": d["alpha"], "deposit_accumulator": "int64 fixed point",
                   "field_state": "FP64 k-space master of E and B, updated in FP64 (both "
                                  "forms); FP32 real-space fields, push and deposit weights",
                   "sort_interval": chosen["sort_interval"],
                   "sorts_in_timed_region": -(-args.steps // max(chosen["sort_interval"], 1)),
                   "parallelism": "single GPU"},
        "kernels": kernels,
        "tiling": chosen,
        "roofline": {"bound": "hbm", "kernel": "push_deposit", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "alg_bytes_per_launch": alg_bytes,
                     "source_hash": source_hash(),
                     "timing": "HIP events around each launch in a profiled pass of %d steps "
                               "(%.4f ms/step with the events)" % (args.steps,
                                                                     1e3 * profiled_wall / args.steps)},
    }

    if args.fp64_steps < 0:
        args.fp64_steps = args.steps
    if args.fp64_steps > 0:
        sim64, t64, _ = run_form(hpic, torch, [d], "fp64", args.warmup, args.fp64_steps,
                                 tiling=tiling or _as_tiling(chosen))
        sim64.close()
        out["fp64_form"] = {"value": npart * args.fp64_steps / t64,
                            "ms_per_step": 1e3 * t64 / args.fp64_steps,
                            "steps": args.fp64_steps,
                            "fp32_speedup": value / (npart * args.fp64_steps / t64)}
    if args.err_steps > 0:
        cps, hist, diag = precision_cartesian(hpic, [d], args.err_steps, (10, 30, 100, 300))
        tab = _single_run_table(cps, hist, diag)
        out["err_vs_fp64"] = {"steps": args.err_steps, "E_rel_l2": tab["fp32"]["E"][-1],
                              "B_rel_l2": tab["fp32"]["B"][-1], "J_rel_l2": tab["fp32"]["J"][-1],
                              "gauss_rel_l2_fp32": tab["gauss_rel_l2_fp32"], "history": tab}
    if args.scan_steps > 0:
        out["scan2d"] = scan_leg(hpic, torch, W, args.scan_steps, args.tune_steps, args.precision)
    if args.d3_steps > 0:
        d3t = [int(v) for v in args.d3_tiling.split(",")] if args.d3_tiling else None
        out["drift3d"] = d3_leg(hpic, torch, W, args.d3_steps, args.tune_steps, args.precision, d3t)
    if args.q3d_steps > 0:
        out["quasi3d"] = q3d_leg(hpic, torch, W, args.q3d_steps, args.precision)
    if args.shape_steps > 0:
        out["shapes2d"] = shape_leg(hpic, torch, d, args.shape_steps, args.tune_steps, tiling)
    if args.nci_steps > 0:
        out["nci_table1"] = nci_leg(args.nci_steps)
    if args.lwfa_steps > 0:
        out["lwfa_boosted"] = lwfa_leg(hpic, torch, W, args.lwfa_steps)
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * n * 4
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
