"""NCI contrast harness on the relativistic plasma drift of Table 1.

A cold plasma (n = 100 n_p, gamma = 50) drifts along x1 through a periodic
51.2 x 51.2 box of 256 x 256 cells (dx = 0.2, dt = 0.4 dx1 = 0.08).  The
numerical Cherenkov instability grows from the particle noise; Sec. 3-4
follow it through the energy in E2:

* without the k1 low-pass filter of the current (filter fraction 1) the
  (mu, nu1) = (0, +-1) modes near the edge of the k1 Brillouin zone grow
  fastest;
* with the filter at half the x1 Nyquist wavenumber they are gone and the
  slower (0, 0) modes at k1 / kg1 of about 0.15-0.26 remain;
* the modified spectral symbol of Eq. (29) removes those as well, leaving the
  (+-1, +-2) modes, which the cubic particle shape weakens further (Fig. 3).

``run`` advances any set of such cases on the GPU (cases that share the
particle shape and gather go into one batched handle) and returns the E2
energy history of each, the fitted growth rate over a window and the location
in (k1, k2) of the strongest E2 mode at the end.  Everything runs through the
C-ABI library; this module only sets the runs up and reads diagnostics.
"""
import math

import numpy as np

from . import hpic
from . import workloads as W

# The four runs of Fig. 3 plus the unfiltered reference of Sec. 3.
CASES = {
    "no_filter": dict(alpha=1.0, kmod=0, shape=2),
    "filter": dict(alpha=0.5, kmod=0, shape=2),
    "filter_kmod": dict(alpha=0.5, kmod=1, shape=2),
    "filter_kmod_cubic": dict(alpha=0.5, kmod=1, shape=3),
}


def _config(d, precision, alpha, kmod, shape, interp):
    n1, n2, _ = d["n"]
    dx1, dx2, _ = d["dx"]
    return hpic.config(n1, n2, dx1, dx2, d["dt"], alpha=alpha, precision=precision, kmod=kmod,
                       shape=shape, interp=interp)


def peak_mode(E2, dx1, dx2):
    """(k1, k2) of the largest |E2(k1, k2)|^2 of a real [n2][n1] field, with
    k1 >= 0 and k1 / kg1 (kg1 = 2 pi / dx1)."""
    n2, n1 = E2.shape
    s = np.abs(np.fft.rfft2(E2)) ** 2
    s[0, 0] = 0.0
    j, i = np.unravel_index(np.argmax(s), s.shape)
    k1 = 2.0 * math.pi * i / (n1 * dx1)
    k2 = 2.0 * math.pi * (j if j <= n2 // 2 else j - n2) / (n2 * dx2)
    return dict(k1=k1, k2=k2, k1_over_kg1=k1 * dx1 / (2.0 * math.pi),
                k1_over_nyquist=k1 * dx1 / math.pi)


def growth_rate(t, w, lo, hi):
    """Least-squares slope of ln W over lo <= t <= hi, halved: the growth rate
    of the field amplitude (W ~ |E|^2 ~ exp(2 Gamma t))."""
    t = np.asarray(t)
    sel = (t >= lo) & (t <= hi)
    if sel.sum() < 2:
        return float("nan")
    y = np.log(np.maximum(np.asarray(w)[sel], 1e-300))
    return float(0.5 * np.polyfit(t[sel], y, 1)[0])


def run(cases=("no_filter", "filter"), steps=4000, every=50, precision="fp32", ppc=(2, 2),
        n=(256, 256), seed=None, fit=None, graphs=True):
    """Advance each named case (keys of CASES, or dicts alpha/kmod/shape/interp)
    for `steps` steps from the same seeded plasma and record W_E2 every `every`
    steps.  fit = (t_lo, t_hi) adds the growth rate over that window."""
    kw = dict(ppc=ppc, n=n)
    if seed is not None:
        kw["seed"] = seed
    d = W.nci_table1(**kw)
    specs = {}
    for c in cases:
        spec = dict(CASES[c]) if isinstance(c, str) else dict(c)
        spec.setdefault("interp", 0)
        specs[c if isinstance(c, str) else repr(sorted(c.items()))] = spec
    groups = {}
    for name, s in specs.items():
        groups.setdefault((s["shape"], s["interp"]), []).append(name)
    x = np.stack([d["xi"][k] * d["dx"][k] for k in range(2)])
    out = {}
    for (shape, interp), names in groups.items():
        cfgs = [_config(d, precision, specs[nm]["alpha"], specs[nm]["kmod"], shape, interp)
                for nm in names]
        sim = hpic.Sim(cfgs)
        try:
            for r in range(len(names)):
                sim.set_particles(r, x, d["u"], d["w"], d["qm"], d["q"])
                sim.set_background(r, True, d["jbg"])
            if graphs:
                sim.use_graphs(True)
            t, hist = [0.0], [[sim.diagnostics(r)["W_E"][1]] for r in range(len(names))]
            done = 0
            while done < steps:
                k = min(every, steps - done)
                sim.step(k)
                done += k
                t.append(done * d["dt"])
                for r in range(len(names)):
                    hist[r].append(sim.diagnostics(r)["W_E"][1])
            for r, nm in enumerate(names):
                res = dict(spec=specs[nm], t=t, W_E2=hist[r],
                           peak=peak_mode(sim.field(r, 1), d["dx"][0], d["dx"][1]))
                if fit is not None:
                    res["growth_rate"] = growth_rate(t, hist[r], *fit)
                out[nm] = res
        finally:
            sim.close()
    return out


def growth_window(t, w, margin=1.5, min_points=3):
    """Linear-growth window of an energy history: the samples between the
    noise level (median of the first samples) plus `margin` decades and the
    saturation level (the maximum) minus `margin` decades.  Returns
    (t_lo, t_hi) or None."""
    lw = np.log10(np.maximum(np.asarray(w, dtype=float), 1e-300))
    t = np.asarray(t, dtype=float)
    if lw.size < 8:
        return None
    noise = float(np.median(lw[1:6]))
    sat = float(lw.max())
    sel = np.nonzero((lw > noise + margin) & (lw < sat - margin))[0]
    if sel.size < min_points:
        return None
    # the first contiguous stretch
    inside = set(sel.tolist())
    stop = sel[0]
    while stop + 1 in inside:
        stop += 1
    return float(t[sel[0]]), float(t[stop])


def dt_scan(ratios=(0.25, 0.3, 0.35, 0.4, 0.45, 0.5), steps=30000, every=200, precision="fp32",
            ppc=(2, 2), n=(256, 256), seed=None):
    """Growth of the (0, 0) NCI modes against the time step (Sec. 3 and Fig. 2
    (a)-(b): reducing dt lowers their growth rate and raises their k1): the
    Table 1 drift with the k1 filter at half the Nyquist wavenumber, one run
    per dt = ratio dx1 (all in one batched handle), E2 energy and strongest E2
    mode every `every` steps.  Per run: the fitted amplitude growth rate over
    the linear-growth window and the mode's k1/kg1 in the middle of it."""
    kw = dict(ppc=ppc, n=n)
    if seed is not None:
        kw["seed"] = seed
    d = W.nci_table1(**kw)
    n1, n2, _ = d["n"]
    dx1, dx2, _ = d["dx"]
    cfgs = [hpic.config(n1, n2, dx1, dx2, r * dx1, alpha=0.5, precision=precision)
            for r in ratios]
    x = np.stack([d["xi"][k] * d["dx"][k] for k in range(2)])
    sim = hpic.Sim(cfgs)
    try:
        for i in range(len(ratios)):
            sim.set_particles(i, x, d["u"], d["w"], d["qm"], d["q"])
            sim.set_background(i, True, d["jbg"])
        sim.use_graphs(True)
        hist = [[] for _ in ratios]
        peaks = [[] for _ in ratios]
        done = 0
        while done < steps:
            k = min(every, steps - done)
            sim.step(k)
            done += k
            for i in range(len(ratios)):
                hist[i].append(sim.diagnostics(i)["W_E"][1])
                peaks[i].append(peak_mode(sim.field(i, 1), dx1, dx2))
    finally:
        sim.close()
    out = []
    for i, r in enumerate(ratios):
        t = [(j + 1) * every * r * dx1 for j in range(len(hist[i]))]
        win = growth_window(t, hist[i])
        res = dict(ratio=r, dt=r * dx1, t_end=t[-1],
                   log10_W_E2_max=math.log10(max(max(hist[i]), 1e-300)))
        if win is not None:
            res["window"] = win
            res["growth_rate"] = growth_rate(t, hist[i], *win)
            mid = int(np.argmin(np.abs(np.asarray(t) - 0.5 * (win[0] + win[1]))))
            res["k1_over_kg1"] = peaks[i][mid]["k1_over_kg1"]
            res["k2"] = peaks[i][mid]["k2"]
        out.append(res)
    return out


def main(argv=None):
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--cases", default="no_filter,filter,filter_kmod,filter_kmod_cubic")
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--every", type=int, default=200)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--fit", default=None, help="t_lo,t_hi of the growth-rate window")
    ap.add_argument("--history", action="store_true", help="print every recorded W_E2")
    ap.add_argument("--dt-scan", action="store_true",
                    help="growth of the (0, 0) modes against dt/dx1 instead of the four cases")
    a = ap.parse_args(argv)
    if a.dt_scan:
        import time as _t
        t0 = _t.time()
        for r in dt_scan(steps=a.steps, precision=a.precision):
            print(json.dumps(r), flush=True)
        print(json.dumps(dict(wall_s=round(_t.time() - t0, 2))), flush=True)
        return
    fit = tuple(float(v) for v in a.fit.split(",")) if a.fit else None
    t0 = time.time()
    res = run(a.cases.split(","), a.steps, a.every, a.precision, fit=fit)
    for name, r in res.items():
        line = dict(case=name, **r["spec"], t_end=r["t"][-1],
                    log10_W_E2_start=math.log10(max(r["W_E2"][0], 1e-300)),
                    log10_W_E2_end=math.log10(max(r["W_E2"][-1], 1e-300)),
                    log10_W_E2_max=math.log10(max(max(r["W_E2"]), 1e-300)), peak=r["peak"])
        if "growth_rate" in r:
            line["growth_rate"] = r["growth_rate"]
        if a.history:
            line["t"] = r["t"]
            line["log10_W_E2"] = [round(math.log10(max(v, 1e-300)), 4) for v in r["W_E2"]]
        print(json.dumps(line), flush=True)
    print(json.dumps(dict(wall_s=round(time.time() - t0, 2))), flush=True)


if __name__ == "__main__":
    main()
