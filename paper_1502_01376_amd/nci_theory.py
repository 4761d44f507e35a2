"""Linear theory of the numerical Cerenkov instability (NCI) of a cold plasma
drifting along x1, for the hybrid solver (Sec. 3 and Appendix A).

Appendix A gives the numerical dispersion relation of one aliased beam
resonance (mu, nu1): the beam term times the electromagnetic term plus a
coupling C (Eqs. (A.1)-(A.2)), with the hybrid solver's symbols [k]_E1 =
[k]_B1 = k1 (spectral along x1) and [k]_E2 = [k]_B2 = sin(k2 dx2/2)/(dx2/2)
(Eq. (A.3)); and, expanding about the resonance omega' = k1' v0, a cubic in
the frequency shift (Eqs. (A.4)-(A.6)).  Its readings, where the printed text
is garbled or silent:

* the interpolation factor of one axis is the Fourier transform of the order-l
  B-spline at the aliased wavenumber, s_l(k) = (sin(k dx/2)/(k dx/2))^(l+1)
  (the printed s_l drops the k in the denominator), with (-1)^nu1 for
  quantities on half nodes along x1 (E1, B2, B3, j1);
* the printed S_E1 is given twice and S_E3 never: the second one is S_E3,
  which does not enter the 2D relation;
* B3 reaches the particles at integer time as the mean of its two half-step
  values, a factor cos(omega dt/2): S_B3 = S'_B3 cos(omega dt/2) in (A.1),
  which is what the zeta0, zeta1 terms of the cubic expand;
* the current of the charge-conserving deposit has the order l - 1 along its
  own axis (S_j1 = s_{l-1}(k1') s_l(k2), S_j2 = s_l(k1') s_{l-1}(k2)); the
  current correction of Eq. (11) multiplies j1 by [k]1,FD/[k]1 at the grid
  wavenumber, and the low-pass filter multiplies both by f(k1) (reading:
  `corrected=True`, the scheme the GPU path runs; False gives the printed
  S_j1);
* the Eq. (29) modification replaces [k]_E1 = [k]_B1 by k1 + dk_mod(k1).

Units: c = 1, frequencies in the reference plasma frequency; the beam's
plasma frequency squared is its density n (Table 1: n = 100).  Growth rates
are Im(omega), the amplitude growth rate.
"""
import math

import numpy as np


class Params:
    """Grid, time step and beam of the drifting-plasma set-up (Table 1 by
    default: dx = (0.2, 0.2), dt = 0.4 dx1, gamma = 50, n = 100)."""

    def __init__(self, dx1=0.2, dx2=0.2, dt=0.08, gamma=50.0, density=100.0, shape=2,
                 interp="momentum", corrected=True, alpha=0.5, kmod=None):
        self.dx1, self.dx2, self.dt = float(dx1), float(dx2), float(dt)
        self.gamma = float(gamma)
        self.v0 = math.sqrt(1.0 - 1.0 / self.gamma ** 2)
        self.wp2 = float(density)
        self.l = int(shape)
        self.interp = interp
        self.corrected = bool(corrected)
        self.alpha = float(alpha)
        self.kmod = kmod  # None or (k1l, k1u, dkmax) in units of kg1
        self.kg1 = 2 * math.pi / self.dx1
        self.wg = 2 * math.pi / self.dt


def sinc_pow(k, dx, p):
    """(sin(k dx/2)/(k dx/2))^p, 1 at k = 0."""
    x = np.asarray(k, dtype=float) * dx / 2
    s = np.where(np.abs(x) < 1e-12, 1.0, np.sin(x) / np.where(x == 0, 1.0, x))
    return s ** p


def dk_mod(k1, prm):
    """Eq. (29): the bump added to the spectral symbol on k1l <= |k1| <= k1u
    (odd in k1)."""
    k1 = np.asarray(k1, dtype=float)
    if prm.kmod is None:
        return np.zeros_like(k1)
    lo, hi, dmax = (v * prm.kg1 for v in prm.kmod)
    mid = 0.5 * (lo + hi)
    a = np.abs(k1)
    bump = dmax * np.cos((a - mid) / (lo - mid) * math.pi / 2) ** 2
    return np.where((a >= lo) & (a <= hi), np.sign(k1) * bump, 0.0)


def symbols(k1, k2, mu, nu1, prm):
    """Operators and interpolation factors of Eqs. (A.1)-(A.6) at the grid
    wavenumber (k1, k2) for the resonance (mu, nu1).  S_B3 is returned
    without its time factor (S'_B3)."""
    k1 = np.asarray(k1, dtype=float)
    k2 = np.asarray(k2, dtype=float)
    l = prm.l
    k1a = k1 + nu1 * prm.kg1                       # aliased x1 wavenumber
    sgn = (-1.0) ** nu1
    kE1 = k1 + dk_mod(k1, prm)                     # spectral (or modified) along x1
    kE2 = np.sin(k2 * prm.dx2 / 2) / (prm.dx2 / 2)  # Yee along x2
    s1 = lambda p: sinc_pow(k1a, prm.dx1, p)
    s2 = lambda p: sinc_pow(k2, prm.dx2, p)
    if prm.interp == "momentum":
        SE1 = s1(l + 1) * s2(l + 1) * sgn
        SE2 = s1(l + 1) * s2(l + 1)
        SB3 = s1(l + 1) * s2(l + 1) * sgn
    else:  # energy-conserving: one order lower along each staggered direction
        SE1 = s1(l) * s2(l + 1) * sgn
        SE2 = s1(l + 1) * s2(l)
        SB3 = s1(l) * s2(l) * sgn
    Sj1 = s1(l) * s2(l + 1) * sgn
    Sj2 = s1(l + 1) * s2(l)
    if prm.corrected:
        fd = np.sin(k1 * prm.dx1 / 2) / (prm.dx1 / 2)
        Sj1 = Sj1 * np.where(kE1 == 0, 1.0, fd / np.where(kE1 == 0, 1.0, kE1))
    filt = np.where(np.abs(k1) <= prm.alpha * math.pi / prm.dx1 * (1 + 1e-12), 1.0, 0.0)
    return dict(k1a=k1a, kE1=kE1, kE2=kE2, SE1=SE1, SE2=SE2, SB3=SB3, Sj1=Sj1 * filt,
                Sj2=Sj2 * filt)


def dispersion(omega, k1, k2, mu, nu1, prm):
    """Left-hand side of Eq. (A.1) with the coupling term (A.2) at the complex
    frequency omega."""
    sy = symbols(k1, k2, mu, nu1, prm)
    w = np.asarray(omega, dtype=complex)
    h = prm.dt / 2
    ww = np.sin(w * h) / h                         # [omega]
    wp = w + mu * prm.wg                           # omega'
    res = wp - sy["k1a"] * prm.v0                  # omega' - k1' v0
    sm = (-1.0) ** mu
    g = prm.gamma
    SB3 = sy["SB3"] * np.cos(w * h)
    kk = sy["kE1"] ** 2 + sy["kE2"] ** 2
    beam = res ** 2 - prm.wp2 / g ** 3 * sm * sy["Sj1"] * sy["SE1"] * wp / ww
    em = ww ** 2 - kk - prm.wp2 / g * sm * sy["Sj2"] * (sy["SE2"] * ww - SB3 * sy["kE1"] * prm.v0) / res
    k2v = np.asarray(k2, dtype=float)
    C = prm.wp2 / g * sm / ww * (
        sy["Sj1"] * sy["SE1"] * wp * sy["kE2"] ** 2 * (prm.v0 ** 2 - 1)
        + sy["Sj2"] * sy["SE2"] * sy["kE2"] ** 2 * res
        + sy["Sj1"] * sy["kE2"] * (sy["SE2"] * sy["kE1"] * k2v * prm.v0
                                   - SB3 * k2v * prm.v0 ** 2 * ww))
    return beam * em + C


def cubic_coefficients(k1, k2, mu, nu1, prm):
    """A2, B2, C2, D2 of Eqs. (A.4)-(A.5) (with the printed v0 -> 1 in the
    expansion point k1~ = k1 + nu1 kg1 - mu omega_g, Eq. (A.6))."""
    sy = symbols(k1, k2, mu, nu1, prm)
    h = prm.dt / 2
    kt = sy["k1a"] - mu * prm.wg
    xi0 = np.sin(kt * h) / h
    xi1 = np.cos(kt * h)
    ze0 = np.cos(kt * h)
    ze1 = -np.sin(kt * h) * h
    f = prm.wp2 / prm.gamma * (-1.0) ** mu
    k2v = np.asarray(k2, dtype=float)
    kE1, kE2 = sy["kE1"], sy["kE2"]
    Sj1, Sj2, SE2, SB3 = sy["Sj1"], sy["Sj2"], sy["SE2"], sy["SB3"]
    A2 = 2 * xi0 ** 3 * xi1
    B2 = xi0 ** 2 * (xi0 ** 2 - kE1 * kE1 - kE2 * kE2 - f * Sj2 * (SE2 * xi1 - ze1 * SB3 * kE1))
    C2 = f * (xi0 ** 2 * Sj2 * (ze0 * SB3 * kE1 - SE2 * xi0) - xi1 * Sj1 * kE2 * k2v * SE2 * kE1
              + xi0 * kE2 * (Sj2 * SE2 * kE2 - Sj1 * k2v * ze1 * SB3 * xi0))
    D2 = f * xi0 * kE2 * k2v * Sj1 * (SE2 * kE1 - ze0 * SB3 * xi0)
    return A2, B2, C2, D2


def cubic_roots(k1, k2, mu, nu1, prm):
    """The three roots delta omega' of Eq. (A.4) at one (k1, k2)."""
    A2, B2, C2, D2 = (float(v) for v in cubic_coefficients(k1, k2, mu, nu1, prm))
    if A2 == 0.0:
        return np.array([], dtype=complex)
    return np.roots([A2, B2, C2, D2])


def refine(omega0, k1, k2, mu, nu1, prm, steps=30, tol=1e-12):
    """Newton's method on Eq. (A.1) from omega0 (complex step derivative by
    central differences); returns the root or None if it does not converge."""
    w = complex(omega0)
    for _ in range(steps):
        d = dispersion(w, k1, k2, mu, nu1, prm)
        e = 1e-7 * max(1.0, abs(w))
        dd = (dispersion(w + e, k1, k2, mu, nu1, prm) - dispersion(w - e, k1, k2, mu, nu1, prm)) / (2 * e)
        if dd == 0:
            return None
        step = complex(d / dd)
        w -= step
        if abs(step) < tol * max(1.0, abs(w)):
            return w
    return None


def unstable_root(k1, k2, mu, nu1, prm):
    """Growing root near the resonance at (k1, k2): the cubic's root with the
    largest imaginary part, refined on the full relation; None if the cubic
    has no growing root or the refinement leaves its neighbourhood."""
    r = cubic_roots(k1, k2, mu, nu1, prm)
    if r.size == 0:
        return None
    d = r[np.argmax(r.imag)]
    if d.imag <= 0:
        return None
    sy = symbols(k1, k2, mu, nu1, prm)
    w0 = float(sy["k1a"]) * prm.v0 - mu * prm.wg + d
    w = refine(w0, k1, k2, mu, nu1, prm)
    if w is None or abs(w - w0) > 0.5 * abs(d) + 1e-9:
        return None
    return w


def _cubic_grid(k1, k2, mu, nu1, prm):
    K1, K2 = np.meshgrid(k1, k2, indexing="ij")
    A2, B2, C2, D2 = cubic_coefficients(K1, K2, mu, nu1, prm)
    g = np.zeros(K1.shape)
    for a in range(K1.shape[0]):
        for b in range(K1.shape[1]):
            if A2[a, b] != 0.0:
                r = np.roots([A2[a, b], B2[a, b], C2[a, b], D2[a, b]])
                g[a, b] = max(0.0, r.imag.max())
    return g


def growth_map(prm, mu=0, nu1=0, n1=96, n2=96, k1_range=None):
    """Im(omega) of the growing root over k1 in (0, pi/dx1] (or k1_range, in
    units of kg1) and k2 in (0, pi/dx2] from the cubic (vectorised); zero
    where it has none."""
    lo, hi = (1e-3, 0.5) if k1_range is None else k1_range
    k1 = np.linspace(lo, hi, n1) * prm.kg1
    k2 = np.linspace(0.5 / n2, 1.0, n2) * math.pi / prm.dx2
    return k1, k2, _cubic_grid(k1, k2, mu, nu1, prm)


def fastest(prm, mu=0, nu1=0, n1=96, n2=96, k1_range=None, zoom=2, refine_top=12):
    """The fastest-growing mode of resonance (mu, nu1): a scan of the zone
    with the cubic (A.4), zoomed `zoom` times around its maximum; the
    `refine_top` largest points of the last grid are then refined on the full
    relation (A.1) and the largest imaginary part kept.  Returns the growth
    rate (Im omega; the cubic's where no refinement converged), k1/kg1,
    k2 dx2/(2 pi), the cubic's maximum and whether the full relation gave the
    value."""
    k1, k2, g = growth_map(prm, mu, nu1, n1, n2, k1_range)
    for _ in range(zoom):
        i, j = np.unravel_index(np.argmax(g), g.shape)
        if g[i, j] <= 0:
            break
        d1 = (k1[1] - k1[0]) * 2 / prm.kg1
        c1 = k1[i] / prm.kg1
        d2 = (k2[1] - k2[0]) * 2
        c2 = k2[j]
        k1 = np.linspace(max(c1 - d1, 1e-4), c1 + d1, n1 // 2) * prm.kg1
        k2 = np.linspace(max(c2 - d2, 1e-6), min(c2 + d2, math.pi / prm.dx2), n2 // 2)
        g = _cubic_grid(k1, k2, mu, nu1, prm)
    i, j = np.unravel_index(np.argmax(g), g.shape)
    est = float(g[i, j])
    out = {"growth_rate_cubic": est, "growth_rate": est, "full_relation": False,
           "k1_over_kg1": float(k1[i] / prm.kg1),
           "k2_dx2_over_2pi": float(k2[j] * prm.dx2 / (2 * math.pi))}
    if est <= 0:
        return out
    best = None
    for flat in np.argsort(g, axis=None)[::-1][:refine_top]:
        a, b = np.unravel_index(flat, g.shape)
        if g[a, b] <= 0:
            break
        w = unstable_root(k1[a], k2[b], mu, nu1, prm)
        if w is not None and (best is None or w.imag > best[0]):
            best = (w.imag, a, b)
    if best is not None:
        out.update(growth_rate=float(best[0]), full_relation=True,
                   k1_over_kg1=float(k1[best[1]] / prm.kg1),
                   k2_dx2_over_2pi=float(k2[best[2]] * prm.dx2 / (2 * math.pi)))
    return out


def dt_scan(ratios=(0.25, 0.3, 0.35, 0.4, 0.45, 0.5), **kw):
    """Fig. 2 (a)-(b), theory: growth rate and k1/kg1 of the fastest (0, 0)
    mode against dt/dx1 for the Table 1 drift (hybrid solver)."""
    out = []
    for r in ratios:
        prm = Params(dt=r * kw.get("dx1", 0.2), **kw)
        f = fastest(prm, 0, 0, k1_range=(0.05, 0.45))
        out.append(dict(ratio=r, **f))
    return out
