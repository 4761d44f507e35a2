"""Seeded synthetic inputs for the hybrid Yee-FFT PIC step.

This module holds only input generation: particle loading, momenta, weights
and analytic initial fields.  It contains none of the method's arithmetic (no
gather, push, deposit, transform or field update), so both the oracle-side
tests and the GPU path can take their inputs from it.

Every generator draws from ``numpy.random.Generator(PCG64(seed))``.  Positions
are returned in cell units ``xi = x / dx`` in ``[0, n)``; momenta are
``u = gamma v`` (c = 1); ``w`` is the density weight of each macro-particle
(charge density = q * sum_p w_p * shape), so a uniform density n with ppc
particles per cell has ``w = n / ppc``.

The named workloads are the drifting-plasma set-ups of the benchmark suite:

* ``drift2d_small``  -- 64 x 32 cells, dx = 0.2, dt = 0.05, quiet 2x2 lattice,
  gamma = 50, thermal spread 1e-4, filter at half the x1 Nyquist wavenumber.
* ``drift2d_laser``  -- 2048 x 512 cells, dx = (0.1, 0.2), dt = 0.045,
  4x2 sub-lattice with uniform jitter (8 per cell), gamma = 20 cold, plus a
  linearly polarised Gaussian laser (a0 = 2, waist 8, length 4).
* ``scan2d``  -- a batched parameter scan of independent drifting-plasma runs
  of uneven sizes: per run N1 from {256, 512, 1024, 2048}, N2 from
  {64, 128, 256, 512}, gamma ~ U[5, 100], density ~ U[0.5, 2], 4..16
  particles per cell at uniformly random positions in each cell, dx = 0.2,
  dt = 0.05, thermal spread 1e-4, filter 0.5, 200 steps.

* ``drift3d``  -- 512 x 128 x 128 cells, dx = 0.2, dt = 0.05, a 2x1x1
  lattice (2 per cell, 16 777 216 particles), gamma = 50 cold along x1, per-cell
  density multiplier U[0.95, 1.05] carried in the weights, 500 steps.

* ``drift_q3d``  -- quasi-3D, 4096 (z) x 256 (r) cells, dz = 0.1, dr = 0.2,
  dt = 0.04, modes m = 0, 1, 2; a plasma column of radius 250 dr (the wall is
  at 256 dr) with 2 (z) x 1 (r) x 4 (theta, equally spaced with a random phase
  per cell) particles per cell, weights proportional to r (uniform density 1),
  gamma = 20 cold along z, and an m = 1 seed: a linearly polarised Gaussian
  pulse E_x = a0 exp(-((z - zc)/L)^2 - (r/W)^2) cos(k0 (z - zc)), B_y = -E_x
  (moving along -z), a0 = 1, W = 8, L = 4, k0 = 10.  Positions are Cartesian
  (z, x, y) in physical units, ``w`` the number of physical particles (charge
  q w), fields per mode complex [M][3][n2+1][n1].

The NCI test set-up of Table 1 (dx = 0.2, dt = 0.4 dx1, periodic,
51.2 x 51.2, gamma = 50, n = 100) is ``nci_table1``; the Lorentz-boosted laser
wakefield set-up of Table 2 (8192 x 512, gamma_b = 14, a moving antenna) is
``lwfa_boosted``.
"""
import math

import numpy as np

SEED0 = 1502013760


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def lattice_2d(n1, n2, sub1, sub2, jitter, gen):
    """Positions of a sub1 x sub2 sub-lattice in every cell (cell units).

    With ``jitter`` false each particle sits at the centre of its sub-cell
    (offsets 1/4, 3/4 for two per direction); with ``jitter`` true it is placed
    uniformly at random inside its sub-cell.
    """
    i1 = np.arange(n1, dtype=np.float64)
    i2 = np.arange(n2, dtype=np.float64)
    a = (np.arange(sub1, dtype=np.float64) + 0.5) / sub1
    b = (np.arange(sub2, dtype=np.float64) + 0.5) / sub2
    # particle order: cell-major (i2, i1), then sub-cell (b, a)
    x1 = (i1[None, :, None, None] + a[None, None, None, :]) + 0.0 * b[None, None, :, None]
    x2 = (i2[:, None, None, None] + b[None, None, :, None]) + 0.0 * a[None, None, None, :]
    x1 = np.broadcast_to(x1, (n2, n1, sub2, sub1)).reshape(-1).copy()
    x2 = np.broadcast_to(x2, (n2, n1, sub2, sub1)).reshape(-1).copy()
    if jitter:
        x1 += (gen.random(x1.size) - 0.5) / sub1
        x2 += (gen.random(x2.size) - 0.5) / sub2
    x1 = np.mod(x1, n1)
    x2 = np.mod(x2, n2)
    return x1, x2


def random_in_cells(n1, n2, ppc, gen):
    """ppc particles per cell at uniformly random positions inside the cell
    (cell units), cell-major order."""
    base1 = np.tile(np.arange(n1, dtype=np.float64), n2)
    base2 = np.repeat(np.arange(n2, dtype=np.float64), n1)
    x1 = np.repeat(base1, ppc) + gen.random(n1 * n2 * ppc)
    x2 = np.repeat(base2, ppc) + gen.random(n1 * n2 * ppc)
    # a draw of exactly 1 - 2^-53 plus the cell index may round up to the next cell
    return np.mod(x1, n1), np.mod(x2, n2)


def drift_momenta(npart, gamma, sigma_u, gen):
    """u = (sqrt(gamma^2 - 1), 0, 0) plus a Gaussian spread sigma_u per component."""
    u = np.zeros((3, npart))
    u[0] = math.sqrt(gamma * gamma - 1.0)
    if sigma_u > 0:
        u += sigma_u * gen.standard_normal((3, npart))
    return u


def mean_current(u, w, q, ncells):
    """Uniform current density of the loaded particles: sum_p q w_p v_p / ncells.

    This is the background current of infinitely heavy co-drifting ions that
    cancels the net electron current (j_bg = -mean_current)."""
    gam = np.sqrt(1.0 + (u * u).sum(axis=0))
    return (q * w[None, :] * u / gam[None, :]).sum(axis=1) / ncells


def laser_2d(n1, n2, dx1, dx2, a0, waist, length, k0, x1c, x2c):
    """Gaussian laser polarised along x3, moving in -x1, from the vector potential

        A3 = a0 exp(-((x1-x1c)/L)^2) exp(-((x2-x2c)/W)^2) cos(k0 (x1-x1c))

    E3 = -dA3/dt = -dA3/dx1 (a wave moving in -x1) and B = curl(A3 e3) =
    (dA3/dx2, -dA3/dx1, 0), each evaluated analytically at its Yee node.
    Returns E, B as [3][n2][n1] arrays."""

    def parts(x1, x2):
        s1 = x1 - x1c
        s2 = x2 - x2c
        g1 = np.exp(-(s1 / length) ** 2)
        g2 = np.exp(-(s2 / waist) ** 2)
        c = np.cos(k0 * s1)
        s = np.sin(k0 * s1)
        d1 = a0 * g2 * (-2.0 * s1 / length ** 2 * g1 * c - g1 * k0 * s)  # dA3/dx1
        d2 = a0 * g1 * c * (-2.0 * s2 / waist ** 2 * g2)                 # dA3/dx2
        return d1, d2

    i1 = np.arange(n1, dtype=np.float64)
    i2 = np.arange(n2, dtype=np.float64)
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    # E3 at (i1, i2)
    X1, X2 = np.meshgrid(i1 * dx1, i2 * dx2)
    d1, _ = parts(X1, X2)
    E[2] = -d1
    # B1 at (i1, i2 + 1/2)
    X1, X2 = np.meshgrid(i1 * dx1, (i2 + 0.5) * dx2)
    _, d2 = parts(X1, X2)
    B[0] = d2
    # B2 at (i1 + 1/2, i2)
    X1, X2 = np.meshgrid((i1 + 0.5) * dx1, i2 * dx2)
    d1, _ = parts(X1, X2)
    B[1] = -d1
    return E, B


def drift2d(n1, n2, dx1, dx2, dt, sub=(2, 2), gamma=50.0, sigma_u=1e-4, density=1.0,
            jitter=False, alpha=0.5, seed=SEED0, laser=None, name="drift2d"):
    """A 2D electron plasma drifting along x1 over a neutralising background.

    Returns a dict with the grid, particle arrays and initial fields."""
    gen = rng(seed)
    x1, x2 = lattice_2d(n1, n2, sub[0], sub[1], jitter, gen)
    npart = x1.size
    ppc = sub[0] * sub[1]
    u = drift_momenta(npart, gamma, sigma_u, gen)
    w = np.full(npart, density / ppc)
    q, qm = -1.0, -1.0
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    if laser is not None:
        E, B = laser_2d(n1, n2, dx1, dx2, **laser)
    jbg = -mean_current(u, w, q, n1 * n2)
    return dict(name=name, geom=2, n=(n1, n2, 1), dx=(dx1, dx2, 1.0), dt=dt, alpha=alpha,
                xi=np.stack([x1, x2]), u=u, w=w, q=q, qm=qm, E=E, B=B, jbg=jbg, seed=seed)


def drift2d_small(seed=SEED0 + 0):
    """64 x 32 cells, dx = 0.2, dt = 0.05, 2x2 quiet lattice (8192 particles),
    uniform density, gamma = 50 with thermal spread 1e-4, filter 0.5, 100 steps."""
    d = drift2d(64, 32, 0.2, 0.2, 0.05, sub=(2, 2), gamma=50.0, sigma_u=1e-4, seed=seed,
                name="drift2d_64x32_g50")
    d["steps"] = 100
    return d


def drift2d_laser(seed=SEED0 + 1, n1=2048, n2=512):
    """2048 x 512 cells, dx = (0.1, 0.2), dt = 0.045, 8 per cell as a jittered
    4x2 sub-lattice (8 388 608 particles), gamma = 20 cold, Gaussian laser
    a0 = 2, waist 8, length 4, k0 = 10, moving against the drift."""
    dx1, dx2 = 0.1, 0.2
    L1, L2 = n1 * dx1, n2 * dx2
    laser = dict(a0=2.0, waist=8.0, length=4.0, k0=10.0, x1c=0.75 * L1, x2c=0.5 * L2)
    d = drift2d(n1, n2, dx1, dx2, 0.045, sub=(4, 2), gamma=20.0, sigma_u=0.0, jitter=True,
                seed=seed, laser=laser, name="drift2d_%dx%d_g20_laser" % (n1, n2))
    d["steps"] = 1000
    return d


SCAN_N1 = (256, 512, 1024, 2048)
SCAN_N2 = (64, 128, 256, 512)


def scan2d_params(nruns=64, seed=SEED0 + 4, shrink=1):
    """Per-run parameters of the parameter scan: run r draws, from its own
    generator seeded seed + 1000 r, N1, N2, gamma, density and particles per
    cell.  ``shrink`` divides both grid sizes (small versions for tests)."""
    out = []
    for r in range(nruns):
        gen = rng(seed + 1000 * r)
        n1 = int(gen.choice(SCAN_N1)) // shrink
        n2 = int(gen.choice(SCAN_N2)) // shrink
        gamma = float(gen.uniform(5.0, 100.0))
        density = float(gen.uniform(0.5, 2.0))
        ppc = int(gen.integers(4, 17))
        out.append(dict(run=r, n1=n1, n2=n2, gamma=gamma, density=density, ppc=ppc,
                        seed=seed + 1000 * r))
    return out


def scan2d_run(p, dx=0.2, dt=0.05, sigma_u=1e-4, alpha=0.5):
    """One run of the parameter scan from its parameters (see scan2d_params)."""
    gen = rng(p["seed"] + 1)
    n1, n2, ppc = p["n1"], p["n2"], p["ppc"]
    x1, x2 = random_in_cells(n1, n2, ppc, gen)
    npart = x1.size
    u = drift_momenta(npart, p["gamma"], sigma_u, gen)
    w = np.full(npart, p["density"] / ppc)
    q, qm = -1.0, -1.0
    E = np.zeros((3, n2, n1))
    jbg = -mean_current(u, w, q, n1 * n2)
    return dict(name="scan2d_run%d_%dx%d" % (p["run"], n1, n2), geom=2, n=(n1, n2, 1),
                dx=(dx, dx, 1.0), dt=dt, alpha=alpha, xi=np.stack([x1, x2]), u=u, w=w, q=q,
                qm=qm, E=E, B=E.copy(), jbg=jbg, seed=p["seed"], steps=200)


def scan2d(nruns=64, seed=SEED0 + 4, shrink=1):
    """All runs of the parameter scan (see scan2d_params, scan2d_run)."""
    return [scan2d_run(p) for p in scan2d_params(nruns, seed, shrink)]


def drift3d(n1=512, n2=128, n3=128, dx=0.2, dt=0.05, sub=(2, 1, 1), gamma=50.0, sigma_u=0.0,
            spread=0.05, jitter=False, alpha=0.5, seed=SEED0 + 2, name=None):
    """A 3D electron plasma drifting along x1 over a neutralising background:
    a sub-lattice in every cell (offsets (k + 1/2) / sub, or uniform inside
    the sub-cell with ``jitter``), weights n_cell / ppc with n_cell drawn per
    cell from U[1 - spread, 1 + spread].  Positions ``xi`` are [3][np] in cell
    units, fields [3][n3][n2][n1]."""
    gen = rng(seed)
    ppc = sub[0] * sub[1] * sub[2]
    cells = n1 * n2 * n3
    dens = 1.0 + spread * (2.0 * gen.random(cells) - 1.0)
    offs = [(np.arange(sub[d], dtype=np.float64) + 0.5) / sub[d] for d in range(3)]
    o1, o2, o3 = np.meshgrid(offs[0], offs[1], offs[2], indexing="ij")
    o = np.stack([o1.ravel(), o2.ravel(), o3.ravel()])          # [3][ppc]
    cell = np.arange(cells, dtype=np.int64)
    i1 = cell % n1
    i2 = (cell // n1) % n2
    i3 = cell // (n1 * n2)
    base = np.stack([i1, i2, i3]).astype(np.float64)            # [3][cells]
    xi = (base[:, :, None] + o[:, None, :]).reshape(3, -1)       # cell-major
    if jitter:
        for d in range(3):
            xi[d] += (gen.random(xi.shape[1]) - 0.5) / sub[d]
    for d, n in enumerate((n1, n2, n3)):
        xi[d] = np.mod(xi[d], n)
    npart = xi.shape[1]
    u = drift_momenta(npart, gamma, sigma_u, gen)
    w = np.repeat(dens / ppc, ppc)
    q, qm = -1.0, -1.0
    E = np.zeros((3, n3, n2, n1))
    jbg = -mean_current(u, w, q, cells)
    return dict(name=name or "drift3d_%dx%dx%d_g%g" % (n1, n2, n3, gamma), geom=3,
                n=(n1, n2, n3), dx=(dx, dx, dx), dt=dt, alpha=alpha, xi=xi, u=u, w=w, q=q, qm=qm,
                E=E, B=E.copy(), jbg=jbg, seed=seed, steps=500)


def nci_table1(seed=SEED0 + 10, ppc=(2, 2), n=(256, 256)):
    """Table 1: dx = (0.2, 0.2), dt = 0.4 dx1, periodic, 51.2 x 51.2 (256 x 256
    cells), gamma = 50, n/n_p = 100."""
    d = drift2d(n[0], n[1], 0.2, 0.2, 0.08, sub=ppc, gamma=50.0, sigma_u=1e-4, density=100.0,
                seed=seed, name="nci_table1")
    return d


def lwfa_boosted(n1=8192, n2=512, gamma_b=14.0, ppc=(2, 2), sigma_u=1e-4, seed=SEED0 + 13,
                 name=None):
    """Lorentz-boosted 2D laser wakefield set-up of Table 2 (Sec. 6), in the
    boosted frame with lab-frame laser units (k0 = omega0 = 1, c = 1, density
    in units of the lab critical density):

    * grid dx1 = dx2 = 0.0982 gamma_b (1 + beta_b) (2.746 for gamma_b = 14),
      dt = 0.225 dx1, 8192 x 512 cells, filter at half the x1 Nyquist
      wavenumber;
    * plasma of density 1.148e-3 gamma_b streaming along -x1 with
      u1 = -gamma_b beta_b plus a Gaussian spread sigma_u per component (1e-4,
      as in the Table 1 runs: the seed of the numerical Cherenkov instability,
      which a cold quiet plasma would take from round-off alone), on a quiet
      ppc sub-lattice (2 x 2, 16 777 216 particles), filling the periodic box,
      with co-streaming ions as a fixed neutralising background (charge and
      uniform current);
    * the laser (a0 = 4, waist 117.81, polarised along x3, field FWHM
      70.64 gamma_b (1 + beta_b) in the boosted frame) launched by a moving
      antenna at rest in the lab frame (v = -beta_b): surface current
      K = 2 (1 + beta_b) a0 omega' sin^2(pi s/T) sin(omega s), omega' =
      1/(gamma_b (1 + beta_b)) the boosted laser frequency, omega =
      omega' (1 + beta_b) the drive frequency, T = 2 FWHM / (1 + beta_b);
    * 6400 steps (t' = 3955, the time of Fig. 4's boosted-frame snapshots).

    Returns a ``drift2d``-style dict plus ``antenna`` (keyword arguments of
    ``hpic.Sim.set_antenna``) and ``laser`` (the boosted-frame parameters)."""
    gen = rng(seed)
    beta_b = math.sqrt(1.0 - 1.0 / (gamma_b * gamma_b))
    dx = 0.0982 * gamma_b * (1.0 + beta_b)
    dt = 0.225 * dx
    density = 1.148e-3 * gamma_b
    x1, x2 = lattice_2d(n1, n2, ppc[0], ppc[1], False, gen)
    npart = x1.size
    u = np.zeros((3, npart))
    u[0] = -gamma_b * beta_b
    if sigma_u > 0:
        u += sigma_u * gen.standard_normal((3, npart))
    w = np.full(npart, density / (ppc[0] * ppc[1]))
    q, qm = -1.0, -1.0
    a0, waist = 4.0, 117.81
    fwhm = 70.64 * gamma_b * (1.0 + beta_b)
    omega_b = 1.0 / (gamma_b * (1.0 + beta_b))
    L1, L2 = n1 * dx, n2 * dx
    antenna = dict(x0=0.125 * L1, v=-beta_b, t0=0.0, T=2.0 * fwhm / (1.0 + beta_b),
                   K0=2.0 * (1.0 + beta_b) * a0 * omega_b, omega=omega_b * (1.0 + beta_b),
                   phase=0.0, x2c=0.5 * L2, waist=waist)
    E = np.zeros((3, n2, n1))
    jbg = -mean_current(u, w, q, n1 * n2)
    return dict(name=name or "lwfa_boosted_%dx%d_g%g" % (n1, n2, gamma_b), geom=2,
                n=(n1, n2, 1), dx=(dx, dx, 1.0), dt=dt, alpha=0.5, xi=np.stack([x1, x2]), u=u,
                w=w, q=q, qm=qm, E=E, B=E.copy(), jbg=jbg, seed=seed, steps=6400,
                antenna=antenna, laser=dict(gamma_b=gamma_b, beta_b=beta_b, a0=a0, waist=waist,
                                            fwhm=fwhm, omega=omega_b, density=density))


def drift_q3d(n1=4096, n2=256, dz=0.1, dr=0.2, dt=0.04, modes=3, sub=(2, 1, 4), rfill=None,
              gamma=20.0, sigma_u=0.0, density=1.0, a0=1.0, waist=8.0, length=4.0, k0=10.0,
              alpha=0.5, seed=SEED0 + 3, name=None):
    """Quasi-3D drifting plasma column with an m = 1 seed pulse (see the module
    docstring).  Particles of cell (i, j): z = (i + (a + 1/2)/sub_z) dz,
    r = (j + (b + 1/2)/sub_r) dr, theta = phase_ij + 2 pi c / sub_t; weight
    density * 2 pi r dr dz / ppc (the volume each represents)."""
    gen = rng(seed)
    if rfill is None:
        rfill = n2 - 6
    ppc = sub[0] * sub[1] * sub[2]
    iz, jr = np.meshgrid(np.arange(n1), np.arange(rfill), indexing="ij")
    iz, jr = iz.ravel(), jr.ravel()
    phase = 2.0 * math.pi * gen.random(iz.size)
    oz = (np.arange(sub[0]) + 0.5) / sub[0]
    orr = (np.arange(sub[1]) + 0.5) / sub[1]
    ot = 2.0 * math.pi * np.arange(sub[2]) / sub[2]
    a, b, c = np.meshgrid(oz, orr, ot, indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()                      # [ppc]
    z = ((iz[:, None] + a[None, :]) * dz).ravel()
    r = ((jr[:, None] + b[None, :]) * dr).ravel()
    th = (phase[:, None] + c[None, :]).ravel()
    x = np.stack([z, r * np.cos(th), r * np.sin(th)])
    npart = z.size
    u = drift_momenta(npart, gamma, sigma_u, gen)
    w = density * 2.0 * math.pi * r * dr * dz / ppc
    # m = 1 seed: E_x (Er_1 = E_x, Eth_1 = i E_x), B_y = -E_x (Br_1 = i E_x,
    # Bth_1 = -E_x), each at its staggered node
    zc = 0.75 * n1 * dz
    nr = n2 + 1
    zi, zh = np.arange(n1) * dz, (np.arange(n1) + 0.5) * dz
    ri, rh = np.arange(nr) * dr, (np.arange(nr) + 0.5) * dr

    def pulse(zz, rr):
        return a0 * np.exp(-((zz[None, :] - zc) / length) ** 2 - (rr[:, None] / waist) ** 2) * \
            np.cos(k0 * (zz[None, :] - zc))

    E = np.zeros((modes, 3, nr, n1), dtype=np.complex128)
    B = np.zeros_like(E)
    if modes > 1 and a0 != 0:
        E[1, 1] = pulse(zi, rh)
        E[1, 2] = 1j * pulse(zi, ri)
        B[1, 1] = 1j * pulse(zh, ri)
        B[1, 2] = -pulse(zh, rh)
        for F in (E, B):
            F[1, :, n2] = 0.0
    return dict(name=name or "drift_q3d_%dx%d_m%d_g%g" % (n1, n2, modes, gamma), geom=4,
                n=(n1, n2), dx=(dz, dr), dt=dt, modes=modes, alpha=alpha, x=x, u=u, w=w,
                q=-1.0, qm=-1.0, E=E, B=B, seed=seed, steps=500)
