/*
 * hpic.h -- C ABI of the MI355X hybrid Yee-FFT particle-in-cell library.
 *
 * The library advances relativistic electromagnetic PIC runs with the hybrid
 * Maxwell solver of Yu et al., arXiv:1502.01376: the field equations are
 * solved in (k1, x2) space after an FFT along the drift direction x1, with the
 * x1 derivative spectral (Eq. (20)) and the x2 derivative a Yee finite
 * difference (Eqs. (12)-(17)); the current comes from a local charge-conserving
 * deposit, is corrected by Eq. (11) so that Gauss's law (27) is kept, and is
 * low-pass filtered along k1 (Sec. 4).  Every step of the path runs in HIP
 * kernels on one gfx950 GPU.
 *
 * One step (Sec. 2.1 order): relativistic Boris push with a quadratic field
 * gather, charge-conserving (Esirkepov) deposit of j^{n+1/2}, FFT of j along
 * x1, current correction and filter, hybrid Maxwell update of E and B, inverse
 * FFT of E and B for the next push.
 *
 * Grid conventions: n1 x n2 cells, periodic; field arrays are [i2][i1] with x1
 * fastest; Yee staggering of Eqs. (1)-(6): E1 (i1+1/2, i2), E2 (i1, i2+1/2),
 * E3 (i1, i2), B1 (i1, i2+1/2), B2 (i1+1/2, i2), B3 (i1+1/2, i2+1/2), j like E,
 * rho on (i1, i2); a half-integer position i+1/2 is stored at index i.
 * 3D (HP_GEOM_3D, Sec. 2.2: the x3 differences added to the hybrid update):
 * n1 x n2 x n3 cells, arrays [i3][i2][i1], E1 (i1+1/2, i2, i3), E2 (i1, i2+1/2,
 * i3), E3 (i1, i2, i3+1/2), B1 (i1, i2+1/2, i3+1/2), B2 (i1+1/2, i2, i3+1/2),
 * B3 (i1+1/2, i2+1/2, i3); the transforms run along x1 over the n2 n3 rows.
 * Below, "[dim]" is 2 or 3 and "cells" n1 n2 (2D) or n1 n2 n3 (3D).
 * Quasi-3D (HP_GEOM_Q3D, Sec. 5: the hybrid update per azimuthal mode):
 * z = x1 (n[0] points, dx[0], FFT), r = x2 (n[1] cells of dx[1], axis at
 * r = 0, conducting wall at r = n[1] dx[1]), modes m = 0..n_modes-1 of
 * F = sum_m Re(F_m e^{i m theta}); per mode complex fields [3][n2+1][n1]
 * (Ez, Er, Eth and Bz, Br, Bth on the r-z Yee nodes) passed as interleaved
 * (re, im) doubles.  Particles carry Cartesian positions (z, x, y) and momenta
 * (uz, ux, uy); their phase in mode m is e^{-i m th}, their current is
 * deposited per mode by a charge-conserving scheme (Esirkepov in r-z with
 * the mean phase plus an azimuthal flux from the phase change) and must stay
 * at r < (n2 - 3) dr (no particle boundary at the wall).  Not available for
 * this geometry: the tile calls, raw and fixed-point access, the device-buffer
 * transfers.
 * Units: c = 1, t in 1/w_p, x in c/w_p, E and B in m c w_p / e, density in
 * n_p, current in e n_p c (the 4 pi of the paper's Gaussian form is 1).
 *
 * Errors: every call returns 0 (HP_OK) or a negative HP_E* code; the message
 * of the last failing call on the calling thread is hp_last_error().  A handle
 * must not be used from two threads at once.  No exception crosses the ABI.
 */
#ifndef HPIC_H
#define HPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HP_OK 0
#define HP_EINVAL (-1)   /* bad argument, size or enum */
#define HP_ECOURANT (-2) /* dt above the stability limit of Eq. (22) */
#define HP_ENOMEM (-3)   /* device allocation failed */
#define HP_EDEVICE (-4)  /* HIP runtime error or no device */
#define HP_ERANGE (-5)   /* particle moved a cell or more, or fixed-point headroom exceeded */
#define HP_ENUMERIC (-6) /* non-finite particle momentum or position */
#define HP_ESTATE (-7)   /* call out of order (e.g. step before particles) */

#define HP_GEOM_2D 2
#define HP_GEOM_3D 3
#define HP_GEOM_Q3D 4  /* quasi-3D r-z with azimuthal modes */

#define HP_PREC_FP32_FIXED 0 /* FP32 push/FFT/update, 64-bit fixed-point deposit */
#define HP_PREC_FP64 1       /* FP64 everywhere, FP64 atomics in the deposit */

/* Kernel indices of hp_get_kernel_times. */
#define HP_K_PUSH_DEPOSIT 0
#define HP_K_FFT_J 1
#define HP_K_KUPDATE 2
#define HP_K_IFFT_EB 3
#define HP_K_SORT 4
#define HP_NK 5

/* Per-run configuration.  n[0] (x1, the FFT direction) must be a power of two
 * in [8, 4096]; n[1] >= 4.  dt must satisfy the hybrid Courant condition
 * dt <= 2 / sqrt(pi^2/dx1^2 + 4/dx2^2) of Eq. (22) (for deriv1 = 1 the Yee
 * limit 1/sqrt(1/dx1^2 + 1/dx2^2)), otherwise HP_ECOURANT. */
typedef struct hp_config {
  int32_t geom;              /* HP_GEOM_2D or HP_GEOM_3D (same for all runs of a handle) */
  int32_t n[3];              /* cells per direction (n[2] unused in 2D); n[0] a
                                power of two, 8 .. 8192 for Cartesian runs,
                                8 .. 4096 for quasi-3D runs (LDS of the row
                                transforms) */
  double dx[3];              /* cell sizes */
  double dt;                 /* time step */
  int32_t shape_order;       /* particle shape order: 2 (quadratic) or 3 (cubic
                                B-spline, Sec. 4 and Appendix A; 2D only).  The
                                FP32 form keeps continuity exact in integers for
                                both (integer weights with exact sum 2^P) */
  int32_t interp;            /* 0: momentum-conserving gather (Appendix A, first
                                variant: the quadratic spline at every component's
                                node); 1: energy-conserving (second variant: linear
                                weights along the component's staggered directions,
                                so that J.E of the Esirkepov current is the work on
                                the particle) */
  double filter_frac;        /* low-pass cutoff alpha: keep |k1| <= alpha pi/dx1
                                (Sec. 4); >= 1 disables */
  int32_t deriv1;            /* 0: spectral k1 (Eq. (20)); 1: FD [k]1 (Eq. (28)) */
  int32_t correct;           /* 1: current correction of Eq. (11); 0 only for tests */
  int32_t n_modes;           /* azimuthal modes (quasi-3D; unused in 2D) */
  int32_t precision;         /* HP_PREC_FP32_FIXED or HP_PREC_FP64; same for all runs */
  int32_t fixed_shape_bits;  /* P: shape factors quantised to 2^-P; 0 = automatic:
                                22 if all particle charges are equal, else 20 */
  int32_t fixed_weight_bits; /* Q: charges quantised to 2^-Q of the largest;
                                0 = automatic (exact for equal weights, else the
                                largest Q <= 15 the headroom allows) */
  int32_t sort_interval;     /* particle tile sort every K steps; 0 = automatic */
  int32_t kmod;              /* 1: modified spectral symbol of Eq. (29) (Sec. 4),
                                [k]1 = k1 + dk_max cos^2((k1 - k1m)/(k1l - k1m) pi/2)
                                on k1l <= k1 <= k1u with k1l = 0.15 kg1, k1u = 0.26 kg1,
                                dk_max = 0.01 kg1, kg1 = 2 pi/dx1; the j1 correction
                                becomes [k]1,FD/[k]1,mod.  0: off */
  int32_t reserved[7];
} hp_config;

/* FP64 diagnostics of one run (Sec. 2.3 and energies), see hp_diagnostics. */
typedef struct hp_diag {
  double W_E[3];        /* field energy 1/2 sum E_c^2 dV per component */
  double W_B[3];        /* 1/2 sum B_c^2 dV */
  double kinetic;       /* sum_p m w_p (gamma_p - 1) dV */
  double gauss_l2;      /* || D.E - f (rho + rho_bg) ||_2 over (kappa1, i2), Eq. (27) */
  double gauss_linf;    /* max-norm of the same residual */
  double gauss_ref_l2;  /* || f (rho + rho_bg) ||_2 (scale for the residual) */
  double cont_linf;     /* max-norm of the continuity residual (23) of the last step, or -1 */
  int64_t cont_int;     /* FP32_FIXED: max |2 (rho_new - rho_old) - div J| in integers, or -1 */
  double charge_total;  /* sum of rho dV */
  int64_t step;         /* steps taken */
} hp_diag;

typedef struct hp_sim hp_sim;

/* Creates a handle with nruns independent runs (one batched launch per stage
 * advances all of them).  cfgs[nruns] is read before return.  The library owns
 * *out and all device memory; release with hp_destroy.  Errors: HP_EINVAL,
 * HP_ECOURANT, HP_ENOMEM, HP_EDEVICE. */
int hp_create(const hp_config *cfgs, int32_t nruns, hp_sim **out);
void hp_destroy(hp_sim *sim);
const char *hp_last_error(void);

/* All later device work of the handle is enqueued on this HIP stream (NULL:
 * the null stream).  The stream stays owned by the caller. */
int hp_set_stream(hp_sim *sim, void *hip_stream);

/* Loads n particles of one species into a run (replacing any previous ones).
 * x is [dim][n] in physical units (wrapped into the box), u = gamma v is [3][n],
 * w[n] the density weight (charge density = q sum w S).  Host buffers are
 * caller-owned and copied before return.  Sets the fixed-point charge unit of
 * the run.  Quasi-3D: x is [3][n] Cartesian (z, x, y), u = (uz, ux, uy), w the
 * number of physical particles (charge q w; weights grow with r for a uniform
 * density), every r = hypot(x, y) below (n2 - 3) dr.  Errors: HP_EINVAL
 * (species != 0, n out of range, non-finite input, quasi-3D r too large),
 * HP_ERANGE (fixed-point headroom). */
int hp_set_particles(hp_sim *sim, int32_t run, int32_t species, int64_t n, const double *x,
                     const double *u, const double *w, double q_over_m, double q);

/* As hp_set_particles (the scheme's particle input of Sec. 2: positions,
 * momenta, weights), Cartesian runs only, with x[dim][n], u[3][n], w[n] FP64
 * arrays in device memory (for example torch tensors on the handle's device).
 * The conversion to cell index + offset runs on the device with the same
 * operations as the host loader, so the run holds the same bits either way.
 * A first device pass validates the input and measures the charges and the
 * particles per cell; on an error nothing of the run changes.  The buffers stay
 * caller-owned and are read on the handle's stream before return (the call
 * synchronises).  Errors: HP_EINVAL (a pointer that is not device memory, a
 * quasi-3D handle, or as hp_set_particles), HP_ERANGE (fixed-point headroom). */
int hp_set_particles_device(hp_sim *sim, int32_t run, int32_t species, int64_t n,
                            const double *x, const double *u, const double *w, double q_over_m,
                            double q);

/* Sets E^0 and B^0 of a run from host arrays E[3][cells], B[3][cells] at
 * their Yee nodes (mode must be 0).  Quasi-3D: mode m, complex interleaved
 * E[3][n2+1][n1][2], B likewise. */
int hp_set_fields(hp_sim *sim, int32_t run, int32_t mode, const double *E, const double *B);

/* Background of a run: with rho_from_particles = 1 the fixed charge density
 * rho_bg = -rho_e(now) is recorded (used only by the Gauss diagnostic); j_bg[3]
 * is a uniform current added to the deposited one every step (NULL: zero).
 * Quasi-3D: rho_bg per mode; rho_from_particles = 2 also records the
 * co-drifting current of mode 0 along z, minus the z-average of the
 * particles' current u_z/gamma at this moment (a z-independent profile per
 * row, added every step); j_bg must be NULL or zero. */
int hp_set_background(hp_sim *sim, int32_t run, int32_t rho_from_particles,
                      const double *j_bg);

/* Moving antenna of a 2D run (Sec. 6 launches the laser of its boosted-frame
 * runs with a moving antenna and gives no form; this is the form used here):
 * a sheet of out-of-plane surface current K(t) g(x2) at x1 = x0 + v t
 * (periodic), K(t) = K0 sin^2(pi s / T) sin(omega s + phase) for
 * 0 <= s = t - t0 <= T and 0 otherwise, g(x2) = exp(-((x2 - x2c)/waist)^2)
 * with the periodic distance (waist <= 0: g = 1).  Each step adds
 * j3(i, j) += K(t) g(j dx2) S2(x_a/dx1 - i) / dx1 (S2 the quadratic B-spline)
 * at the step's time centre t = (n + 1/2) dt, where n counts the handle's
 * steps.  Such a sheet radiates E3 = -K(t_ret) / (2 (1 -+ v)) towards +-x1 at
 * the Doppler-shifted frequency omega / (1 -+ v); j3 carries no charge in 2D.
 * Lengths, times and velocities in the units of hp_config. */
typedef struct hp_antenna {
  double x0;       /* position along x1 at t = 0 */
  double v;        /* velocity along x1, |v| < 1 */
  double t0, T;    /* on for t0 <= t <= t0 + T, T > 0 */
  double K0;       /* surface-current amplitude */
  double omega;    /* angular frequency of the drive */
  double phase;    /* phase of the drive at t = t0 */
  double x2c;      /* centre of the transverse profile */
  double waist;    /* 1/e half width of the field profile (<= 0: uniform) */
} hp_antenna;

/* Sets (a != NULL) or removes (a == NULL) the antenna of a 2D run; one per
 * run, copied.  HP_EINVAL for a 3D or quasi-3D run or a parameter out of
 * range (non-finite, |v| >= 1, T <= 0).  The time of the handle's step counter
 * is used, so an antenna set after some steps sees the time those steps
 * reached; checkpoints keep the counter, not the antenna. */
int hp_set_antenna(hp_sim *sim, int32_t run, const hp_antenna *a);

/* Advances every run nsteps steps, asynchronously on the handle's stream.
 * Kernel-detected errors (HP_ERANGE, HP_ENUMERIC) are reported by the next
 * synchronous call. */
int hp_step(hp_sim *sim, int32_t nsteps);

/* Particle tiling of a handle (all runs): the tile shape of the sort and of
 * the push+deposit workgroups, the sort interval, and the LDS budget of one
 * push workgroup derived from the tile shape. */
typedef struct hp_tune {
  int32_t tile[2];        /* cells per tile along x1, x2 (clipped to each grid) */
  int32_t sort_interval;  /* steps between particle sorts */
  int32_t lds_bytes;      /* LDS of one push+deposit workgroup */
  double ms_per_step;     /* hp_autotune: measured time per step of the choice */
  int32_t candidates;     /* hp_autotune: settings timed */
  int32_t steps;          /* hp_autotune: steps advanced */
} hp_tune;

/* Sets the tile shape (1..4096 cells per direction; 3D tiles are
 * tile1 x tile2 x tile2) and sort interval
 * (1..1024 steps) and re-sorts the particles.  Results of the FP32_FIXED form
 * are bit-identical for every setting.  HP_EINVAL out of range.
 * Quasi-3D handles: the bins of the periodic particle sort, tile1 z columns x
 * tile2 radial rows (default 4 x 2), and its interval (default 64 steps; a
 * load sorts before the first step); the push works on waves of 64
 * consecutive particles, so the bins set how compact a wave is.  The sort
 * only permutes storage: FP32_FIXED results are bit-identical for every
 * setting (FP64: equal to rounding, the deposit's atomics add in another
 * order).  lds_bytes reads 0 for these handles. */
int hp_set_tiling(hp_sim *sim, int32_t tile1, int32_t tile2, int32_t sort_interval);
int hp_get_tiling(hp_sim *sim, hp_tune *out);

/* Autotuner: advances every run by exactly nsteps steps (as hp_step) while
 * timing candidate tile shapes and then sort intervals on the live runs, each
 * over two sort blocks, and keeps the fastest (also for later hp_step calls).
 * With too few steps the remaining candidates are skipped.  Synchronous.
 * out may be NULL. */
int hp_autotune(hp_sim *sim, int32_t nsteps, hp_tune *out);

/* With enable = 1 (the default) hp_step replays each block of one particle
 * sort and sort_interval steps as a captured HIP graph (when sort_interval is
 * even and no profiling is active); 0 launches every kernel separately.
 * Results are identical either way. */
int hp_use_graphs(hp_sim *sim, int32_t enable);

/* Waits for the handle's stream and reports kernel-detected errors. */
int hp_synchronize(hp_sim *sim);

/* Copies field component comp (0..2 = E1..E3, 3..5 = B1..B3) of a run into
 * out[count], count = cells (else HP_EINVAL).  Synchronous.  Quasi-3D: mode
 * m, complex interleaved, count = 2 (n2+1) n1. */
int hp_get_field(hp_sim *sim, int32_t run, int32_t comp, int32_t mode, double *out,
                 size_t count);

/* Current j^{n-1/2} of the last step, component comp (0..2), in physical
 * units on the j nodes: corrected = 0 as deposited (plus background);
 * corrected = 1 after Eq. (11) and the filter (transformed back to x1). */
int hp_get_current(hp_sim *sim, int32_t run, int32_t comp, int32_t corrected, double *out,
                   size_t count);

/* Quasi-3D (Sec. 5, the per-mode hybrid solve): the current density deposited
 * in the last step for azimuthal mode `mode` and component comp (0 jz, 1 jr,
 * 2 jth) on the r-z Yee nodes, before the correction of Eq. (11) and the
 * filter, without the background: complex interleaved [n2+1][n1][2], count =
 * 2 (n2+1) n1 doubles.  out is caller-owned; synchronous.  HP_EINVAL for a
 * Cartesian handle or a bad comp, mode or count. */
int hp_get_current_mode(hp_sim *sim, int32_t run, int32_t comp, int32_t mode, double *out,
                        size_t count);

/* FP32_FIXED only: the raw 64-bit accumulator of the last step's deposit. */
int hp_get_current_fixed(hp_sim *sim, int32_t run, int32_t comp, int64_t *out, size_t count);

/* Number of particles of a run. */
int hp_get_particle_count(hp_sim *sim, int32_t run, int64_t *n);

/* Particles of a run in the library's current order: x[dim][n] physical
 * positions, u[3][n], w[n], id[n] (index given at hp_set_particles).  Any
 * pointer may be NULL.  n must equal the particle count. */
int hp_get_particles(hp_sim *sim, int32_t run, int64_t n, double *x, double *u, double *w,
                     int64_t *id);

/* FP32_FIXED only: raw state, cell[dim][n] (i1, i2, i3), off[dim][n] in [0,1),
 * u[3][n], qw[n] (charge times weight), id[n].  Any pointer may be NULL. */
int hp_get_particles_raw(hp_sim *sim, int32_t run, int64_t n, int32_t *cell, float *off,
                         float *u, float *qw, int32_t *id);

/* Device-buffer reads (Cartesian runs), enqueued on the handle's stream and
 * asynchronous: the outputs are valid once that stream's work up to here has
 * completed (hp_synchronize or the caller's own stream synchronisation).
 * Outputs are caller-owned device memory of the form's real type, float for
 * HP_PREC_FP32_FIXED and double for HP_PREC_FP64 (written "real" below).
 *
 * hp_get_field_device: the real-space field component comp (0..2 = E1..E3,
 * 3..5 = B1..B3) that the next gather reads, at its Yee nodes (Eqs. (1)-(6)),
 * into out[count] real, count = cells, layout [n3][n2][n1].
 *
 * hp_get_particles_device: the particle state in the library's current order:
 * cell[dim][n] (int32 i1, i2, i3), off[dim][n] real offsets in [0,1),
 * u[3][n] real, qw[n] real (charge times weight), id[n] (int32 index given at
 * loading).  Any pointer may be NULL; n must equal the particle count.
 *
 * hp_get_current_device: the current j^{n-1/2} of the last step, component comp
 * (0..2), as hp_get_current returns it (corrected = 0: as deposited, plus the
 * background, in physical units on the j nodes; 1: after the correction of
 * Eq. (11) and the filter, transformed back to x1), into out[count] double,
 * count = cells, layout [n3][n2][n1].  The same values as the host read, bit
 * for bit.
 *
 * Errors: HP_EINVAL (a pointer that is not device memory, bad comp or count,
 * a quasi-3D handle). */
int hp_get_field_device(hp_sim *sim, int32_t run, int32_t comp, void *out, size_t count);
int hp_get_current_device(hp_sim *sim, int32_t run, int32_t comp, int32_t corrected, double *out,
                          size_t count);
int hp_get_particles_device(hp_sim *sim, int32_t run, int64_t n, int32_t *cell, void *off,
                            void *u, void *qw, int32_t *id);

/* FP64 diagnostics of a run (energies, Gauss residual, continuity residual of
 * the last step when the previous hp_diagnostics call was one step earlier). */
int hp_diagnostics(hp_sim *sim, int32_t run, hp_diag *out);

/* Checkpoint of every run of the handle (particles, real-space fields, the
 * FP64 k-space master, the last deposit, the background): with blob == NULL
 * writes the needed size to *size; otherwise fills blob (size bytes,
 * caller-owned; synchronous).  hp_set_state restores a handle created with the
 * same configs (Cartesian or quasi-3D); resuming is bit-exact.  Errors:
 * HP_EINVAL (buffer too small, a blob of another geometry, precision or run
 * count, a truncated blob). */
int hp_get_state(hp_sim *sim, void *blob, size_t *size);
int hp_set_state(hp_sim *sim, const void *blob, size_t size);

/* FP32_FIXED only: the deposit kernel alone on host-given particles of a run's
 * grid (n moves from cell0/off0 to cell1/off1, cells as [2][n]), returning the
 * 64-bit accumulators j_out[3][n2][n1].  For bit-exact tests. */
int hp_debug_deposit(hp_sim *sim, int32_t run, int64_t n, const int32_t *cell0,
                     const float *off0, const int32_t *cell1, const float *off1,
                     const float *v3, const float *qw, int64_t *j_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the deposit
 * of hp_debug_deposit with the same arguments, results and errors, staged in
 * a region that the library holds on each GPU from load to process end
 * instead of fresh allocations; it calls no hipMalloc or hipFree.  Limits:
 * n <= 262144 moves and a grid of at most 262144 cells (else HP_EINVAL); the
 * region is 16 MiB per GPU.  Every call on a GPU shares that GPU's region
 * (the last call's contents stay in it; the accumulators are cleared before
 * each deposit), so calls that overlap on one GPU, from two threads or two
 * streams, race. */
int hp_debug_deposit_noalloc(hp_sim *sim, int32_t run, int64_t n, const int32_t *cell0,
                             const float *off0, const int32_t *cell1, const float *off1,
                             const float *v3, const float *qw, int64_t *j_out);

/* FP32_FIXED only: out[0] = P, out[1] = inv_wunit, out[2] = c3, out[3] = Q of a
 * run (the fixed-point parameters of the deposit).  3D: out[0] = 0, out[2] = cj,
 * the integer scale of the per-node contributions (j_d = -(dx_d/dt) J_d /
 * (6 inv_wunit cj)). */
int hp_get_fixed_params(hp_sim *sim, int32_t run, double *out);

/* Per-kernel timing with HIP events on the handle's stream: enable = 1 starts
 * recording (and clears the totals), 0 stops.  hp_get_kernel_times returns the
 * summed milliseconds ms[HP_NK] and launch counts n[HP_NK] (synchronous). */
int hp_profile(hp_sim *sim, int32_t enable);
int hp_get_kernel_times(hp_sim *sim, double *ms, int64_t *n);

/* Push+deposit statistics since the last hp_profile call: out[0] = particle
 * tiles whose bounding box did not fit the workgroup's LDS (gathered and
 * deposited through global memory instead), out[1] = tiles processed.
 * Synchronous. */
int hp_get_push_stats(hp_sim *sim, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif
