/*
 * hpic_oracle.h -- declarations of the plain FP64 CPU oracle for the hybrid
 * Yee-FFT particle-in-cell step of Yu et al., arXiv:1502.01376.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle is what the GPU library is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Conventions (all routines):
 *  - 2D grid of n1 x n2 cells, periodic in x1 and x2 (Table 1: periodic).
 *  - Arrays of a field component are row-major [i2][i1], x1 fastest.
 *  - Yee staggering (Eqs. (1)-(6)): E1 at (i1+1/2, i2), E2 at (i1, i2+1/2),
 *    E3 at (i1, i2); B1 at (i1, i2+1/2), B2 at (i1+1/2, i2), B3 at
 *    (i1+1/2, i2+1/2); j is staggered like E and rho sits on (i1, i2).
 *    A half-integer position i+1/2 is stored at index i.
 *  - Particle positions are given in cell units (xi = x / dx), so a node i
 *    sits at xi = i.
 *  - Units: c = 1, t in 1/w_p, x in c/w_p, E and B in m c w_p / e, charge
 *    density in e n_p and current in e n_p c.  The 4*pi and c of the paper's
 *    Gaussian equations are 1 in these units.
 */
#ifndef HPIC_ORACLE_H
#define HPIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2D grid and solver options.  alpha is the low-pass cutoff as a fraction of
 * the x1 Nyquist wavenumber (Sec. 4; alpha >= 1 disables the filter).
 * deriv1 = 0 uses the spectral derivative k1 along x1 (Eq. (20)); deriv1 = 1
 * uses the finite-difference symbol [k]1 of Eq. (28), which turns the hybrid
 * update back into the Yee scheme (end of Sec. 2.1).  correct = 1 applies the
 * current correction of Eq. (11); 0 is an ablation used by tests.  jbg is a
 * uniform background current added to the deposited current.  kmod = 1 uses
 * the modified spectral symbol of Eq. (29), [k]1 = k1 + dk_mod(k1) with
 * dk_mod = dk_max cos^2((k1 - k1m)/(k1l - k1m) pi/2) for k1l <= k1 <= k1u,
 * k1l = 0.15 kg1, k1u = 0.26 kg1, dk_max = 0.01 kg1, kg1 = 2 pi / dx1 (the
 * values Sec. 4 gives for the Table 1 set-up); the current correction is then
 * [k]1,FD / [k]1,mod so that the Gauss law still holds. */
typedef struct or_grid2 {
  int32_t n1, n2;
  double dx1, dx2, dt;
  double alpha;
  int32_t deriv1;
  int32_t correct;
  double jbg[3];
  int32_t kmod;  /* 1: [k]1 = k1 + dk_mod(k1) of Eq. (29), Table 1 coefficients */
  int32_t interp; /* 0: momentum-conserving gather; 1: energy-conserving (linear
                     weights along each staggered direction, Appendix A) */
  int32_t shape;  /* particle shape order: 2 quadratic (0 reads as 2), 3 cubic */
} or_grid2;

/* Complex FFT of length n (power of two), in place.  sign = -1 computes
 * X_k = sum_j x_j exp(-2 pi i j k / n); sign = +1 the same sum with +i and no
 * 1/n factor.  Returns 0, or -1 if n is not a power of two. */
int or_fft(int32_t n, double *re, double *im, int32_t sign);

/* Forward transform of nrows real rows of length n1 along x1: F[row][kappa]
 * for kappa = 0..n1/2 (the Nyquist bin is kept).  Inverse: rebuilds the full
 * spectrum by Hermitian symmetry and returns the real rows including 1/n1. */
/* Threads of the oracle's OpenMP loops (particles, rows, row bands of the
 * deposit): results are the same bits for any count. */
void or_set_threads(int32_t n);
int32_t or_get_threads(void);

int or_rfft_rows(int32_t n1, int32_t nrows, const double *f, double *Fre, double *Fim);
int or_irfft_rows(int32_t n1, int32_t nrows, const double *Fre, const double *Fim, double *f);

/* Momentum-conserving quadratic gather of E and B (each [3][n2][n1]) at np
 * particles (xi1, xi2 in cell units).  Ep, Bp are [3][np]. */
void or_gather2(const or_grid2 *g, const double *E, const double *B, int64_t np,
                const double *xi1, const double *xi2, double *Ep, double *Bp);

/* Relativistic Boris rotation of the momenta u = gamma v, in place. */
void or_boris(int64_t np, double qm, double dt, const double *Ep, const double *Bp,
              double *u1, double *u2, double *u3);

/* Esirkepov charge-conserving deposit (quadratic shape) of particles moving
 * from (xa1, xa2) to (xb1, xb2) (cell units, xb not wrapped) over one step,
 * added into J [3][n2][n1].  v3 is the out-of-plane velocity and qw the
 * charge times weight of each particle.  Returns 0, or -1 if a particle moved
 * one cell or more along a coordinate. */
int or_deposit2(const or_grid2 *g, int64_t np, const double *xa1, const double *xa2,
                const double *xb1, const double *xb2, const double *v3, const double *qw,
                double *J);

/* Charge density on the integer nodes, quadratic shape, added into rho. */
void or_rho2(const or_grid2 *g, int64_t np, const double *xi1, const double *xi2,
             const double *qw, double *rho);

/* One field update E^n, B^n -> E^{n+1}, B^{n+1} with the current j^{n+1/2}
 * (J [3][n2][n1], the background g->jbg is added here).  Hybrid solver:
 * FFT along x1, current correction and filter, Eqs. (12)-(17) with B split
 * into two half steps, inverse FFT. */
int or_field_update2(const or_grid2 *g, double *E, double *B, const double *J);

/* The same update done directly in real space with the Yee differences of
 * Eqs. (1)-(6) (no FFT, no filter, no correction; jbg is added). */
void or_yee_update2(const or_grid2 *g, double *E, double *B, const double *J);

/* Moving antenna (Sec. 6 launches the laser of the boosted-frame runs with a
 * moving antenna; the text gives no form, this is the reading used here): a
 * sheet of out-of-plane surface current K(t) g(x2) at x1 = x_a(t) = x0 + v t
 * (periodic in x1), K(t) = K0 sin^2(pi s / T) sin(omega s + phase) for
 * 0 <= s = t - t0 <= T and 0 otherwise, g(x2) = exp(-((x2 - x2c)/waist)^2)
 * with the periodic distance (waist <= 0: g = 1).  A sheet with K(t) emits
 * E3 = -K(t_ret) / (2 (1 -+ v)) towards +-x1, at the Doppler-shifted
 * frequency omega / (1 -+ v); j3 has no divergence in 2D, so it carries no
 * charge. */
typedef struct or_antenna {
  double x0, v, t0, T, K0, omega, phase, x2c, waist;
} or_antenna;

/* Adds the antenna's current at time t to J3 (J is [3][n2][n1]): the sheet
 * is spread over the x1 nodes with the quadratic B-spline of its position,
 * j3(i, j) += K(t) g(j dx2) S2(x_a/dx1 - i) / dx1 (integer nodes in x2, where
 * j3 lives). */
void or_antenna2(const or_grid2 *g, const or_antenna *a, double t, double *J);

/* One whole step: gather, Boris push, move, deposit, field update.  Positions
 * are wrapped back into [0, n) at the end.  J receives the deposited current
 * (without background).  ant (or NULL): an antenna whose current at the time
 * centre t + dt/2 of the step is added before the field update (t: time at
 * the start of the step).  Returns 0, or -1 on a move of a cell or more. */
int or_step2(const or_grid2 *g, double qm, int64_t np, double *xi1, double *xi2,
             double *u1, double *u2, double *u3, const double *qw, double *E, double *B,
             double *J, const or_antenna *ant, double t);

/* Gauss-law residual of Eq. (27) in (kappa1, i2) space: R = D.E - f rho, with
 * the same x1 derivative as the update and f the current filter.  rho is the
 * total charge density on the nodes.  R is [n2][n1/2+1]. */
int or_gauss2(const or_grid2 *g, const double *E, const double *rho, double *Rre, double *Rim);

/* ---- Fixed-point deposit, in the precision of the GPU kernel ----
 * Where floating point decides an integer, the oracle takes that decision in
 * the kernel's precision (FP32), so that both sides land on the same integers.
 * Positions are a cell index plus an FP32 offset in [0,1).  Shape factors are
 * quantised to integers with exact sum 2^P; the integer Esirkepov weights then
 * satisfy the discrete continuity equation exactly (see the .c file). */
int or_deposit2_fixed(int32_t n1, int32_t n2, int32_t P, float inv_wunit, float c3,
                      int64_t np, const int32_t *ca1, const int32_t *ca2, const float *fa1,
                      const float *fa2, const int32_t *cb1, const int32_t *cb2,
                      const float *fb1, const float *fb2, const float *v3, const float *qw,
                      int64_t *J);
void or_rho2_fixed(int32_t n1, int32_t n2, int32_t P, float inv_wunit, int64_t np,
                   const int32_t *c1, const int32_t *c2, const float *f1, const float *f2,
                   const float *qw, int64_t *rho);

/* ---- 3D Cartesian ----
 * n1 x n2 x n3 cells, periodic; arrays [comp][i3][i2][i1], x1 fastest; Yee
 * staggering E1 (i1+1/2, i2, i3), E2 (i1, i2+1/2, i3), E3 (i1, i2, i3+1/2),
 * B1 (i1, i2+1/2, i3+1/2), B2 (i1+1/2, i2, i3+1/2), B3 (i1+1/2, i2+1/2, i3).
 * The hybrid solver transforms along x1 and differences along x2 and x3
 * (Sec. 2.2).  Same options as or_grid2. */
typedef struct or_grid3 {
  int32_t n1, n2, n3;
  double dx1, dx2, dx3, dt;
  double alpha;
  int32_t deriv1;
  int32_t correct;
  double jbg[3];
  int32_t kmod;
  int32_t interp; /* as in or_grid2 */
} or_grid3;

void or_gather3(const or_grid3 *g, const double *E, const double *B, int64_t np,
                const double *xi1, const double *xi2, const double *xi3, double *Ep, double *Bp);
int or_deposit3(const or_grid3 *g, int64_t np, const double *xa1, const double *xa2,
                const double *xa3, const double *xb1, const double *xb2, const double *xb3,
                const double *qw, double *J);
void or_rho3(const or_grid3 *g, int64_t np, const double *xi1, const double *xi2,
             const double *xi3, const double *qw, double *rho);
int or_field_update3(const or_grid3 *g, double *E, double *B, const double *J);
void or_yee_update3(const or_grid3 *g, double *E, double *B, const double *J);
int or_step3(const or_grid3 *g, double qm, int64_t np, double *xi1, double *xi2, double *xi3,
             double *u1, double *u2, double *u3, const double *qw, double *E, double *B,
             double *J);
int or_gauss3(const or_grid3 *g, const double *E, const double *rho, double *Rre, double *Rim);
/* Kernel-precision 3D deposit (FP32 Esirkepov weights, each node's
 * contribution rounded once to an integer; see the .c file).  ca, cb are cell
 * indices [3][np], fa, fb FP32 offsets [3][np]; J is int64 [3][cells]. */
int or_deposit3_fixed(int32_t n1, int32_t n2, int32_t n3, float inv_wunit, float cj, int64_t np,
                      const int32_t *ca, const float *fa, const int32_t *cb, const float *fb,
                      const float *qw, int64_t *J);

/* ---- Quasi-3D (r-z, azimuthal modes m = 0..nmodes-1): field solver ----
 * z = x1 (FFT, periodic, n1 points, dz), r = x2 (n2 cells of dr, axis at r = 0,
 * conducting wall at r = n2 dr).  Per mode complex arrays [3][n2+1][n1]
 * (components Ez, Er, Eth, or Bz, Br, Bth; see the .c file for the staggering
 * and the axis rules); E, B, J pass all modes back to back as interleaved
 * (re, im) doubles: [nmodes][3][n2+1][n1][2]. */
typedef struct or_gridq {
  int32_t n1, n2, nmodes;
  double dz, dr, dt;
  double alpha;
  int32_t deriv1;
  int32_t correct;
  int32_t kmod;
  int32_t interp; /* as in or_grid2 */
} or_gridq;

int or_field_update_q(const or_gridq *g, double *E, double *B, const double *J);
int or_yee_update_q(const or_gridq *g, double *E, double *B, const double *J);
int or_gauss_q(const or_gridq *g, const double *E, const double *rho, double *R);

/* ---- Quasi-3D particles (see the .c file for the mode convention, the
 * axis mirror rule and the per-mode charge-conserving deposit).  Positions
 * z, x, y and momenta uz, ux, uy are Cartesian (physical units); fields and
 * currents are [nmodes][3][n2+1][n1] complex, rho [nmodes][n2+1][n1] complex;
 * Ep, Bp are Cartesian [3][np] in the order (z, x, y).  Every function
 * returns -1 if a particle is at r >= (n2 - 3) dr (or, for the deposit, moved
 * a cell or more), 0 otherwise. */
int or_gather_q(const or_gridq *g, const double *E, const double *B, int64_t np,
                const double *z, const double *x, const double *y, double *Ep, double *Bp);
int or_deposit_q(const or_gridq *g, int64_t np, const double *za, const double *xa,
                 const double *ya, const double *zb, const double *xb, const double *yb,
                 const double *qw, double *J);
int or_rho_q(const or_gridq *g, int64_t np, const double *z, const double *x, const double *y,
             const double *qw, double *rho);
int or_jbg_q(const or_gridq *g, int64_t np, const double *x, const double *y, const double *uz,
             const double *ux, const double *uy, const double *qw, double *jbg);
int or_step_q(const or_gridq *g, double qm, int64_t np, double *z, double *x, double *y,
              double *uz, double *ux, double *uy, const double *qw, double *E, double *B,
              double *J, const double *jbg);

#ifdef __cplusplus
}
#endif
#endif
