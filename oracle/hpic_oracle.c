/*
 * hpic_oracle.c -- plain FP64 CPU oracle for the hybrid Yee-FFT
 * particle-in-cell step of Yu et al., "Mitigation of numerical Cerenkov
 * radiation and instability using a hybrid finite difference-FFT Maxwell
 * solver and a local charge conserving current deposit", arXiv:1502.01376.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the reference the GPU library is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it; the product path never does.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Everything here is written to be checked by eye against the paper, not to
 * be fast: straight loops in FP64, explicit periodic wrapping, twiddles from
 * libm at every butterfly, and the field solver in the literal form of
 * Sec. 2.1 (E, B and j are transformed along x1 at every step, advanced in
 * (k1, x2) space and transformed back).
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *  - Fourier convention f_kappa = sum_i f_i exp(-i k1 x_i) over the storage
 *    index, k1 = 2 pi kappa / (n1 dx1).  With it the forward difference of an
 *    integer-node quantity is i [k]1 xi+ and the backward difference of a
 *    half-node quantity is i [k]1 xi-, xi+- = exp(+-i k1 dx1/2) (Eq. (18)).
 *    The hybrid solver replaces [k]1 by k1 (Eq. (20)); replacing it back by
 *    [k]1 gives the Yee scheme exactly, as stated at the end of Sec. 2.1.
 *    The signs of Eqs. (1)-(6) are used for the curl terms.
 *  - The Nyquist bin kappa1 = n1/2 is kept (its symbols are real).
 *  - B^n in Eqs. (15) and (17) is read as B^{n+1/2}, as in Eqs. (4)-(6).
 *  - B is advanced in two half steps around the E update so that B exists at
 *    integer time for the particle push; this is algebraically the leapfrog
 *    of Eqs. (12)-(17).
 *  - The low-pass filter of Sec. 4 is a sharp mask f(k1) = 1 for
 *    |k1| <= alpha pi/dx1 and 0 above, applied to all current components
 *    after the correction of Eq. (11).
 *  - Pusher: relativistic Boris.  Shape: quadratic B-spline (Table 2, Sec. 4),
 *    momentum-conserving interpolation (Appendix A, first variant).
 *  - Charge-conserving deposit: Esirkepov's scheme for the quadratic shape
 *    (the deposit the paper cites satisfies the continuity equation (23)).
 */
#include "hpic_oracle.h"

#include <complex.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846;

static int wrapi(int64_t i, int64_t n) {
  int64_t r = i % n;
  return (int)(r < 0 ? r + n : r);
}

static int is_pow2(int32_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* ------------------------------------------------------------------------ */
/* FFT: textbook iterative radix-2 Cooley-Tukey with bit-reversed input.     */
/* ------------------------------------------------------------------------ */

int or_fft(int32_t n, double *re, double *im, int32_t sign) {
  if (!is_pow2(n)) return -1;
  /* bit-reversal permutation */
  for (int32_t i = 1, j = 0; i < n; ++i) {
    int32_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double t = re[i]; re[i] = re[j]; re[j] = t;
      t = im[i]; im[i] = im[j]; im[j] = t;
    }
  }
  /* butterflies of growing length */
  for (int32_t len = 2; len <= n; len <<= 1) {
    for (int32_t start = 0; start < n; start += len) {
      for (int32_t k = 0; k < len / 2; ++k) {
        double ang = sign * 2.0 * PI * (double)k / (double)len;
        double wr = cos(ang), wi = sin(ang);
        int32_t a = start + k, b = start + k + len / 2;
        double xr = re[b] * wr - im[b] * wi;
        double xi = re[b] * wi + im[b] * wr;
        re[b] = re[a] - xr;
        im[b] = im[a] - xi;
        re[a] = re[a] + xr;
        im[a] = im[a] + xi;
      }
    }
  }
  return 0;
}

/* Threads of the OpenMP loops (1 without OpenMP); results do not depend on it. */
void or_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int32_t or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int or_rfft_rows(int32_t n1, int32_t nrows, const double *f, double *Fre, double *Fim) {
  if (!is_pow2(n1) || n1 < 2) return -1;
  int32_t nk = n1 / 2 + 1;
  /* rows are independent: with OpenMP each thread transforms its own rows */
#pragma omp parallel
  {
    double *re = malloc(sizeof(double) * n1), *im = malloc(sizeof(double) * n1);
#pragma omp for schedule(static)
    for (int32_t r = 0; r < nrows; ++r) {
      for (int32_t i = 0; i < n1; ++i) { re[i] = f[(int64_t)r * n1 + i]; im[i] = 0.0; }
      or_fft(n1, re, im, -1);
      for (int32_t k = 0; k < nk; ++k) {
        Fre[(int64_t)r * nk + k] = re[k];
        Fim[(int64_t)r * nk + k] = im[k];
      }
    }
    free(re); free(im);
  }
  return 0;
}

int or_irfft_rows(int32_t n1, int32_t nrows, const double *Fre, const double *Fim, double *f) {
  if (!is_pow2(n1) || n1 < 2) return -1;
  int32_t nk = n1 / 2 + 1;
#pragma omp parallel
  {
    double *re = malloc(sizeof(double) * n1), *im = malloc(sizeof(double) * n1);
#pragma omp for schedule(static)
    for (int32_t r = 0; r < nrows; ++r) {
      for (int32_t k = 0; k < nk; ++k) {
        re[k] = Fre[(int64_t)r * nk + k];
        im[k] = Fim[(int64_t)r * nk + k];
      }
      /* the self-conjugate bins of a real row have no imaginary part */
      im[0] = 0.0;
      im[n1 / 2] = 0.0;
      for (int32_t k = nk; k < n1; ++k) { re[k] = re[n1 - k]; im[k] = -im[n1 - k]; }
      or_fft(n1, re, im, +1);
      for (int32_t i = 0; i < n1; ++i) f[(int64_t)r * n1 + i] = re[i] / (double)n1;
    }
    free(re); free(im);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Particle shape and field gather                                           */
/* ------------------------------------------------------------------------ */

/* Quadratic B-spline: weight of a node at signed distance delta (cells). */
static double spline2(double delta) {
  double a = fabs(delta);
  if (a < 0.5) return 0.75 - a * a;
  if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
  return 0.0;
}

/* Linear (first-order) B-spline: weight of a node at signed distance delta. */
static double spline1(double delta) {
  double a = fabs(delta);
  return a < 1.0 ? 1.0 - a : 0.0;
}

/* Cubic B-spline: (4 - 6 a^2 + 3 a^3)/6 for a < 1, (2 - a)^3/6 for 1 <= a < 2. */
static double spline3c(double delta) {
  double a = fabs(delta);
  if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
  if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
  return 0.0;
}

/* B-spline of order 1, 2 or 3. */
static double spline_n(int order, double delta) {
  return order == 3 ? spline3c(delta) : order == 1 ? spline1(delta) : spline2(delta);
}

/* Shape order of a 2D grid (0 reads as the quadratic default). */
static int shape2(const or_grid2 *g) { return g->shape == 3 ? 3 : 2; }

/* Weight of a node along one direction for a component with staggering s
 * (0 or 1/2 cell) there: the quadratic spline, except that the energy-
 * conserving variant (Appendix A, second variant) lowers the order by one
 * along the staggered directions, which makes the work of the gathered field
 * on a particle equal to J.E of its Esirkepov current. */
static double gather_w(int interp, double s, double delta) {
  return (interp == 1 && s > 0.0) ? spline1(delta) : spline2(delta);
}
/* The same for a shape of order l (the variant lowers it to l - 1). */
static double gather_wn(int order, int interp, double s, double delta) {
  return spline_n((interp == 1 && s > 0.0) ? order - 1 : order, delta);
}

/* Staggering offsets (in cells) of E1..E3 and B1..B3 along x1 and x2, from the
 * index subscripts of Eqs. (1)-(6). */
static const double STAG_E[3][2] = {{0.5, 0.0}, {0.0, 0.5}, {0.0, 0.0}};
static const double STAG_B[3][2] = {{0.0, 0.5}, {0.5, 0.0}, {0.5, 0.5}};

/* Quadratic interpolation of one staggered component F at xi. */
static double interp2(const or_grid2 *g, const double *F, double s1, double s2, double xi1,
                      double xi2) {
  double e1 = xi1 - s1, e2 = xi2 - s2;
  int l = shape2(g);
  /* every node within two cells; the spline is zero beyond its support */
  int64_t m1 = (int64_t)floor(e1), m2 = (int64_t)floor(e2);
  double acc = 0.0;
  for (int64_t b = m2 - 2; b <= m2 + 3; ++b) {
    double w2 = gather_wn(l, g->interp, s2, e2 - (double)b);
    for (int64_t a = m1 - 2; a <= m1 + 3; ++a) {
      double w1 = gather_wn(l, g->interp, s1, e1 - (double)a);
      acc += w1 * w2 * F[(int64_t)wrapi(b, g->n2) * g->n1 + wrapi(a, g->n1)];
    }
  }
  return acc;
}

void or_gather2(const or_grid2 *g, const double *E, const double *B, int64_t np,
                const double *xi1, const double *xi2, double *Ep, double *Bp) {
  int64_t cells = (int64_t)g->n1 * g->n2;
  /* particles are independent: with OpenMP the loop is split over threads */
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    for (int c = 0; c < 3; ++c) {
      Ep[c * np + p] = interp2(g, E + c * cells, STAG_E[c][0], STAG_E[c][1], xi1[p], xi2[p]);
      Bp[c * np + p] = interp2(g, B + c * cells, STAG_B[c][0], STAG_B[c][1], xi1[p], xi2[p]);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Relativistic Boris push (half electric kick, magnetic rotation, half kick)*/
/* ------------------------------------------------------------------------ */

void or_boris(int64_t np, double qm, double dt, const double *Ep, const double *Bp,
              double *u1, double *u2, double *u3) {
  double h = 0.5 * qm * dt;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double e[3] = {h * Ep[p], h * Ep[np + p], h * Ep[2 * np + p]};
    double um[3] = {u1[p] + e[0], u2[p] + e[1], u3[p] + e[2]};
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * Bp[p] / gm, h * Bp[np + p] / gm, h * Bp[2 * np + p] / gm};
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double s[3] = {2.0 * t[0] / (1.0 + tt), 2.0 * t[1] / (1.0 + tt), 2.0 * t[2] / (1.0 + tt)};
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                    um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    double uq[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]),
                    um[1] + (up[2] * s[0] - up[0] * s[2]),
                    um[2] + (up[0] * s[1] - up[1] * s[0])};
    u1[p] = uq[0] + e[0];
    u2[p] = uq[1] + e[1];
    u3[p] = uq[2] + e[2];
  }
}

/* ------------------------------------------------------------------------ */
/* Esirkepov deposit, FP64                                                   */
/* ------------------------------------------------------------------------ */

int or_deposit2(const or_grid2 *g, int64_t np, const double *xa1, const double *xa2,
                const double *xb1, const double *xb2, const double *v3, const double *qw,
                double *J) {
  int64_t cells = (int64_t)g->n1 * g->n2;
  double *J1 = J, *J2 = J + cells, *J3 = J + 2 * cells;
  int status = 0, l = shape2(g);
  /* With OpenMP each thread owns a band of rows [r0, r1) of J and walks all
   * particles in order, adding only into its rows: every node receives its
   * contributions in particle order, as in one thread, so the result does not
   * depend on the number of threads. */
#pragma omp parallel reduction(min : status)
  {
    int32_t r0 = 0, r1 = g->n2;
#ifdef _OPENMP
    {
      int nt = omp_get_num_threads(), t = omp_get_thread_num();
      r0 = (int32_t)((int64_t)g->n2 * t / nt);
      r1 = (int32_t)((int64_t)g->n2 * (t + 1) / nt);
    }
#endif
    for (int64_t p = 0; p < np; ++p) {
      if (fabs(xb1[p] - xa1[p]) >= 1.0 || fabs(xb2[p] - xa2[p]) >= 1.0) { status = -1; continue; }
      /* a common window per coordinate holds the old and new stencils: the
       * nodes within two cells of either position (W = 6 covers the quadratic
       * and the cubic shape; the spline is zero beyond its support) */
      int64_t b1 = (int64_t)floor(fmin(xa1[p], xb1[p])) - 2;
      int64_t b2 = (int64_t)floor(fmin(xa2[p], xb2[p])) - 2;
      int row[6], mine = 0;
      for (int b = 0; b < 6; ++b) {
        row[b] = wrapi(b2 + b, g->n2);
        mine |= (row[b] >= r0 && row[b] < r1);
      }
      if (!mine) continue;
      double S0x[6], S1x[6], S0y[6], S1y[6];
      for (int a = 0; a < 6; ++a) {
        S0x[a] = spline_n(l, xa1[p] - (double)(b1 + a));
        S1x[a] = spline_n(l, xb1[p] - (double)(b1 + a));
        S0y[a] = spline_n(l, xa2[p] - (double)(b2 + a));
        S1y[a] = spline_n(l, xb2[p] - (double)(b2 + a));
      }
      double f1 = -qw[p] * g->dx1 / g->dt, f2 = -qw[p] * g->dx2 / g->dt;
      /* j1: running sum along x1 of the W1 weights (continuity, Eq. (23)) */
      for (int b = 0; b < 6; ++b) {
        if (row[b] < r0 || row[b] >= r1) continue;
        double acc = 0.0;
        for (int a = 0; a < 6; ++a) {
          double W1 = (S1x[a] - S0x[a]) * 0.5 * (S0y[b] + S1y[b]);
          acc += f1 * W1;
          J1[(int64_t)row[b] * g->n1 + wrapi(b1 + a, g->n1)] += acc;
        }
      }
      /* j2: running sum along x2 of the W2 weights */
      for (int a = 0; a < 6; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 6; ++b) {
          double W2 = (S1y[b] - S0y[b]) * 0.5 * (S0x[a] + S1x[a]);
          acc += f2 * W2;
          if (row[b] >= r0 && row[b] < r1)
            J2[(int64_t)row[b] * g->n1 + wrapi(b1 + a, g->n1)] += acc;
        }
      }
      /* j3: out-of-plane current with the time-averaged shape W3 */
      for (int b = 0; b < 6; ++b) {
        if (row[b] < r0 || row[b] >= r1) continue;
        for (int a = 0; a < 6; ++a) {
          double W3 = S0x[a] * S0y[b] / 3.0 + S1x[a] * S0y[b] / 6.0 + S0x[a] * S1y[b] / 6.0 +
                      S1x[a] * S1y[b] / 3.0;
          J3[(int64_t)row[b] * g->n1 + wrapi(b1 + a, g->n1)] += qw[p] * v3[p] * W3;
        }
      }
    }
  }
  return status;
}

void or_rho2(const or_grid2 *g, int64_t np, const double *xi1, const double *xi2,
             const double *qw, double *rho) {
  int l = shape2(g);
  for (int64_t p = 0; p < np; ++p) {
    int64_t m1 = (int64_t)floor(xi1[p]), m2 = (int64_t)floor(xi2[p]);
    for (int64_t b = m2 - 2; b <= m2 + 3; ++b)
      for (int64_t a = m1 - 2; a <= m1 + 3; ++a)
        rho[(int64_t)wrapi(b, g->n2) * g->n1 + wrapi(a, g->n1)] +=
            qw[p] * spline_n(l, xi1[p] - (double)a) * spline_n(l, xi2[p] - (double)b);
  }
}

/* ------------------------------------------------------------------------ */
/* Field solvers                                                             */
/* ------------------------------------------------------------------------ */

/* x1 symbols for mode kappa: the derivative k1 or [k]1, the current
 * correction of Eq. (11), and the filter mask of Sec. 4. */
typedef struct {
  double complex dp, dm; /* forward (integer->half) and backward (half->integer) */
  double corr, filt;
} xsym;

/* The modification of Eq. (29) to the spectral x1 symbol (zero outside the
 * bump [k1l, k1u]); coefficients of Sec. 4 for the Table 1 set-up. */
static double dk_mod(double k1, double dx1) {
  double kg = 2.0 * PI / dx1;
  double kl = 0.15 * kg, ku = 0.26 * kg, dkmax = 0.01 * kg, km = 0.5 * (kl + ku);
  if (fabs(k1) < kl || fabs(k1) > ku) return 0.0;
  double c = cos((fabs(k1) - km) / (kl - km) * PI / 2.0);
  return dkmax * c * c;
}

static xsym x1_symbols(const or_grid2 *g, int32_t kappa) {
  xsym s;
  double k1 = 2.0 * PI * (double)kappa / ((double)g->n1 * g->dx1);
  double h = 0.5 * k1 * g->dx1;
  double kfd = sin(h) / (0.5 * g->dx1);
  double kk = g->deriv1 ? kfd : k1 + (g->kmod ? dk_mod(k1, g->dx1) : 0.0);
  s.dp = I * kk * cexp(I * h);  /* i [k]1 xi+ */
  s.dm = I * kk * cexp(-I * h); /* i [k]1 xi- */
  s.corr = (g->deriv1 || !g->correct || kappa == 0) ? 1.0 : kfd / kk;
  s.filt = ((double)kappa <= g->alpha * 0.5 * (double)g->n1) ? 1.0 : 0.0;
  return s;
}

static void to_k(int32_t n1, int32_t n2, const double *f, double complex *F) {
  int32_t nk = n1 / 2 + 1;
  double *re = malloc(sizeof(double) * n2 * nk), *im = malloc(sizeof(double) * n2 * nk);
  or_rfft_rows(n1, n2, f, re, im);
  for (int64_t i = 0; i < (int64_t)n2 * nk; ++i) F[i] = re[i] + I * im[i];
  free(re); free(im);
}

static void from_k(int32_t n1, int32_t n2, const double complex *F, double *f) {
  int32_t nk = n1 / 2 + 1;
  double *re = malloc(sizeof(double) * n2 * nk), *im = malloc(sizeof(double) * n2 * nk);
  for (int64_t i = 0; i < (int64_t)n2 * nk; ++i) { re[i] = creal(F[i]); im[i] = cimag(F[i]); }
  or_irfft_rows(n1, n2, re, im, f);
  free(re); free(im);
}

/* Faraday half step B -= (dt/2) curl E in (kappa1, x2) space, Eqs. (12)-(14). */
static void faraday_half2(const or_grid2 *g, const double complex *Ek, double complex *Bk) {
  int32_t n2 = g->n2, nk = g->n1 / 2 + 1;
  int64_t plane = (int64_t)n2 * nk;
  const double complex *E1 = Ek, *E2 = Ek + plane, *E3 = Ek + 2 * plane;
  double complex *B1 = Bk, *B2 = Bk + plane, *B3 = Bk + 2 * plane;
  double hdt = 0.5 * g->dt;
  for (int32_t k = 0; k < nk; ++k) {
    xsym s = x1_symbols(g, k);
    for (int32_t i2 = 0; i2 < n2; ++i2) {
      int64_t c = (int64_t)i2 * nk + k, up = (int64_t)wrapi(i2 + 1, n2) * nk + k;
      double complex cE1 = (E3[up] - E3[c]) / g->dx2;
      double complex cE2 = -s.dp * E3[c];
      double complex cE3 = s.dp * E2[c] - (E1[up] - E1[c]) / g->dx2;
      B1[c] -= hdt * cE1;
      B2[c] -= hdt * cE2;
      B3[c] -= hdt * cE3;
    }
  }
}

int or_field_update2(const or_grid2 *g, double *E, double *B, const double *J) {
  int32_t n1 = g->n1, n2 = g->n2, nk = n1 / 2 + 1;
  if (!is_pow2(n1) || n1 < 2 || n2 < 1) return -1;
  int64_t cells = (int64_t)n1 * n2, plane = (int64_t)n2 * nk;
  double complex *Ek = malloc(sizeof(double complex) * 3 * plane);
  double complex *Bk = malloc(sizeof(double complex) * 3 * plane);
  double complex *Jk = malloc(sizeof(double complex) * 3 * plane);
  double *tmp = malloc(sizeof(double) * cells);
  for (int c = 0; c < 3; ++c) {
    to_k(n1, n2, E + c * cells, Ek + c * plane);
    to_k(n1, n2, B + c * cells, Bk + c * plane);
    for (int64_t i = 0; i < cells; ++i) tmp[i] = J[c * cells + i] + g->jbg[c];
    to_k(n1, n2, tmp, Jk + c * plane);
  }
  /* Eq. (11) on j1, then the low-pass mask on every component */
  for (int32_t k = 0; k < nk; ++k) {
    xsym s = x1_symbols(g, k);
    for (int32_t i2 = 0; i2 < n2; ++i2) {
      int64_t c = (int64_t)i2 * nk + k;
      Jk[c] *= s.corr * s.filt;
      Jk[plane + c] *= s.filt;
      Jk[2 * plane + c] *= s.filt;
    }
  }
  /* B^{n+1/2} = B^n - (dt/2) curl E^n */
  faraday_half2(g, Ek, Bk);
  /* E^{n+1} = E^n + dt (curl B^{n+1/2} - j), Eqs. (15)-(17) */
  {
    double complex *E1 = Ek, *E2 = Ek + plane, *E3 = Ek + 2 * plane;
    const double complex *B1 = Bk, *B2 = Bk + plane, *B3 = Bk + 2 * plane;
    for (int32_t k = 0; k < nk; ++k) {
      xsym s = x1_symbols(g, k);
      for (int32_t i2 = 0; i2 < n2; ++i2) {
        int64_t c = (int64_t)i2 * nk + k, dn = (int64_t)wrapi(i2 - 1, n2) * nk + k;
        double complex cB1 = (B3[c] - B3[dn]) / g->dx2;
        double complex cB2 = -s.dm * B3[c];
        double complex cB3 = s.dm * B2[c] - (B1[c] - B1[dn]) / g->dx2;
        E1[c] += g->dt * (cB1 - Jk[c]);
        E2[c] += g->dt * (cB2 - Jk[plane + c]);
        E3[c] += g->dt * (cB3 - Jk[2 * plane + c]);
      }
    }
  }
  /* B^{n+1} = B^{n+1/2} - (dt/2) curl E^{n+1} */
  faraday_half2(g, Ek, Bk);
  for (int c = 0; c < 3; ++c) {
    from_k(n1, n2, Ek + c * plane, E + c * cells);
    from_k(n1, n2, Bk + c * plane, B + c * cells);
  }
  free(Ek); free(Bk); free(Jk); free(tmp);
  return 0;
}

/* Real-space Yee half step for B, Eqs. (1)-(3) with dt/2. */
static void yee_faraday_half2(const or_grid2 *g, const double *E, double *B) {
  int32_t n1 = g->n1, n2 = g->n2;
  int64_t cells = (int64_t)n1 * n2;
  const double *E1 = E, *E2 = E + cells, *E3 = E + 2 * cells;
  double *B1 = B, *B2 = B + cells, *B3 = B + 2 * cells;
  double h = 0.5 * g->dt;
  for (int32_t i2 = 0; i2 < n2; ++i2) {
    for (int32_t i1 = 0; i1 < n1; ++i1) {
      int64_t c = (int64_t)i2 * n1 + i1;
      int64_t e1 = (int64_t)i2 * n1 + wrapi(i1 + 1, n1); /* (i1+1, i2) */
      int64_t e2 = (int64_t)wrapi(i2 + 1, n2) * n1 + i1; /* (i1, i2+1) */
      B1[c] -= h * (E3[e2] - E3[c]) / g->dx2;
      B2[c] += h * (E3[e1] - E3[c]) / g->dx1;
      B3[c] += -h * (E2[e1] - E2[c]) / g->dx1 + h * (E1[e2] - E1[c]) / g->dx2;
    }
  }
}

void or_yee_update2(const or_grid2 *g, double *E, double *B, const double *J) {
  int32_t n1 = g->n1, n2 = g->n2;
  int64_t cells = (int64_t)n1 * n2;
  yee_faraday_half2(g, E, B);
  double *E1 = E, *E2 = E + cells, *E3 = E + 2 * cells;
  const double *B1 = B, *B2 = B + cells, *B3 = B + 2 * cells;
  for (int32_t i2 = 0; i2 < n2; ++i2) {
    for (int32_t i1 = 0; i1 < n1; ++i1) {
      int64_t c = (int64_t)i2 * n1 + i1;
      int64_t w1 = (int64_t)i2 * n1 + wrapi(i1 - 1, n1); /* (i1-1, i2) */
      int64_t w2 = (int64_t)wrapi(i2 - 1, n2) * n1 + i1; /* (i1, i2-1) */
      E1[c] += -g->dt * (J[c] + g->jbg[0]) + g->dt * (B3[c] - B3[w2]) / g->dx2;
      E2[c] += -g->dt * (J[cells + c] + g->jbg[1]) - g->dt * (B3[c] - B3[w1]) / g->dx1;
      E3[c] += -g->dt * (J[2 * cells + c] + g->jbg[2]) + g->dt * (B2[c] - B2[w1]) / g->dx1 -
               g->dt * (B1[c] - B1[w2]) / g->dx2;
    }
  }
  yee_faraday_half2(g, E, B);
}

/* ------------------------------------------------------------------------ */
/* Whole step                                                                */
/* ------------------------------------------------------------------------ */

/* Antenna current (reading of Sec. 6, see the header): surface current K(t)
 * of a sheet at x_a(t), spread over x1 with the quadratic B-spline. */
void or_antenna2(const or_grid2 *g, const or_antenna *a, double t, double *J) {
  double s = t - a->t0;
  if (!(s >= 0.0 && s <= a->T) || !(a->T > 0.0)) return;
  double env = sin(PI * s / a->T);
  double K = a->K0 * env * env * sin(a->omega * s + a->phase);
  double L1 = g->n1 * g->dx1, L2 = g->n2 * g->dx2;
  double xa = fmod(a->x0 + a->v * t, L1);
  if (xa < 0.0) xa += L1;
  double sa = xa / g->dx1;
  int64_t cells = (int64_t)g->n1 * g->n2;
  double *J3 = J + 2 * cells;
  for (int32_t j = 0; j < g->n2; ++j) {
    double gx = 1.0;
    if (a->waist > 0.0) {
      double d = fmod(j * g->dx2 - a->x2c, L2);
      if (d < -0.5 * L2) d += L2;
      if (d >= 0.5 * L2) d -= L2;
      gx = exp(-(d / a->waist) * (d / a->waist));
    }
    /* every node whose spline support contains the sheet */
    for (int32_t i = (int32_t)floor(sa) - 2; i <= (int32_t)floor(sa) + 3; ++i) {
      double w = spline2(sa - i);
      if (w == 0.0) continue;
      J3[(int64_t)j * g->n1 + wrapi(i, g->n1)] += K * gx * w / g->dx1;
    }
  }
}

int or_step2(const or_grid2 *g, double qm, int64_t np, double *xi1, double *xi2,
             double *u1, double *u2, double *u3, const double *qw, double *E, double *B,
             double *J, const or_antenna *ant, double t) {
  int64_t cells = (int64_t)g->n1 * g->n2;
  double *Ep = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
  double *Bp = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
  double *xn1 = malloc(sizeof(double) * (np > 0 ? np : 1));
  double *xn2 = malloc(sizeof(double) * (np > 0 ? np : 1));
  double *v3 = malloc(sizeof(double) * (np > 0 ? np : 1));
  or_gather2(g, E, B, np, xi1, xi2, Ep, Bp);
  or_boris(np, qm, g->dt, Ep, Bp, u1, u2, u3);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double gam = sqrt(1.0 + u1[p] * u1[p] + u2[p] * u2[p] + u3[p] * u3[p]);
    xn1[p] = xi1[p] + g->dt * (u1[p] / gam) / g->dx1;
    xn2[p] = xi2[p] + g->dt * (u2[p] / gam) / g->dx2;
    v3[p] = u3[p] / gam;
  }
  memset(J, 0, sizeof(double) * 3 * cells);
  int status = or_deposit2(g, np, xi1, xi2, xn1, xn2, v3, qw, J);
  if (ant) or_antenna2(g, ant, t + 0.5 * g->dt, J);
  if (or_field_update2(g, E, B, J) != 0) status = -1;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    xi1[p] = fmod(xn1[p], (double)g->n1);
    if (xi1[p] < 0.0) xi1[p] += (double)g->n1;
    xi2[p] = fmod(xn2[p], (double)g->n2);
    if (xi2[p] < 0.0) xi2[p] += (double)g->n2;
  }
  free(Ep); free(Bp); free(xn1); free(xn2); free(v3);
  return status;
}

int or_gauss2(const or_grid2 *g, const double *E, const double *rho, double *Rre, double *Rim) {
  int32_t n1 = g->n1, n2 = g->n2, nk = n1 / 2 + 1;
  if (!is_pow2(n1) || n1 < 2) return -1;
  int64_t cells = (int64_t)n1 * n2, plane = (int64_t)n2 * nk;
  double complex *E1 = malloc(sizeof(double complex) * plane);
  double complex *E2 = malloc(sizeof(double complex) * plane);
  double complex *R = malloc(sizeof(double complex) * plane);
  to_k(n1, n2, E, E1);
  to_k(n1, n2, E + cells, E2);
  to_k(n1, n2, rho, R);
  for (int32_t k = 0; k < nk; ++k) {
    xsym s = x1_symbols(g, k);
    for (int32_t i2 = 0; i2 < n2; ++i2) {
      int64_t c = (int64_t)i2 * nk + k, dn = (int64_t)wrapi(i2 - 1, n2) * nk + k;
      double complex div = s.dm * E1[c] + (E2[c] - E2[dn]) / g->dx2;
      R[c] = div - s.filt * R[c];
    }
  }
  for (int64_t i = 0; i < plane; ++i) { Rre[i] = creal(R[i]); Rim[i] = cimag(R[i]); }
  free(E1); free(E2); free(R);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Fixed-point deposit in the kernel's precision                             */
/* ------------------------------------------------------------------------ */
/*
 * The GPU accumulates the current in 64-bit integers.  To keep the discrete
 * continuity equation (23) exact in those integers, the shape factors of each
 * coordinate are themselves integers that sum to exactly 2^P:
 *   d = offset from the nearest node in [-1/2, 1/2)   (FP32, exact)
 *   D = rint(d 2^P)                                    (FP32 rint)
 *   s(-1) = round((2^(P-1) - D)^2 / 2^(P+1)),  s(+1) = round((2^(P-1) + D)^2 / 2^(P+1))
 *   s(0)  = 2^P - s(-1) - s(+1)
 * which are the quadratic B-spline weights 1/2 (1/2 -+ d)^2 and 3/4 - d^2 times
 * 2^P, rounded (halves up).  With the integer charge Q = rint(qw * inv_wunit)
 * the Esirkepov weights become exact integer products:
 *   J1[a][b] = Q C1[a] (S0y[b] + S1y[b]),   C1[a] = sum_{a'<=a} (S1x[a'] - S0x[a'])
 *   J2[a][b] = Q C2[b] (S0x[a] + S1x[a]),   C2[b] = sum_{b'<=b} (S1y[b'] - S0y[b'])
 * and 2 (rho_new - rho_old) = div J holds node by node in integers, where
 * rho = Q s1 s2.  Physical units: j1 = -(dx1/dt) J1 / (inv_wunit 2^(2P+1)) and
 * likewise j2 with dx2.  The out-of-plane j3 does not enter the continuity
 * equation in 2D; it is FP32 with the same operation order as the kernel:
 *   h = ((qw inv_wunit) v3) c3,  x0[a] = S0x[a] h,  x1[a] = S1x[a] h,
 *   t0[b] = 2 S0y[b] + S1y[b],   t1[b] = S0y[b] + 2 S1y[b],
 *   J3 += rint(fma(x0[a], t0[b], x1[a] t1[b]))
 * (the product x1 t1 rounded once, then one fused multiply-add), which is
 * h times 6 W3 of the Esirkepov scheme, so that j3 = J3 / (inv_wunit c3 6 2^(2P)).
 * This file is compiled with floating-point contraction off so that each FP32
 * operation rounds once, as in the kernel.
 */

static int32_t fixed_shape(int32_t cell, float f, int32_t P, int64_t s[3]) {
  int32_t up = (f >= 0.5f);
  float d = up ? (f - 1.0f) : f;
  float scaled = d * (float)(1 << P);
  int64_t D = (int64_t)rintf(scaled);
  int64_t h = (int64_t)1 << (P - 1);
  int64_t bias = (int64_t)1 << P;
  s[0] = ((h - D) * (h - D) + bias) >> (P + 1);
  s[2] = ((h + D) * (h + D) + bias) >> (P + 1);
  s[1] = ((int64_t)1 << P) - s[0] - s[2];
  return cell + up;
}

static int32_t wrap_delta(int32_t db, int32_t n) {
  int32_t d = wrapi(db, n);
  return d > n / 2 ? d - n : d;
}

int or_deposit2_fixed(int32_t n1, int32_t n2, int32_t P, float inv_wunit, float c3,
                      int64_t np, const int32_t *ca1, const int32_t *ca2, const float *fa1,
                      const float *fa2, const int32_t *cb1, const int32_t *cb2,
                      const float *fb1, const float *fb2, const float *v3, const float *qw,
                      int64_t *J) {
  int64_t cells = (int64_t)n1 * n2;
  int64_t *J1 = J, *J2 = J + cells, *J3 = J + 2 * cells;
  int status = 0;
  for (int64_t p = 0; p < np; ++p) {
    int32_t d1 = wrap_delta(cb1[p] - ca1[p], n1), d2 = wrap_delta(cb2[p] - ca2[p], n2);
    if (d1 < -1 || d1 > 1 || d2 < -1 || d2 > 1) { status = -1; continue; }
    int64_t sa1[3], sa2[3], sb1[3], sb2[3];
    int32_t na1 = fixed_shape(ca1[p], fa1[p], P, sa1);
    int32_t nb1 = fixed_shape(ca1[p] + d1, fb1[p], P, sb1);
    int32_t na2 = fixed_shape(ca2[p], fa2[p], P, sa2);
    int32_t nb2 = fixed_shape(ca2[p] + d2, fb2[p], P, sb2);
    if (na1 - nb1 > 1 || nb1 - na1 > 1 || na2 - nb2 > 1 || nb2 - na2 > 1) { status = -1; continue; }
    int32_t base1 = (na1 < nb1 ? na1 : nb1) - 1, base2 = (na2 < nb2 ? na2 : nb2) - 1;
    int64_t S0x[4] = {0, 0, 0, 0}, S1x[4] = {0, 0, 0, 0}, S0y[4] = {0, 0, 0, 0},
            S1y[4] = {0, 0, 0, 0};
    for (int k = 0; k < 3; ++k) {
      S0x[na1 - 1 - base1 + k] = sa1[k];
      S1x[nb1 - 1 - base1 + k] = sb1[k];
      S0y[na2 - 1 - base2 + k] = sa2[k];
      S1y[nb2 - 1 - base2 + k] = sb2[k];
    }
    float qs = qw[p] * inv_wunit;
    int64_t Q = (int64_t)rintf(qs);
    int64_t C1[4], C2[4], acc1 = 0, acc2 = 0;
    for (int a = 0; a < 4; ++a) {
      acc1 += S1x[a] - S0x[a];
      acc2 += S1y[a] - S0y[a];
      C1[a] = acc1;
      C2[a] = acc2;
    }
    for (int b = 0; b < 4; ++b) {
      for (int a = 0; a < 4; ++a) {
        int64_t idx = (int64_t)wrapi(base2 + b, n2) * n1 + wrapi(base1 + a, n1);
        J1[idx] += Q * C1[a] * (S0y[b] + S1y[b]);
        J2[idx] += Q * C2[b] * (S0x[a] + S1x[a]);
      }
    }
    float hv = qs * v3[p];
    float h = hv * c3;
    for (int b = 0; b < 4; ++b) {
      for (int a = 0; a < 4; ++a) {
        float x0 = (float)S0x[a] * h;
        float x1 = (float)S1x[a] * h;
        float B0 = (float)S0y[b], B1 = (float)S1y[b];
        float t0 = 2.0f * B0 + B1;
        float t1 = B0 + 2.0f * B1;
        float p1 = x1 * t1;
        float v = fmaf(x0, t0, p1);
        int64_t idx = (int64_t)wrapi(base2 + b, n2) * n1 + wrapi(base1 + a, n1);
        J3[idx] += (int64_t)rintf(v);
      }
    }
  }
  return status;
}

void or_rho2_fixed(int32_t n1, int32_t n2, int32_t P, float inv_wunit, int64_t np,
                   const int32_t *c1, const int32_t *c2, const float *f1, const float *f2,
                   const float *qw, int64_t *rho) {
  for (int64_t p = 0; p < np; ++p) {
    int64_t s1[3], s2[3];
    int32_t m1 = fixed_shape(c1[p], f1[p], P, s1);
    int32_t m2 = fixed_shape(c2[p], f2[p], P, s2);
    int64_t Q = (int64_t)rintf(qw[p] * inv_wunit);
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        rho[(int64_t)wrapi(m2 - 1 + b, n2) * n1 + wrapi(m1 - 1 + a, n1)] += Q * s1[a] * s2[b];
  }
}

/* ======================================================================== */
/* 3D Cartesian                                                              */
/* ======================================================================== */
/*
 * Grid n1 x n2 x n3, periodic, arrays [comp][i3][i2][i1].  Yee staggering
 * extended to three dimensions in the standard way (Sec. 2.2 gives the 3D
 * form by adding the x3 differences): E1 at (i1+1/2, i2, i3), E2 at
 * (i1, i2+1/2, i3), E3 at (i1, i2, i3+1/2), B1 at (i1, i2+1/2, i3+1/2),
 * B2 at (i1+1/2, i2, i3+1/2), B3 at (i1+1/2, i2+1/2, i3).  The hybrid solver
 * transforms along x1 only; x2 and x3 use centred finite differences.
 */

static const double STAG3_E[3][3] = {{0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5}};
static const double STAG3_B[3][3] = {{0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}};

static int64_t idx3(const or_grid3 *g, int64_t a, int64_t b, int64_t c) {
  return ((int64_t)wrapi(c, g->n3) * g->n2 + wrapi(b, g->n2)) * g->n1 + wrapi(a, g->n1);
}

static double interp3(const or_grid3 *g, const double *F, const double s[3], double x1,
                      double x2, double x3) {
  double e1 = x1 - s[0], e2 = x2 - s[1], e3 = x3 - s[2];
  int64_t m1 = (int64_t)floor(e1 + 0.5), m2 = (int64_t)floor(e2 + 0.5), m3 = (int64_t)floor(e3 + 0.5);
  double acc = 0.0;
  for (int64_t c = m3 - 1; c <= m3 + 1; ++c) {
    double w3 = gather_w(g->interp, s[2], e3 - (double)c);
    for (int64_t b = m2 - 1; b <= m2 + 1; ++b) {
      double w2 = gather_w(g->interp, s[1], e2 - (double)b);
      for (int64_t a = m1 - 1; a <= m1 + 1; ++a)
        acc += gather_w(g->interp, s[0], e1 - (double)a) * w2 * w3 * F[idx3(g, a, b, c)];
    }
  }
  return acc;
}

void or_gather3(const or_grid3 *g, const double *E, const double *B, int64_t np,
                const double *xi1, const double *xi2, const double *xi3, double *Ep, double *Bp) {
  int64_t cells = (int64_t)g->n1 * g->n2 * g->n3;
  for (int64_t p = 0; p < np; ++p)
    for (int c = 0; c < 3; ++c) {
      Ep[c * np + p] = interp3(g, E + c * cells, STAG3_E[c], xi1[p], xi2[p], xi3[p]);
      Bp[c * np + p] = interp3(g, B + c * cells, STAG3_B[c], xi1[p], xi2[p], xi3[p]);
    }
}

/* Esirkepov deposit in 3D (quadratic shape).  With S0, S1 the old and new
 * shape factors per coordinate on a common 4-node window and DS = S1 - S0,
 *   W1 = DS1 (S0_2 S0_3 + DS2 S0_3 / 2 + S0_2 DS3 / 2 + DS2 DS3 / 3)
 * and cyclically for W2, W3; then W1 + W2 + W3 = S1_1 S1_2 S1_3 - S0_1 S0_2 S0_3
 * and j_d is the running sum of -q w (dx_d / dt) W_d along x_d, which makes the
 * continuity equation hold node by node. */
int or_deposit3(const or_grid3 *g, int64_t np, const double *xa1, const double *xa2,
                const double *xa3, const double *xb1, const double *xb2, const double *xb3,
                const double *qw, double *J) {
  int64_t cells = (int64_t)g->n1 * g->n2 * g->n3;
  const double *xa[3] = {xa1, xa2, xa3}, *xb[3] = {xb1, xb2, xb3};
  const double dx[3] = {g->dx1, g->dx2, g->dx3};
  int status = 0;
  for (int64_t p = 0; p < np; ++p) {
    int bad = 0;
    for (int d = 0; d < 3; ++d) bad |= fabs(xb[d][p] - xa[d][p]) >= 1.0;
    if (bad) { status = -1; continue; }
    int64_t base[3];
    double S0[3][4], S1[3][4], DS[3][4];
    for (int d = 0; d < 3; ++d) {
      base[d] = (int64_t)fmin(floor(xa[d][p] + 0.5), floor(xb[d][p] + 0.5)) - 1;
      for (int k = 0; k < 4; ++k) {
        S0[d][k] = spline2(xa[d][p] - (double)(base[d] + k));
        S1[d][k] = spline2(xb[d][p] - (double)(base[d] + k));
        DS[d][k] = S1[d][k] - S0[d][k];
      }
    }
    /* component d: running sum along x_d; (e, f) are the other two axes */
    for (int d = 0; d < 3; ++d) {
      int e = (d + 1) % 3, f = (d + 2) % 3;
      double fac = -qw[p] * dx[d] / g->dt;
      for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) {
          double tr = S0[e][i] * S0[f][j] + 0.5 * DS[e][i] * S0[f][j] +
                      0.5 * S0[e][i] * DS[f][j] + DS[e][i] * DS[f][j] / 3.0;
          double acc = 0.0;
          for (int k = 0; k < 4; ++k) {
            acc += fac * DS[d][k] * tr;
            int64_t n[3];
            n[d] = base[d] + k;
            n[e] = base[e] + i;
            n[f] = base[f] + j;
            J[d * cells + idx3(g, n[0], n[1], n[2])] += acc;
          }
        }
      }
    }
  }
  return status;
}

void or_rho3(const or_grid3 *g, int64_t np, const double *xi1, const double *xi2,
             const double *xi3, const double *qw, double *rho) {
  for (int64_t p = 0; p < np; ++p) {
    int64_t m1 = (int64_t)floor(xi1[p] + 0.5), m2 = (int64_t)floor(xi2[p] + 0.5),
            m3 = (int64_t)floor(xi3[p] + 0.5);
    for (int64_t c = m3 - 1; c <= m3 + 1; ++c)
      for (int64_t b = m2 - 1; b <= m2 + 1; ++b)
        for (int64_t a = m1 - 1; a <= m1 + 1; ++a)
          rho[idx3(g, a, b, c)] += qw[p] * spline2(xi1[p] - (double)a) *
                                   spline2(xi2[p] - (double)b) * spline2(xi3[p] - (double)c);
  }
}

static xsym x1_symbols3(const or_grid3 *g, int32_t kappa) {
  or_grid2 g2;
  g2.n1 = g->n1; g2.n2 = g->n2; g2.dx1 = g->dx1; g2.dx2 = g->dx2; g2.dt = g->dt;
  g2.alpha = g->alpha; g2.deriv1 = g->deriv1; g2.correct = g->correct;
  g2.kmod = g->kmod;
  return x1_symbols(&g2, kappa);
}

/* Faraday half step B -= (dt/2) curl E in (kappa1, x2, x3) space:
 * curl E = (D2+ E3 - D3+ E2, D3+ E1 - D1+ E3, D1+ E2 - D2+ E1). */
static void faraday_half3(const or_grid3 *g, const double complex *Ek, double complex *Bk) {
  int32_t n2 = g->n2, n3 = g->n3, nk = g->n1 / 2 + 1;
  int64_t vol = (int64_t)n3 * n2 * nk;
  const double complex *E1 = Ek, *E2 = Ek + vol, *E3 = Ek + 2 * vol;
  double complex *B1 = Bk, *B2 = Bk + vol, *B3 = Bk + 2 * vol;
  double hdt = 0.5 * g->dt;
  for (int32_t k = 0; k < nk; ++k) {
    xsym s = x1_symbols3(g, k);
    for (int32_t i3 = 0; i3 < n3; ++i3)
      for (int32_t i2 = 0; i2 < n2; ++i2) {
        int64_t c = ((int64_t)i3 * n2 + i2) * nk + k;
        int64_t u2 = ((int64_t)i3 * n2 + wrapi(i2 + 1, n2)) * nk + k;
        int64_t u3 = ((int64_t)wrapi(i3 + 1, n3) * n2 + i2) * nk + k;
        double complex cE1 = (E3[u2] - E3[c]) / g->dx2 - (E2[u3] - E2[c]) / g->dx3;
        double complex cE2 = (E1[u3] - E1[c]) / g->dx3 - s.dp * E3[c];
        double complex cE3 = s.dp * E2[c] - (E1[u2] - E1[c]) / g->dx2;
        B1[c] -= hdt * cE1;
        B2[c] -= hdt * cE2;
        B3[c] -= hdt * cE3;
      }
  }
}

int or_field_update3(const or_grid3 *g, double *E, double *B, const double *J) {
  int32_t n1 = g->n1, n2 = g->n2, n3 = g->n3, nk = n1 / 2 + 1;
  if (!is_pow2(n1) || n1 < 2 || n2 < 1 || n3 < 1) return -1;
  int32_t rows = n2 * n3;
  int64_t cells = (int64_t)n1 * rows, vol = (int64_t)rows * nk;
  double complex *Ek = malloc(sizeof(double complex) * 3 * vol);
  double complex *Bk = malloc(sizeof(double complex) * 3 * vol);
  double complex *Jk = malloc(sizeof(double complex) * 3 * vol);
  double *tmp = malloc(sizeof(double) * cells);
  for (int c = 0; c < 3; ++c) {
    to_k(n1, rows, E + c * cells, Ek + c * vol);
    to_k(n1, rows, B + c * cells, Bk + c * vol);
    for (int64_t i = 0; i < cells; ++i) tmp[i] = J[c * cells + i] + g->jbg[c];
    to_k(n1, rows, tmp, Jk + c * vol);
  }
  for (int32_t k = 0; k < nk; ++k) {
    xsym s = x1_symbols3(g, k);
    for (int32_t r = 0; r < rows; ++r) {
      int64_t c = (int64_t)r * nk + k;
      Jk[c] *= s.corr * s.filt;
      Jk[vol + c] *= s.filt;
      Jk[2 * vol + c] *= s.filt;
    }
  }
  faraday_half3(g, Ek, Bk);
  {
    double complex *E1 = Ek, *E2 = Ek + vol, *E3 = Ek + 2 * vol;
    const double complex *B1 = Bk, *B2 = Bk + vol, *B3 = Bk + 2 * vol;
    /* curl B = (D2- B3 - D3- B2, D3- B1 - D1- B3, D1- B2 - D2- B1) */
    for (int32_t k = 0; k < nk; ++k) {
      xsym s = x1_symbols3(g, k);
      for (int32_t i3 = 0; i3 < n3; ++i3)
        for (int32_t i2 = 0; i2 < n2; ++i2) {
          int64_t c = ((int64_t)i3 * n2 + i2) * nk + k;
          int64_t d2 = ((int64_t)i3 * n2 + wrapi(i2 - 1, n2)) * nk + k;
          int64_t d3 = ((int64_t)wrapi(i3 - 1, n3) * n2 + i2) * nk + k;
          double complex cB1 = (B3[c] - B3[d2]) / g->dx2 - (B2[c] - B2[d3]) / g->dx3;
          double complex cB2 = (B1[c] - B1[d3]) / g->dx3 - s.dm * B3[c];
          double complex cB3 = s.dm * B2[c] - (B1[c] - B1[d2]) / g->dx2;
          E1[c] += g->dt * (cB1 - Jk[c]);
          E2[c] += g->dt * (cB2 - Jk[vol + c]);
          E3[c] += g->dt * (cB3 - Jk[2 * vol + c]);
        }
    }
  }
  faraday_half3(g, Ek, Bk);
  for (int c = 0; c < 3; ++c) {
    from_k(n1, rows, Ek + c * vol, E + c * cells);
    from_k(n1, rows, Bk + c * vol, B + c * cells);
  }
  free(Ek); free(Bk); free(Jk); free(tmp);
  return 0;
}

/* Direct real-space Yee update in 3D (Yee's centred differences in all three
 * directions; no FFT, filter or correction; jbg added). */
static void yee_faraday_half3(const or_grid3 *g, const double *E, double *B) {
  int64_t cells = (int64_t)g->n1 * g->n2 * g->n3;
  const double *E1 = E, *E2 = E + cells, *E3 = E + 2 * cells;
  double *B1 = B, *B2 = B + cells, *B3 = B + 2 * cells;
  double h = 0.5 * g->dt;
  for (int32_t i3 = 0; i3 < g->n3; ++i3)
    for (int32_t i2 = 0; i2 < g->n2; ++i2)
      for (int32_t i1 = 0; i1 < g->n1; ++i1) {
        int64_t c = idx3(g, i1, i2, i3);
        int64_t p1 = idx3(g, i1 + 1, i2, i3), p2 = idx3(g, i1, i2 + 1, i3), p3 = idx3(g, i1, i2, i3 + 1);
        B1[c] -= h * ((E3[p2] - E3[c]) / g->dx2 - (E2[p3] - E2[c]) / g->dx3);
        B2[c] -= h * ((E1[p3] - E1[c]) / g->dx3 - (E3[p1] - E3[c]) / g->dx1);
        B3[c] -= h * ((E2[p1] - E2[c]) / g->dx1 - (E1[p2] - E1[c]) / g->dx2);
      }
}

void or_yee_update3(const or_grid3 *g, double *E, double *B, const double *J) {
  int64_t cells = (int64_t)g->n1 * g->n2 * g->n3;
  yee_faraday_half3(g, E, B);
  double *E1 = E, *E2 = E + cells, *E3 = E + 2 * cells;
  const double *B1 = B, *B2 = B + cells, *B3 = B + 2 * cells;
  for (int32_t i3 = 0; i3 < g->n3; ++i3)
    for (int32_t i2 = 0; i2 < g->n2; ++i2)
      for (int32_t i1 = 0; i1 < g->n1; ++i1) {
        int64_t c = idx3(g, i1, i2, i3);
        int64_t m1 = idx3(g, i1 - 1, i2, i3), m2 = idx3(g, i1, i2 - 1, i3), m3 = idx3(g, i1, i2, i3 - 1);
        E1[c] += g->dt * ((B3[c] - B3[m2]) / g->dx2 - (B2[c] - B2[m3]) / g->dx3 - (J[c] + g->jbg[0]));
        E2[c] += g->dt * ((B1[c] - B1[m3]) / g->dx3 - (B3[c] - B3[m1]) / g->dx1 -
                          (J[cells + c] + g->jbg[1]));
        E3[c] += g->dt * ((B2[c] - B2[m1]) / g->dx1 - (B1[c] - B1[m2]) / g->dx2 -
                          (J[2 * cells + c] + g->jbg[2]));
      }
  yee_faraday_half3(g, E, B);
}

int or_step3(const or_grid3 *g, double qm, int64_t np, double *xi1, double *xi2, double *xi3,
             double *u1, double *u2, double *u3, const double *qw, double *E, double *B,
             double *J) {
  int64_t cells = (int64_t)g->n1 * g->n2 * g->n3;
  int64_t m = np > 0 ? np : 1;
  double *Ep = malloc(sizeof(double) * 3 * m), *Bp = malloc(sizeof(double) * 3 * m);
  double *xn1 = malloc(sizeof(double) * m), *xn2 = malloc(sizeof(double) * m),
         *xn3 = malloc(sizeof(double) * m);
  or_gather3(g, E, B, np, xi1, xi2, xi3, Ep, Bp);
  or_boris(np, qm, g->dt, Ep, Bp, u1, u2, u3);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    double gam = sqrt(1.0 + u1[p] * u1[p] + u2[p] * u2[p] + u3[p] * u3[p]);
    xn1[p] = xi1[p] + g->dt * (u1[p] / gam) / g->dx1;
    xn2[p] = xi2[p] + g->dt * (u2[p] / gam) / g->dx2;
    xn3[p] = xi3[p] + g->dt * (u3[p] / gam) / g->dx3;
  }
  memset(J, 0, sizeof(double) * 3 * cells);
  int status = or_deposit3(g, np, xi1, xi2, xi3, xn1, xn2, xn3, qw, J);
  if (or_field_update3(g, E, B, J) != 0) status = -1;
  double *xs[3] = {xi1, xi2, xi3}, *xn[3] = {xn1, xn2, xn3};
  const int32_t n[3] = {g->n1, g->n2, g->n3};
  for (int d = 0; d < 3; ++d)
    for (int64_t p = 0; p < np; ++p) {
      double v = fmod(xn[d][p], (double)n[d]);
      xs[d][p] = v < 0.0 ? v + (double)n[d] : v;
    }
  free(Ep); free(Bp); free(xn1); free(xn2); free(xn3);
  return status;
}

int or_gauss3(const or_grid3 *g, const double *E, const double *rho, double *Rre, double *Rim) {
  int32_t n1 = g->n1, n2 = g->n2, n3 = g->n3, nk = n1 / 2 + 1;
  if (!is_pow2(n1) || n1 < 2) return -1;
  int32_t rows = n2 * n3;
  int64_t cells = (int64_t)n1 * rows, vol = (int64_t)rows * nk;
  double complex *E1 = malloc(sizeof(double complex) * vol);
  double complex *E2 = malloc(sizeof(double complex) * vol);
  double complex *E3 = malloc(sizeof(double complex) * vol);
  double complex *R = malloc(sizeof(double complex) * vol);
  to_k(n1, rows, E, E1);
  to_k(n1, rows, E + cells, E2);
  to_k(n1, rows, E + 2 * cells, E3);
  to_k(n1, rows, rho, R);
  for (int32_t k = 0; k < nk; ++k) {
    xsym s = x1_symbols3(g, k);
    for (int32_t i3 = 0; i3 < n3; ++i3)
      for (int32_t i2 = 0; i2 < n2; ++i2) {
        int64_t c = ((int64_t)i3 * n2 + i2) * nk + k;
        int64_t d2 = ((int64_t)i3 * n2 + wrapi(i2 - 1, n2)) * nk + k;
        int64_t d3 = ((int64_t)wrapi(i3 - 1, n3) * n2 + i2) * nk + k;
        double complex div = s.dm * E1[c] + (E2[c] - E2[d2]) / g->dx2 + (E3[c] - E3[d3]) / g->dx3;
        R[c] = div - s.filt * R[c];
      }
  }
  for (int64_t i = 0; i < vol; ++i) { Rre[i] = creal(R[i]); Rim[i] = cimag(R[i]); }
  free(E1); free(E2); free(E3); free(R);
  return 0;
}

/* ---- 3D deposit in the kernel's precision ----
 * The product of three shape factors does not fit the 64-bit budget of an
 * exact integer scheme with arbitrary charges, so the 3D FP32 form computes
 * the Esirkepov weights of its FP32 particle offsets in FP64 and rounds each
 * node's contribution once to an integer on a fine scale (cj = 2^40 per unit
 * charge); the integers then add up in any order to the same 64-bit total, and
 * continuity (Eq. (23)) holds to about 2^-41 of a particle's charge per node
 * and step instead of to FP32 rounding.  Per coordinate, FP64 shape factors at
 * the three nodes around the nearest node m (d = offset from m, exact):
 *   a = 0.5 - d, b = 0.5 + d:  s(-1) = 0.5 (a a),  s(0) = 0.75 - d d,  s(+1) = 0.5 (b b)
 * placed on the common 4-node window; DS = S1 - S0; running sums
 * C[k] = C[k-1] + DS[k] in order.  For component d with the other two axes
 * (e, f) in cyclic order:
 *   u0[j] = 2 S0_f[j] + S1_f[j],  u1[j] = S0_f[j] + 2 S1_f[j]
 *   T[i][j] = S0_e[i] u0[j] + S1_e[i] u1[j]          (6 times the Esirkepov bracket)
 *   J_d[k][i][j] += rint((C_d[k] g) T[i][j]),  g = (qw inv_wunit) cj,  k = 0..2
 * each FP64 operation rounded once in this order (no contraction), so that
 * j_d = -(dx_d / dt) J_d / (6 inv_wunit cj).  |J| per particle <= 6 cj. */
static int32_t dshape3_fixed(int32_t cell, float f, double s[3]) {
  int32_t up = (f >= 0.5f);
  double d = up ? ((double)f - 1.0) : (double)f;
  double a = 0.5 - d, b = 0.5 + d;
  s[0] = 0.5 * (a * a);
  s[1] = 0.75 - d * d;
  s[2] = 0.5 * (b * b);
  return cell + up;
}

int or_deposit3_fixed(int32_t n1, int32_t n2, int32_t n3, float inv_wunit, float cj, int64_t np,
                      const int32_t *ca, const float *fa, const int32_t *cb, const float *fb,
                      const float *qw, int64_t *J) {
  or_grid3 g;
  memset(&g, 0, sizeof g);
  g.n1 = n1; g.n2 = n2; g.n3 = n3;
  int64_t cells = (int64_t)n1 * n2 * n3;
  const int32_t n[3] = {n1, n2, n3};
  int status = 0;
  for (int64_t p = 0; p < np; ++p) {
    double S0[3][4], S1[3][4], C[3][4];
    int32_t base[3], bad = 0;
    for (int d = 0; d < 3; ++d) {
      int32_t dd = wrap_delta(cb[d * np + p] - ca[d * np + p], n[d]);
      if (dd < -1 || dd > 1) bad = 1;
      double sa[3], sb[3];
      int32_t na = dshape3_fixed(ca[d * np + p], fa[d * np + p], sa);
      int32_t nb = dshape3_fixed(ca[d * np + p] + dd, fb[d * np + p], sb);
      if (na - nb > 1 || nb - na > 1) bad = 1;
      base[d] = (na < nb ? na : nb) - 1;
      for (int k = 0; k < 4; ++k) S0[d][k] = S1[d][k] = 0.0;
      if (!bad)
        for (int k = 0; k < 3; ++k) {
          S0[d][na - 1 - base[d] + k] = sa[k];
          S1[d][nb - 1 - base[d] + k] = sb[k];
        }
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) {
        acc = acc + (S1[d][k] - S0[d][k]);
        C[d][k] = acc;
      }
    }
    if (bad) { status = -1; continue; }
    double gq = ((double)qw[p] * (double)inv_wunit) * (double)cj;
    for (int d = 0; d < 3; ++d) {
      int e = (d + 1) % 3, f = (d + 2) % 3;
      double u0[4], u1[4];
      for (int j = 0; j < 4; ++j) {
        u0[j] = 2.0 * S0[f][j] + S1[f][j];
        u1[j] = S0[f][j] + 2.0 * S1[f][j];
      }
      for (int k = 0; k < 3; ++k) {
        double cg = C[d][k] * gq;
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) {
            double T = S0[e][i] * u0[j] + S1[e][i] * u1[j];
            int64_t m[3];
            m[d] = base[d] + k;
            m[e] = base[e] + i;
            m[f] = base[f] + j;
            J[d * cells + idx3(&g, m[0], m[1], m[2])] += (int64_t)rint(cg * T);
          }
      }
    }
  }
  return status;
}

/* ======================================================================== */
/* Quasi-3D (r-z with azimuthal modes): field solver                         */
/* ======================================================================== */
/*
 * Fields are expanded in azimuthal modes F(z, r, th) = sum_m Re(F_m(z, r) e^{i m th});
 * each mode is a complex field on an r-z Yee grid, with z = x1 (the FFT
 * direction, periodic) and r = x2 (finite differences, axis at r = 0,
 * conducting wall at r = n2 dr).  Storage per mode: [6][n2+1][n1] complex,
 * components Ez, Er, Eth, Bz, Br, Bth (the Cartesian order with x1 = z,
 * x2 = r, x3 = th) on the staggered nodes Ez (z+1/2, r_j), Er (z, r_{j+1/2}),
 * Eth (z, r_j), Bz (z, r_{j+1/2}), Br (z+1/2, r_j), Bth (z+1/2, r_{j+1/2}),
 * r_j = j dr; half-r components use rows 0..n2-1.  The curls, with
 * d/dth -> i m:
 *   (curl E)_z  = (1/r) d_r(r Eth) - (i m / r) Er
 *   (curl E)_r  = (i m / r) Ez - d_z Eth
 *   (curl E)_th = d_z Er - d_r Ez
 * and the same for B; d_z is i k1 xi+- (the hybrid symbol, FD symbol for
 * deriv1 = 1), d_r the staggered difference, (1/r) d_r (r .) its volume form.
 * Axis rules (from the behaviour ~ r^|m| of the z components and ~ r^(|m|-1)
 * of the r, th components near r = 0): m = 0: Eth = Br = 0 on the axis and
 * (curl B)_z = 4 Bth(dr/2) / dr there (Stokes over the disc of radius dr/2);
 * m = 1: Ez = 0 on the axis, (i m / r) Ez -> i Ez(dr) / dr and
 * d_r Bz -> 2 Bz(dr/2) / dr; m >= 2: every component is zero on the axis.
 * Wall: Ez = Eth = 0 (and Br keeps its initial zero).
 */
static double complex *qf(const or_gridq *g, double complex *F, int m, int c) {
  return F + ((int64_t)m * 6 + c) * (int64_t)(g->n2 + 1) * g->n1;
}

/* x1 symbol for the complex (c2c) transform: kappa in [0, n1), signed k1 */
static xsym x1_symbols_q(const or_gridq *g, int32_t kappa) {
  or_grid2 g2;
  memset(&g2, 0, sizeof g2);
  int32_t ks = kappa <= g->n1 / 2 ? kappa : kappa - g->n1;
  g2.n1 = g->n1; g2.dx1 = g->dz; g2.dt = g->dt; g2.alpha = g->alpha;
  g2.deriv1 = g->deriv1; g2.correct = g->correct; g2.kmod = g->kmod;
  xsym s = x1_symbols(&g2, ks < 0 ? -ks : ks);
  if (ks < 0) {  /* symbols of -|k| are the conjugates: i(-k) e^{-i k dz/2} */
    s.dp = conj(s.dp);
    s.dm = conj(s.dm);
  }
  return s;
}

/* B -= h curl E for one mode in (kappa, r) space (h = dt/2). */
static void q_faraday(const or_gridq *g, int m, double complex *F, double h) {
  int32_t n1 = g->n1, n2 = g->n2;
  double dr = g->dr;
  double complex *Ez = qf(g, F, m, 0), *Er = qf(g, F, m, 1), *Et = qf(g, F, m, 2);
  double complex *Bz = qf(g, F, m, 3), *Br = qf(g, F, m, 4), *Bt = qf(g, F, m, 5);
  double complex im = I * (double)m;
  for (int32_t k = 0; k < n1; ++k) {
    xsym s = x1_symbols_q(g, k);
    for (int32_t j = 0; j < n2; ++j) {          /* half-r rows: Bz, Bth */
      int64_t c = (int64_t)j * n1 + k, u = (int64_t)(j + 1) * n1 + k;
      double rh = (j + 0.5) * dr;
      double complex cz = ((j + 1) * dr * Et[u] - j * dr * Et[c]) / (rh * dr) - im / rh * Er[c];
      double complex ct = s.dp * Er[c] - (Ez[u] - Ez[c]) / dr;
      Bz[c] -= h * cz;
      Bt[c] -= h * ct;
    }
    for (int32_t j = 0; j <= n2; ++j) {         /* integer-r rows: Br */
      int64_t c = (int64_t)j * n1 + k;
      double complex cr;
      if (j == n2) continue;                    /* wall: stays zero */
      if (j == 0) {
        if (m != 1) continue;                   /* zero on the axis */
        cr = I * Ez[(int64_t)n1 + k] / dr - s.dp * Et[c];
      } else {
        cr = im / (j * dr) * Ez[c] - s.dp * Et[c];
      }
      Br[c] -= h * cr;
    }
  }
}

/* E += dt (curl B - J) for one mode. */
static void q_ampere(const or_gridq *g, int m, double complex *F, const double complex *Jm) {
  int32_t n1 = g->n1, n2 = g->n2;
  double dr = g->dr, dt = g->dt;
  double complex *Ez = qf(g, F, m, 0), *Er = qf(g, F, m, 1), *Et = qf(g, F, m, 2);
  double complex *Bz = qf(g, F, m, 3), *Br = qf(g, F, m, 4), *Bt = qf(g, F, m, 5);
  int64_t plane = (int64_t)(n2 + 1) * n1;
  const double complex *Jz = Jm, *Jr = Jm + plane, *Jt = Jm + 2 * plane;
  double complex im = I * (double)m;
  for (int32_t k = 0; k < n1; ++k) {
    xsym s = x1_symbols_q(g, k);
    for (int32_t j = 0; j < n2; ++j) {          /* Er on half-r rows */
      int64_t c = (int64_t)j * n1 + k;
      double rh = (j + 0.5) * dr;
      Er[c] += dt * (im / rh * Bz[c] - s.dm * Bt[c] - Jr[c]);
    }
    for (int32_t j = 0; j < n2; ++j) {          /* Ez, Eth on integer rows; wall stays 0 */
      int64_t c = (int64_t)j * n1 + k, d = (int64_t)(j - 1) * n1 + k;
      if (j == 0) {
        if (m == 0) Ez[c] += dt * (4.0 * Bt[c] / dr - Jz[c]);
        if (m == 1) Et[c] += dt * (s.dm * Br[c] - 2.0 * Bz[c] / dr - Jt[c]);
        continue;
      }
      double rj = j * dr;
      double complex cz = ((j + 0.5) * dr * Bt[c] - (j - 0.5) * dr * Bt[d]) / (rj * dr) - im / rj * Br[c];
      double complex ct = s.dm * Br[c] - (Bz[c] - Bz[d]) / dr;
      Ez[c] += dt * (cz - Jz[c]);
      Et[c] += dt * (ct - Jt[c]);
    }
  }
}

/* Complex transform of every row of a mode's component along z. */
static void q_rows(const or_gridq *g, double complex *F, int32_t nrows, int sign) {
  int32_t n1 = g->n1;
  double *re = malloc(sizeof(double) * n1), *im = malloc(sizeof(double) * n1);
  for (int32_t r = 0; r < nrows; ++r) {
    double complex *row = F + (int64_t)r * n1;
    for (int32_t i = 0; i < n1; ++i) { re[i] = creal(row[i]); im[i] = cimag(row[i]); }
    or_fft(n1, re, im, sign);
    double sc = sign > 0 ? 1.0 / n1 : 1.0;
    for (int32_t i = 0; i < n1; ++i) row[i] = sc * (re[i] + I * im[i]);
  }
  free(re); free(im);
}

int or_field_update_q(const or_gridq *g, double *Ed, double *Bd, const double *Jd) {
  int32_t n1 = g->n1, n2 = g->n2, M = g->nmodes;
  if (!is_pow2(n1) || n1 < 2 || n2 < 2 || M < 1) return -1;
  int64_t plane = (int64_t)(n2 + 1) * n1;
  /* work array [m][6][rows][n1] with E and B of each mode */
  double complex *F = malloc(sizeof(double complex) * 6 * plane * M);
  double complex *Jk = malloc(sizeof(double complex) * 3 * plane);
  const double complex *E = (const double complex *)Ed, *B = (const double complex *)Bd,
                       *J = (const double complex *)Jd;
  for (int m = 0; m < M; ++m) {
    memcpy(qf(g, F, m, 0), E + (int64_t)m * 3 * plane, sizeof(double complex) * 3 * plane);
    memcpy(qf(g, F, m, 3), B + (int64_t)m * 3 * plane, sizeof(double complex) * 3 * plane);
    q_rows(g, qf(g, F, m, 0), 6 * (n2 + 1), -1);
    memcpy(Jk, J + (int64_t)m * 3 * plane, sizeof(double complex) * 3 * plane);
    q_rows(g, Jk, 3 * (n2 + 1), -1);
    for (int32_t k = 0; k < n1; ++k) {
      xsym s = x1_symbols_q(g, k);
      for (int32_t j = 0; j <= n2; ++j) {
        int64_t c = (int64_t)j * n1 + k;
        Jk[c] *= s.corr * s.filt;           /* Eq. (11) on jz, then the filter */
        Jk[plane + c] *= s.filt;
        Jk[2 * plane + c] *= s.filt;
      }
    }
    q_faraday(g, m, F, 0.5 * g->dt);
    q_ampere(g, m, F, Jk);
    q_faraday(g, m, F, 0.5 * g->dt);
    q_rows(g, qf(g, F, m, 0), 6 * (n2 + 1), +1);
    memcpy((double complex *)Ed + (int64_t)m * 3 * plane, qf(g, F, m, 0), sizeof(double complex) * 3 * plane);
    memcpy((double complex *)Bd + (int64_t)m * 3 * plane, qf(g, F, m, 3), sizeof(double complex) * 3 * plane);
  }
  free(F); free(Jk);
  return 0;
}

/* The same update directly in real space with Yee differences along z (no
 * transform, filter or correction): the reference for deriv1 = 1. */
int or_yee_update_q(const or_gridq *g, double *Ed, double *Bd, const double *Jd) {
  int32_t n1 = g->n1, n2 = g->n2, M = g->nmodes;
  int64_t plane = (int64_t)(n2 + 1) * n1;
  double dz = g->dz, dr = g->dr, dt = g->dt;
  for (int m = 0; m < M; ++m) {
    double complex *Ez = (double complex *)Ed + (int64_t)m * 3 * plane, *Er = Ez + plane, *Et = Ez + 2 * plane;
    double complex *Bz = (double complex *)Bd + (int64_t)m * 3 * plane, *Br = Bz + plane, *Bt = Bz + 2 * plane;
    const double complex *Jz = (const double complex *)Jd + (int64_t)m * 3 * plane, *Jr = Jz + plane, *Jt = Jz + 2 * plane;
    double complex im = I * (double)m;
    for (int half = 0; half < 3; ++half) {
      if (half == 1) {
        for (int32_t j = 0; j < n2; ++j)
          for (int32_t i = 0; i < n1; ++i) {
            int64_t c = (int64_t)j * n1 + i, w = (int64_t)j * n1 + wrapi(i - 1, n1);
            double rh = (j + 0.5) * dr;
            Er[c] += dt * (im / rh * Bz[c] - (Bt[c] - Bt[w]) / dz - Jr[c]);
          }
        for (int32_t j = 0; j < n2; ++j)
          for (int32_t i = 0; i < n1; ++i) {
            int64_t c = (int64_t)j * n1 + i, d = (int64_t)(j - 1) * n1 + i;
            int64_t w = (int64_t)j * n1 + wrapi(i - 1, n1);
            double complex dzBr = (Br[c] - Br[w]) / dz;
            if (j == 0) {
              if (m == 0) Ez[c] += dt * (4.0 * Bt[c] / dr - Jz[c]);
              if (m == 1) Et[c] += dt * (dzBr - 2.0 * Bz[c] / dr - Jt[c]);
              continue;
            }
            double rj = j * dr;
            Ez[c] += dt * (((j + 0.5) * dr * Bt[c] - (j - 0.5) * dr * Bt[d]) / (rj * dr) - im / rj * Br[c] - Jz[c]);
            Et[c] += dt * (dzBr - (Bz[c] - Bz[d]) / dr - Jt[c]);
          }
        continue;
      }
      double h = 0.5 * dt;
      for (int32_t j = 0; j < n2; ++j)
        for (int32_t i = 0; i < n1; ++i) {
          int64_t c = (int64_t)j * n1 + i, u = (int64_t)(j + 1) * n1 + i;
          int64_t e = (int64_t)j * n1 + wrapi(i + 1, n1);
          double rh = (j + 0.5) * dr;
          double complex cz = ((j + 1) * dr * Et[u] - j * dr * Et[c]) / (rh * dr) - im / rh * Er[c];
          double complex ct = (Er[e] - Er[c]) / dz - (Ez[u] - Ez[c]) / dr;
          Bz[c] -= h * cz;
          Bt[c] -= h * ct;
        }
      for (int32_t j = 0; j < n2; ++j)
        for (int32_t i = 0; i < n1; ++i) {
          int64_t c = (int64_t)j * n1 + i, e = (int64_t)j * n1 + wrapi(i + 1, n1);
          double complex cr;
          if (j == 0) {
            if (m != 1) continue;
            cr = I * Ez[(int64_t)n1 + i] / dr - (Et[e] - Et[c]) / dz;
          } else {
            cr = im / (j * dr) * Ez[c] - (Et[e] - Et[c]) / dz;
          }
          Br[c] -= h * cr;
        }
    }
  }
  return 0;
}

/* Gauss residual of each mode on the integer nodes (z_i, r_j), j = 0..n2-1:
 * D.E - f rho with D.E = (1/r) d_r(r Er) + (i m / r) Eth + d_z Ez in (kappa, r)
 * space; on the axis only m = 0 is defined (4 Er(dr/2)/dr + d_z Ez), other
 * modes get 0 there.  rho and R are [m][n2+1][n1] complex (row n2 of R is 0). */
int or_gauss_q(const or_gridq *g, const double *Ed, const double *rhod, double *Rd) {
  int32_t n1 = g->n1, n2 = g->n2, M = g->nmodes;
  int64_t plane = (int64_t)(n2 + 1) * n1;
  double complex *T = malloc(sizeof(double complex) * 4 * plane);
  double complex *R = (double complex *)Rd;
  for (int m = 0; m < M; ++m) {
    memcpy(T, (const double complex *)Ed + (int64_t)m * 3 * plane, sizeof(double complex) * 3 * plane);
    memcpy(T + 3 * plane, (const double complex *)rhod + (int64_t)m * plane, sizeof(double complex) * plane);
    q_rows(g, T, 4 * (n2 + 1), -1);
    double complex *Ez = T, *Er = T + plane, *Et = T + 2 * plane, *rh = T + 3 * plane;
    double complex *Rm = R + (int64_t)m * plane;
    for (int32_t k = 0; k < n1; ++k) {
      xsym s = x1_symbols_q(g, k);
      for (int32_t j = 0; j <= n2; ++j) {
        int64_t c = (int64_t)j * n1 + k, d = (int64_t)(j - 1) * n1 + k;
        double complex div = 0;
        if (j == n2) { Rm[c] = 0; continue; }
        if (j == 0) {
          if (m != 0) { Rm[c] = 0; continue; }
          div = 4.0 * Er[c] / g->dr + s.dm * Ez[c];
        } else {
          double rj = j * g->dr;
          div = ((j + 0.5) * Er[c] - (j - 0.5) * Er[d]) / (j * g->dr) + I * (double)m / rj * Et[c] +
                s.dm * Ez[c];
        }
        Rm[c] = div - s.filt * rh[c];
      }
    }
    q_rows(g, Rm, n2 + 1, +1);
  }
  free(T);
  return 0;
}

/* ======================================================================== */
/* Quasi-3D particles: gather from the modes, push, per-mode charge-        */
/* conserving deposit                                                        */
/* ======================================================================== */
/*
 * Particles carry Cartesian positions (z, x, y) and momenta (uz, ux, uy);
 * r = hypot(x, y) and the phase of mode m is P_m = e^{-i m th} =
 * ((x - i y) / r)^m (1 on the axis).  Node weights in (z, r) are the
 * quadratic B-spline products of the Cartesian code with z and r in cell
 * units, at the staggered node of each component (the r-z Yee nodes of the
 * field solver above).  A stencil row below the axis (row -1) is the mirror
 * point (|r|, th + pi) of row 1 (integer-r nodes) or row 0 (half-r nodes): a
 * scalar or z component of mode m there is (-1)^m times the mirror value, an
 * r or th component -(-1)^m times it.
 *
 * Gather: F_c = sum_m Re(F_{c,m}(z, r) e^{i m th}), then
 * (F_r, F_th) -> (F_x, F_y) by the rotation through th.
 *
 * Charge per node: rho_m = c_m q w P_m W / V_j, c_0 = 1 and c_m = 2 for m >= 1
 * (so that sum_m Re(rho_m e^{i m th}) is the particle's density), volumes
 * V_0 = pi (dr/2)^2 dz (the disc around the axis) and V_j = 2 pi j dr^2 dz.
 *
 * Current, charge-conserving per mode.  With W^0, W^1 the old and new node
 * weights and P^0, P^1 the old and new phases,
 *   W^1 P^1 - W^0 P^0 = (W^1 - W^0) (P^0 + P^1)/2 + (W^0 + W^1)/2 (P^1 - P^0):
 * the first term is split into fluxes through the z and r faces by the
 * Esirkepov decomposition in (z, r) index space (carrying the mean phase),
 * the second is an azimuthal flux Phi_th with i m dt Phi_th = -c_m q w
 * (W^0 + W^1)/2 (P^1 - P^0).  The ghost row folds onto its mirror with the
 * factor (-1)^m for node fluxes (z, th) and -(-1)^m for the flux through the
 * face at r = -dr/2 (it lands on the face at +dr/2), which keeps continuity
 * exact on the folded grid.  Densities: Jz = Phi_z / (A_j dt) with the face
 * areas A_0 = pi dr^2 / 4 and A_j = 2 pi j dr^2, Jr = Phi_r / (2 pi (j+1/2) dr
 * dz dt), Jth = Phi_th / (2 pi dr dz) (rows j >= 1), where the Phi_z, Phi_r
 * here are the flux charges (per step).  Then per mode
 *   rho^{n+1} - rho^n + dt [(Jz_i - Jz_{i-1})/dz
 *     + ((j+1/2) Jr_j - (j-1/2) Jr_{j-1}) / (j dr) + (i m / (j dr)) Jth_j] = 0
 * on the rows j >= 1 and, for m = 0, 4 Jr_0 / dr in place of the radial term
 * on the axis: the discrete divergence of the Gauss residual of the solver.
 * Where continuity fixes no azimuthal current (m = 0 everywhere, m = 1 on the
 * axis) Jth is the direct deposit c_m q w P W3 v_th / V_j with the
 * time-averaged weight W3 of the Cartesian out-of-plane current, the mean
 * phase, and v_th the azimuthal velocity at the mid point of the move; its
 * ghost row folds with -(-1)^m (the azimuthal direction reverses across the
 * axis).  m >= 2 on the axis: no azimuthal current (the fields are zero
 * there).
 *
 * Particles must stay at r < (n2 - 3) dr (no particle boundary at the wall);
 * the functions report -1 otherwise.
 */
static double q_rmax(const or_gridq *g) { return (g->n2 - 3) * g->dr; }

static double q_area(const or_gridq *g, int64_t j) {
  return j == 0 ? 0.25 * PI * g->dr * g->dr : 2.0 * PI * (double)j * g->dr * g->dr;
}

static double complex q_phase(double x, double y, int m) {
  double r = hypot(x, y);
  double complex u = r > 0.0 ? (x - I * y) / r : 1.0;
  double complex p = 1.0;
  for (int k = 0; k < m; ++k) p *= u;
  return p;
}

/* mode m of component Fc (one [n2+1][n1] plane) at node (a, b), b >= -1 */
static double complex q_node(const or_gridq *g, const double complex *Fc, int half_r, int vec,
                             int m, int64_t a, int64_t b) {
  double sign = 1.0;
  if (b < 0) {
    b = half_r ? -b - 1 : -b;
    sign = ((m & 1) ? -1.0 : 1.0) * (vec ? -1.0 : 1.0);
  }
  return sign * Fc[b * g->n1 + wrapi(a, g->n1)];
}

/* Fields F[nmodes][3][n2+1][n1] (E or B), component c with staggering s */
static double q_interp(const or_gridq *g, const double complex *F, int c, const double s[2],
                       double zeta, double rho, double x, double y) {
  int64_t plane = (int64_t)(g->n2 + 1) * g->n1;
  double e1 = zeta - s[0], e2 = rho - s[1];
  int64_t m1 = (int64_t)floor(e1 + 0.5), m2 = (int64_t)floor(e2 + 0.5);
  double acc = 0.0;
  for (int m = 0; m < g->nmodes; ++m) {
    const double complex *Fc = F + ((int64_t)m * 3 + c) * plane;
    double complex v = 0.0;
    for (int64_t b = m2 - 1; b <= m2 + 1; ++b) {
      double w2 = gather_w(g->interp, s[1], e2 - (double)b);
      for (int64_t a = m1 - 1; a <= m1 + 1; ++a)
        v += gather_w(g->interp, s[0], e1 - (double)a) * w2 *
             q_node(g, Fc, s[1] > 0.0, c != 0, m, a, b);
    }
    acc += creal(v * conj(q_phase(x, y, m)));
  }
  return acc;
}

int or_gather_q(const or_gridq *g, const double *Ed, const double *Bd, int64_t np,
                const double *z, const double *x, const double *y, double *Ep, double *Bp) {
  const double complex *E = (const double complex *)Ed, *B = (const double complex *)Bd;
  int status = 0;
  for (int64_t p = 0; p < np; ++p) {
    double r = hypot(x[p], y[p]);
    double fe[3] = {0, 0, 0}, fb[3] = {0, 0, 0};
    if (r < q_rmax(g)) {
      double zeta = z[p] / g->dz, rho = r / g->dr;
      for (int c = 0; c < 3; ++c) {
        fe[c] = q_interp(g, E, c, STAG_E[c], zeta, rho, x[p], y[p]);
        fb[c] = q_interp(g, B, c, STAG_B[c], zeta, rho, x[p], y[p]);
      }
    } else {
      status = -1;
    }
    double ct = r > 0.0 ? x[p] / r : 1.0, st = r > 0.0 ? y[p] / r : 0.0;
    Ep[p] = fe[0];
    Ep[np + p] = fe[1] * ct - fe[2] * st;
    Ep[2 * np + p] = fe[1] * st + fe[2] * ct;
    Bp[p] = fb[0];
    Bp[np + p] = fb[1] * ct - fb[2] * st;
    Bp[2 * np + p] = fb[1] * st + fb[2] * ct;
  }
  return status;
}

/* J[nmodes][3][n2+1][n1] complex (Jz, Jr, Jth) += the current of the moves
 * (za, xa, ya) -> (zb, xb, yb) (zb not wrapped) over one step dt. */
int or_deposit_q(const or_gridq *g, int64_t np, const double *za, const double *xa,
                 const double *ya, const double *zb, const double *xb, const double *yb,
                 const double *qw, double *Jd) {
  int64_t plane = (int64_t)(g->n2 + 1) * g->n1;
  double complex *J = (double complex *)Jd;
  double dz = g->dz, dr = g->dr, dt = g->dt;
  int status = 0;
  for (int64_t p = 0; p < np; ++p) {
    double ra = hypot(xa[p], ya[p]), rb = hypot(xb[p], yb[p]);
    double z0 = za[p] / dz, z1 = zb[p] / dz, r0 = ra / dr, r1 = rb / dr;
    if (fabs(z1 - z0) >= 1.0 || fabs(r1 - r0) >= 1.0 || !(ra < q_rmax(g)) || !(rb < q_rmax(g))) {
      status = -1;
      continue;
    }
    int64_t b1 = (int64_t)fmin(floor(z0 + 0.5), floor(z1 + 0.5)) - 1;
    int64_t b2 = (int64_t)fmin(floor(r0 + 0.5), floor(r1 + 0.5)) - 1;
    double S0z[4], S1z[4], S0r[4], S1r[4];
    for (int a = 0; a < 4; ++a) {
      S0z[a] = spline2(z0 - (double)(b1 + a));
      S1z[a] = spline2(z1 - (double)(b1 + a));
      S0r[a] = spline2(r0 - (double)(b2 + a));
      S1r[a] = spline2(r1 - (double)(b2 + a));
    }
    double xm = 0.5 * (xa[p] + xb[p]), ym = 0.5 * (ya[p] + yb[p]), rm = hypot(xm, ym);
    double vth = rm > 0.0 ? (xm * (yb[p] - ya[p]) - ym * (xb[p] - xa[p])) / (rm * dt) : 0.0;
    for (int m = 0; m < g->nmodes; ++m) {
      double cm = m == 0 ? 1.0 : 2.0, sm = (m & 1) ? -1.0 : 1.0;
      double complex P0 = q_phase(xa[p], ya[p], m), P1 = q_phase(xb[p], yb[p], m);
      double complex Pm = 0.5 * (P0 + P1);
      double complex *Jz = J + ((int64_t)m * 3 + 0) * plane;
      double complex *Jr = J + ((int64_t)m * 3 + 1) * plane;
      double complex *Jt = J + ((int64_t)m * 3 + 2) * plane;
      double complex q = -cm * qw[p] * Pm; /* charge carried by a unit Esirkepov weight */
      /* z faces: running sum along z of (S1z - S0z)(S0r + S1r)/2 */
      for (int b = 0; b < 4; ++b) {
        int64_t row = b2 + b;
        double f = 1.0;
        if (row < 0) { row = -row; f = sm; }
        double acc = 0.0;
        for (int a = 0; a < 4; ++a) {
          acc += (S1z[a] - S0z[a]) * 0.5 * (S0r[b] + S1r[b]);
          Jz[row * g->n1 + wrapi(b1 + a, g->n1)] += f * q * acc / (q_area(g, row) * dt);
        }
      }
      /* r faces: running sum along r of (S1r - S0r)(S0z + S1z)/2; face j is
       * at (j + 1/2) dr */
      for (int a = 0; a < 4; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 4; ++b) {
          acc += (S1r[b] - S0r[b]) * 0.5 * (S0z[a] + S1z[a]);
          int64_t face = b2 + b;
          double f = 1.0;
          if (face < 0) { face = 0; f = -sm; }
          Jr[face * g->n1 + wrapi(b1 + a, g->n1)] +=
              f * q * acc / (2.0 * PI * (face + 0.5) * dr * dz * dt);
        }
      }
      /* azimuthal current */
      for (int b = 0; b < 4; ++b) {
        int64_t row = b2 + b;
        int ghost = row < 0;
        if (ghost) row = -row;
        for (int a = 0; a < 4; ++a) {
          int64_t o = row * g->n1 + wrapi(b1 + a, g->n1);
          if (m == 0 || (m == 1 && row == 0)) {
            double W3 = S0z[a] * S0r[b] / 3.0 + S1z[a] * S0r[b] / 6.0 + S0z[a] * S1r[b] / 6.0 +
                        S1z[a] * S1r[b] / 3.0;
            double f = ghost ? -sm : 1.0;
            Jt[o] += f * cm * qw[p] * Pm * W3 * vth / (q_area(g, row) * dz);
          } else if (row > 0) {
            double Wb = 0.5 * (S0z[a] * S0r[b] + S1z[a] * S1r[b]);
            double f = ghost ? sm : 1.0;
            double complex phi = I * cm * qw[p] * Wb * (P1 - P0) / ((double)m * dt);
            Jt[o] += f * phi / (2.0 * PI * dr * dz);
          }
        }
      }
    }
  }
  return status;
}

/* rho[nmodes][n2+1][n1] complex += the charge density of the particles */
int or_rho_q(const or_gridq *g, int64_t np, const double *z, const double *x, const double *y,
             const double *qw, double *rhod) {
  int64_t plane = (int64_t)(g->n2 + 1) * g->n1;
  double complex *rho = (double complex *)rhod;
  int status = 0;
  for (int64_t p = 0; p < np; ++p) {
    double r = hypot(x[p], y[p]);
    if (!(r < q_rmax(g))) { status = -1; continue; }
    double zeta = z[p] / g->dz, rr = r / g->dr;
    int64_t m1 = (int64_t)floor(zeta + 0.5), m2 = (int64_t)floor(rr + 0.5);
    for (int m = 0; m < g->nmodes; ++m) {
      double cm = m == 0 ? 1.0 : 2.0, sm = (m & 1) ? -1.0 : 1.0;
      double complex P = q_phase(x[p], y[p], m);
      for (int64_t b = m2 - 1; b <= m2 + 1; ++b) {
        int64_t row = b < 0 ? -b : b;
        double f = b < 0 ? sm : 1.0;
        for (int64_t a = m1 - 1; a <= m1 + 1; ++a) {
          double W = spline2(zeta - (double)a) * spline2(rr - (double)b);
          rho[(int64_t)m * plane + row * g->n1 + wrapi(a, g->n1)] +=
              f * cm * qw[p] * P * W / (q_area(g, row) * g->dz);
        }
      }
    }
  }
  return status;
}

/* Co-drifting background current (m = 0, z component, one value per integer
 * row): minus the z-average of the particles' current, from their momenta
 * uz/gamma and radial weights, jbg[j] = -sum_p q w v_z S_r / (n1 dz A_j). */
int or_jbg_q(const or_gridq *g, int64_t np, const double *x, const double *y, const double *uz,
             const double *ux, const double *uy, const double *qw, double *jbg) {
  int status = 0;
  for (int64_t j = 0; j <= g->n2; ++j) jbg[j] = 0.0;
  for (int64_t p = 0; p < np; ++p) {
    double r = hypot(x[p], y[p]);
    if (!(r < q_rmax(g))) { status = -1; continue; }
    double gam = sqrt(1.0 + uz[p] * uz[p] + ux[p] * ux[p] + uy[p] * uy[p]);
    double rr = r / g->dr;
    int64_t m2 = (int64_t)floor(rr + 0.5);
    for (int64_t b = m2 - 1; b <= m2 + 1; ++b) {
      int64_t row = b < 0 ? -b : b;
      jbg[row] -= qw[p] * (uz[p] / gam) * spline2(rr - (double)b) /
                  ((double)g->n1 * g->dz * q_area(g, row));
    }
  }
  return status;
}

/* One quasi-3D step: gather, Boris, move, deposit (J: deposited current, jbg
 * (NULL: none) added to the m = 0 z current of each row), field update, z
 * wrapped into [0, n1 dz). */
int or_step_q(const or_gridq *g, double qm, int64_t np, double *z, double *x, double *y,
              double *uz, double *ux, double *uy, const double *qw, double *E, double *B,
              double *J, const double *jbg) {
  int64_t plane = (int64_t)(g->n2 + 1) * g->n1;
  int64_t n = np > 0 ? np : 1;
  double *Ep = malloc(sizeof(double) * 3 * n), *Bp = malloc(sizeof(double) * 3 * n);
  double *zn = malloc(sizeof(double) * n), *xn = malloc(sizeof(double) * n),
         *yn = malloc(sizeof(double) * n);
  int status = or_gather_q(g, E, B, np, z, x, y, Ep, Bp);
  or_boris(np, qm, g->dt, Ep, Bp, uz, ux, uy);
  for (int64_t p = 0; p < np; ++p) {
    double gam = sqrt(1.0 + uz[p] * uz[p] + ux[p] * ux[p] + uy[p] * uy[p]);
    zn[p] = z[p] + g->dt * uz[p] / gam;
    xn[p] = x[p] + g->dt * ux[p] / gam;
    yn[p] = y[p] + g->dt * uy[p] / gam;
  }
  memset(J, 0, sizeof(double complex) * 3 * plane * g->nmodes);
  if (or_deposit_q(g, np, z, x, y, zn, xn, yn, qw, J) != 0) status = -1;
  if (jbg) {
    double complex *Jz = (double complex *)J;
    for (int64_t j = 0; j <= g->n2; ++j)
      for (int64_t i = 0; i < g->n1; ++i) Jz[j * g->n1 + i] += jbg[j];
  }
  if (or_field_update_q(g, E, B, J) != 0) status = -1;
  double L = g->n1 * g->dz;
  for (int64_t p = 0; p < np; ++p) {
    z[p] = fmod(zn[p], L);
    if (z[p] < 0.0) z[p] += L;
    x[p] = xn[p];
    y[p] = yn[p];
  }
  free(Ep); free(Bp); free(zn); free(xn); free(yn);
  return status;
}
