// hpic_q3d.h -- device-side layout of the quasi-3D (r-z with azimuthal modes)
// runs: per-run descriptor, particle arrays and the launch interface of the
// quasi-3D kernels (solveq.hip, pushq.hip).
#pragma once
#include "hpic_internal.h"

namespace hp {

// ---------------------------------------------------------------- quasi-3D
// One quasi-3D run: azimuthal modes m = 0..M-1 of an r-z grid, z = x1 (n1
// points, FFT, periodic), r = x2 (n2 cells, nr = n2 + 1 rows, axis at j = 0,
// conducting wall at j = n2).  Per mode complex arrays [6][nr][n1] in the
// order Ez, Er, Eth, Bz, Br, Bth, staggered Ez (z+1/2, r_j), Er (z, r_j+1/2),
// Eth (z, r_j), Bz (z, r_j+1/2), Br (z+1/2, r_j), Bth (z+1/2, r_j+1/2).
// Quasi-3D particles: z as cell + offset in [0,1) (cells of dz), transverse
// Cartesian x, y likewise on a lattice of spacing dr (cell ix, iy, offsets fx,
// fy: the position keeps single-precision resolution within a cell anywhere in
// the column), momenta (uz, ux, uy), charge times weight qw.
template <class R>
struct PartsQ {
  int *cell, *ix, *iy;
  R *fz, *fx, *fy, *uz, *ux, *uy, *qw;
  int *id;
};
// Accumulator of the quasi-3D deposit: 64-bit fixed point in the FP32 form
// (order-independent), FP64 in the FP64 form.
template <class R> struct AccQ;
template <> struct AccQ<float> { using T = long long; };
template <> struct AccQ<double> { using T = double; };

template <class R>
struct RunQ {
  using C = typename Cplx<R>::T;
  using A = typename AccQ<R>::T;
  int n1, n2, nr, M, log2n1;
  int interp;        // 0 momentum-conserving gather, 1 energy-conserving
  long long plane;   // nr * n1
  double dz, dr, dt, hdt;
  double2 *Fk[2];    // [M][6][nr][n1] k-space master (FP64), ping-pong by step parity
  C *F;              // [M][6][nr][n1] real-space fields (complex)
  const C *tw;       // [n1]: exp(-2 pi i m / n1)
  const double *sym; // [n1][4]: i [k]1 xi+ (re, im), i [k]1 xi- (re, im), signed k1
  // particle side (np = 0: field solve only)
  PartsQ<R> pt;
  PartsQ<R> pt2;     // the other particle buffer: target of the periodic sort
  int *skey, *srank; // [np]: sort bin of each particle and its rank in the bin
  int *sbin;         // [nbins + 1]: bin counts, then their exclusive prefix sums
  int *ssum;         // [ceil(nbins / 1024) + 1]: per-block sums of the scan
  int sbz, sbr, nbr, nbins;  // bins of sbz z columns x sbr radial rows, nbr bins along r
  int np;
  R qmhdt, dtdz, dtdr, rmax;  // q/m dt/2, dt/dz, dt/dr, limit of r/dr
  R wscale;                       // contribution scale: inv_wunit cj (FP32), 1 (FP64)
  A *J[2];           // [M][3][nr][n1][2] deposit accumulators (re, im), by step parity
  C *Jk;             // [M][3][nr][n1] corrected, filtered current in k space
  const double *jconv;  // [M][3][nr] accumulator -> current density
  const R *kfac;        // [n1][2]: jz factor (correction x filter), filter
  const double *jbgk;   // [nr] n1 x co-drifting background current (m = 0, z)
  const double2 *tw64;  // [n1] FP64 twiddles (diagnostics)
  const double *filt64; // [n1] filter mask (diagnostics)
};
template <class R>
struct LaunchQ {
  // forward transform of the real-space fields into the master of a parity
  static void fields_to_k(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                          int maxn1, hipStream_t s);
  // the hybrid update of every mode, parity -> parity ^ 1 (two passes)
  static void kupdate(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                      hipStream_t s);
  // inverse transform of the master of a parity into the real-space fields
  static void ifft(const RunQ<R> *runs, const Item *items, int nitems, int parity, int maxn1,
                   hipStream_t s);
  // per (run, mode, row): sum |D.E - f rho|^2, max |D.E - f rho| and sum |f rho|^2
  // of the master (rho: [M][nr][n1] complex FP64 density of the run, replaced
  // by its transform along z; NULL for the vacuum law)
  static void gauss(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                    const double2 *rho, double *rows_out, int maxn1, hipStream_t s);
  // counting sort of a run's particles by (z column, radial row) bin into
  // pt2, then pt and pt2 swap places (in the device copy of the run; the
  // caller swaps its host copy)
  static void sort(RunQ<R> *run_dev, int np, int nbins, hipStream_t s);
  // gather, Boris, move and per-mode deposit into J[parity]; items (run,
  // first particle) of 256 particles; modes: the mode count of every run in
  // the launch, or 0 when they differ
  static void push_deposit(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                           int modes, unsigned *err, hipStream_t s);
  // per (run, 3 m + c, row): accumulator J[parity] -> complex current, forward
  // transform, correction and filter, background; clears J[parity ^ 1]
  static void fft_j(const RunQ<R> *runs, const Item *items, int nitems, int parity, int maxn1,
                    hipStream_t s);
  // FP64 charge density of the particles of one run added into rho [M][nr][n1]
  static void rho(const RunQ<R> *run_dev, int np, int M, double2 *rho, hipStream_t s);
  // FP64 co-drifting background current profile jbg[nr] (added into)
  static void jbg(const RunQ<R> *run_dev, int np, double *jbg, hipStream_t s);
};

}  // namespace hp
