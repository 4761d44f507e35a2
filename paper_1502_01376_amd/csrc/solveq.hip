// solveq.hip -- quasi-3D (r-z with azimuthal modes) hybrid field solver on
// gfx950 (Sec. 5: the hybrid update per azimuthal mode, FFT along z = x1 and
// differences along r = x2).
//
// Each mode is a complex field.  The k-space master (FP64) is advanced in
// (kappa1, r) space by two passes over (mode, r row, kappa1), every mode of
// every run in one launch per pass; complex transforms along z per (mode,
// component, row) move between the master and the real-space copy.  The per
// mode curls with d/dth -> i m:
//   (curl E)_z = (1/r) d_r(r Eth) - (i m/r) Er,  (curl E)_r = (i m/r) Ez - d_z Eth,
//   (curl E)_th = d_z Er - d_r Ez, the same for B;
// axis rules: m = 0: Eth = Br = 0 on the axis, (curl B)_z = 4 Bth(dr/2)/dr;
// m = 1: Ez = 0 on the axis, (i m/r) Ez -> i Ez(dr)/dr, d_r Bz -> 2 Bz(dr/2)/dr;
// m >= 2: zero on the axis.  Wall: Ez = Eth = 0, Br stays zero.
#include "hpic_q3d.h"

namespace hp {

// Item = (run, 6 m + component, row).
template <class R>
__global__ void __launch_bounds__(256) k_q_fields_to_k(const RunQ<R> *__restrict__ runs,
                                                       const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const long long base = (long long)it.a * r.plane + (long long)it.b * r.n1;
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) lds[n] = r.F[base + n];
  __syncthreads();
  lds_fft16<C, 6>(lds, r.n1, r.log2n1, 1, r.tw, 1, false);
  double2 *out = r.Fk[parity] + base;
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) out[n] = to_d2(lds[n]);
}

template <class R>
__global__ void __launch_bounds__(256) k_q_ifft(const RunQ<R> *__restrict__ runs,
                                                const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const long long base = (long long)it.a * r.plane + (long long)it.b * r.n1;
  const double2 *X = r.Fk[parity] + base;
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) lds[n] = from_d2<C>(X[n]);
  __syncthreads();
  lds_fft16<C, 6>(lds, r.n1, r.log2n1, 1, r.tw, 1, true);
  const R s = R(1) / (R)r.n1;
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) r.F[base + n] = cscale(lds[n], s);
}

// Current of the step per (run, 3 m + c, row): the deposit accumulators of a
// row -> current density (jconv: face area or node volume, dt and the
// fixed-point scale), the other parity's accumulators cleared, forward complex
// transform along z, the correction of Eq. (11) on jz and the low-pass filter
// (kfac); the co-drifting background (m = 0, z) is added before the transform.
template <class R>
__global__ void __launch_bounds__(256) k_q_fft_j(const RunQ<R> *__restrict__ runs,
                                                 const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  using A = typename AccQ<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const int mc = it.a, row = it.b, m = mc / 3, c = mc - 3 * m;
  const long long base = (long long)mc * r.plane + (long long)row * r.n1;
  const A *Jin = r.J[parity] + 2 * base;
  A *Jclr = r.J[parity ^ 1] + 2 * base;
  // conversion and the co-drifting background (mode 0, z) per node in FP64
  // before the transform: the background cancels the column's bulk current,
  // so that the FP32 transform (FP32 form) rounds relative to its fluctuation
  const double conv = r.jconv[mc * r.nr + row];
  const double bg = (m == 0 && c == 0) ? r.jbgk[row] / (double)r.n1 : 0.0;
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) {
    lds[n] = cmk((R)((double)Jin[2 * n] * conv + bg), (R)((double)Jin[2 * n + 1] * conv));
    Jclr[2 * n] = 0;
    Jclr[2 * n + 1] = 0;
  }
  __syncthreads();
  lds_fft16<C, 6>(lds, r.n1, r.log2n1, 1, r.tw, 1, false);
  C *out = r.Jk + base;
  const int sel = c == 0 ? 0 : 1;
  for (int k = threadIdx.x; k < r.n1; k += blockDim.x) {
    C v = cscale(lds[k], r.kfac[2 * k + sel]);
    out[k] = v;
  }
}

// Item = (run, first element, 0): elements e = (m nr + j) n1 + kappa.
template <class R>
__global__ void __launch_bounds__(256) k_q_update_a(const RunQ<R> *__restrict__ runs,
                                                    const Item *__restrict__ items, int parity) {
  using C = double2;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const int n1 = r.n1, n2 = r.n2, nr = r.nr;
  const long long e = (long long)it.a + threadIdx.x;
  if (e >= (long long)r.M * nr * n1) return;
  const int k = (int)(e % n1);
  const long long mj = e / n1;
  const int j = (int)(mj % nr), m = (int)(mj / nr);
  const C *Fi = r.Fk[parity] + (long long)m * 6 * r.plane;
  C *Fo = r.Fk[parity ^ 1] + (long long)m * 6 * r.plane;
  auto at = [&](int comp, int row) { return Fi[comp * r.plane + (long long)row * n1 + k]; };
  const C dp = cmk(r.sym[4 * k + 0], r.sym[4 * k + 1]);
  const C dm = cmk(r.sym[4 * k + 2], r.sym[4 * k + 3]);
  const double dr = r.dr, h = r.hdt, dt = r.dt, mm = (double)m;
  const C im = cmk(0.0, mm);
  // half-step B on a half row q (Bz, Bth) from E on rows q, q+1
  auto bh_half = [&](int q, C &bz, C &bt) {
    const double rh = (q + 0.5) * dr;
    const C Et0 = at(2, q), Et1 = at(2, q + 1), Er0 = at(1, q), Ez0 = at(0, q), Ez1 = at(0, q + 1);
    const C cz = csub(cscale(csub(cscale(Et1, (q + 1) * dr), cscale(Et0, q * dr)), 1.0 / (rh * dr)),
                      cscale(cmul(im, Er0), 1.0 / rh));
    const C ct = csub(cmul(dp, Er0), cscale(csub(Ez1, Ez0), 1.0 / dr));
    bz = csub(at(3, q), cscale(cz, h));
    bt = csub(at(5, q), cscale(ct, h));
  };
  // half-step Br on the integer row q
  auto bh_r = [&](int q) {
    C cr = cmk(0.0, 0.0);
    if (q == n2) return at(4, q);
    if (q == 0) {
      if (m != 1) return at(4, q);
      cr = csub(cscale(cmk(-at(0, 1).y, at(0, 1).x), 1.0 / dr), cmul(dp, at(2, 0)));
    } else {
      cr = csub(cscale(cmul(im, at(0, q)), 1.0 / (q * dr)), cmul(dp, at(2, q)));
    }
    return csub(at(4, q), cscale(cr, h));
  };
  const long long o = (long long)j * n1 + k;
  const C Br_j = bh_r(j);
  C Bz_j = at(3, j), Bt_j = at(5, j);
  if (j < n2) bh_half(j, Bz_j, Bt_j);
  // E^{n+1}
  C Ez = at(0, j), Er = at(1, j), Et = at(2, j);
  if (j < n2) {
    const double rh = (j + 0.5) * dr;
    // current of the step (zero for a field-only run)
    const typename RunQ<R>::C *Jm = r.Jk + (long long)m * 3 * r.plane;
    const C Jz = to_d2(Jm[o]), Jr = to_d2(Jm[r.plane + o]), Jt = to_d2(Jm[2 * r.plane + o]);
    Er = cadd(Er, cscale(csub(csub(cscale(cmul(im, Bz_j), 1.0 / rh), cmul(dm, Bt_j)), Jr), dt));
    if (j == 0) {
      if (m == 0) Ez = cadd(Ez, cscale(csub(cscale(Bt_j, 4.0 / dr), Jz), dt));
      if (m == 1) Et = cadd(Et, cscale(csub(csub(cmul(dm, Br_j), cscale(Bz_j, 2.0 / dr)), Jt), dt));
    } else {
      C Bz_m, Bt_m;
      bh_half(j - 1, Bz_m, Bt_m);
      const double rj = j * dr;
      const C cz = csub(cscale(csub(cscale(Bt_j, (j + 0.5) * dr), cscale(Bt_m, (j - 0.5) * dr)),
                               1.0 / (rj * dr)),
                        cscale(cmul(im, Br_j), 1.0 / rj));
      const C ct = csub(cmul(dm, Br_j), cscale(csub(Bz_j, Bz_m), 1.0 / dr));
      Ez = cadd(Ez, cscale(csub(cz, Jz), dt));
      Et = cadd(Et, cscale(csub(ct, Jt), dt));
    }
  }
  Fo[o] = Ez;
  Fo[r.plane + o] = Er;
  Fo[2 * r.plane + o] = Et;
  Fo[3 * r.plane + o] = Bz_j;
  Fo[4 * r.plane + o] = Br_j;
  Fo[5 * r.plane + o] = Bt_j;
}

// B^{n+1} = B^{n+1/2} - (dt/2) curl E^{n+1}, in the output master.
template <class R>
__global__ void __launch_bounds__(256) k_q_update_b(const RunQ<R> *__restrict__ runs,
                                                    const Item *__restrict__ items, int parity) {
  using C = double2;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const int n1 = r.n1, n2 = r.n2, nr = r.nr;
  const long long e = (long long)it.a + threadIdx.x;
  if (e >= (long long)r.M * nr * n1) return;
  const int k = (int)(e % n1);
  const long long mj = e / n1;
  const int j = (int)(mj % nr), m = (int)(mj / nr);
  C *F = r.Fk[parity ^ 1] + (long long)m * 6 * r.plane;
  auto at = [&](int comp, int row) { return F[comp * r.plane + (long long)row * n1 + k]; };
  const C dp = cmk(r.sym[4 * k + 0], r.sym[4 * k + 1]);
  const double dr = r.dr, h = r.hdt, mm = (double)m;
  const C im = cmk(0.0, mm);
  const long long o = (long long)j * n1 + k;
  if (j < n2) {
    const double rh = (j + 0.5) * dr;
    const C Et0 = at(2, j), Et1 = at(2, j + 1), Er0 = at(1, j), Ez0 = at(0, j), Ez1 = at(0, j + 1);
    const C cz = csub(cscale(csub(cscale(Et1, (j + 1) * dr), cscale(Et0, j * dr)), 1.0 / (rh * dr)),
                      cscale(cmul(im, Er0), 1.0 / rh));
    const C ct = csub(cmul(dp, Er0), cscale(csub(Ez1, Ez0), 1.0 / dr));
    F[3 * r.plane + o] = csub(at(3, j), cscale(cz, h));
    F[5 * r.plane + o] = csub(at(5, j), cscale(ct, h));
  }
  if (j < n2 && (j > 0 || m == 1)) {
    C cr;
    if (j == 0)
      cr = csub(cscale(cmk(-at(0, 1).y, at(0, 1).x), 1.0 / dr), cmul(dp, at(2, 0)));
    else
      cr = csub(cscale(cmul(im, at(0, j)), 1.0 / (j * dr)), cmul(dp, at(2, j)));
    F[4 * r.plane + o] = csub(at(4, j), cscale(cr, h));
  }
}

// Forward FP64 transform along z of one row (m, j) of a density, in place.
template <class R>
__global__ void __launch_bounds__(256) k_q_rho_fft(const RunQ<R> *__restrict__ runs,
                                                   const Item *__restrict__ items, double2 *rho) {
  extern __shared__ unsigned char smem_raw[];
  double2 *lds = (double2 *)smem_raw;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  double2 *row = rho + (long long)it.a * r.plane + (long long)it.b * r.n1;
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) lds[n] = row[n];
  __syncthreads();
  lds_fft16<double2, 6>(lds, r.n1, r.log2n1, 1, r.tw64, 1, false);
  for (int n = threadIdx.x; n < r.n1; n += blockDim.x) row[n] = lds[n];
}

// Gauss law per (run, m, row): D.E on the integer nodes from the master, rows
// 1..n2-1 and the axis for m = 0, minus the filtered charge density
// f(k1) rho^ (rho: the run's FP64 density [M][nr][n1] already transformed
// along z; NULL: the vacuum law).  rows_out[item][3] = sum |res|^2, max |res|,
// sum |f rho^|^2.
template <class R>
__global__ void __launch_bounds__(256) k_q_gauss(const RunQ<R> *__restrict__ runs,
                                                 const Item *__restrict__ items, int parity,
                                                 const double2 *__restrict__ rho,
                                                 double *rows_out) {
  __shared__ double red[256][3];
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const int m = it.a, j = it.b, n1 = r.n1;
  const double2 *F = r.Fk[parity] + (long long)m * 6 * r.plane;
  const double2 *rk = rho ? rho + (long long)m * r.plane + (long long)j * n1 : nullptr;
  double s2 = 0, smax = 0, sref = 0;
  const bool on = (j > 0 && j < r.n2) || (j == 0 && m == 0);
  for (int k = threadIdx.x; on && k < n1; k += blockDim.x) {
    const double2 dm = make_double2(r.sym[4 * k + 2], r.sym[4 * k + 3]);
    const double2 Ez = F[(long long)j * n1 + k];
    double2 div = cmul(dm, Ez);
    if (j == 0) {
      const double2 Er = F[r.plane + k];
      div.x += 4.0 * Er.x / r.dr;
      div.y += 4.0 * Er.y / r.dr;
    } else {
      const double2 Er = F[r.plane + (long long)j * n1 + k], Erm = F[r.plane + (long long)(j - 1) * n1 + k];
      const double2 Et = F[2 * r.plane + (long long)j * n1 + k];
      const double rj = j * r.dr;
      div.x += ((j + 0.5) * Er.x - (j - 0.5) * Erm.x) / (j * r.dr) - m / rj * Et.y;
      div.y += ((j + 0.5) * Er.y - (j - 0.5) * Erm.y) / (j * r.dr) + m / rj * Et.x;
    }
    if (rk) {
      const double f = r.filt64[k];
      const double2 q = rk[k];
      div.x -= f * q.x;
      div.y -= f * q.y;
      sref += f * f * (q.x * q.x + q.y * q.y);
    }
    const double a2 = div.x * div.x + div.y * div.y;
    s2 += a2;
    smax = fmax(smax, sqrt(a2));
  }
  red[threadIdx.x][0] = s2;
  red[threadIdx.x][1] = smax;
  red[threadIdx.x][2] = sref;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x][0] += red[threadIdx.x + w][0];
      red[threadIdx.x][1] = fmax(red[threadIdx.x][1], red[threadIdx.x + w][1]);
      red[threadIdx.x][2] += red[threadIdx.x + w][2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rows_out[3 * blockIdx.x] = red[0][0];
    rows_out[3 * blockIdx.x + 1] = red[0][1];
    rows_out[3 * blockIdx.x + 2] = red[0][2];
  }
}

template <class R>
void LaunchQ<R>::fields_to_k(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                             int maxn1, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_q_fields_to_k<R>, dim3(nitems), dim3(256),
                     (size_t)maxn1 * sizeof(typename Cplx<R>::T), s, runs, items, parity);
}
template <class R>
void LaunchQ<R>::ifft(const RunQ<R> *runs, const Item *items, int nitems, int parity, int maxn1,
                      hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_q_ifft<R>, dim3(nitems), dim3(256),
                     (size_t)maxn1 * sizeof(typename Cplx<R>::T), s, runs, items, parity);
}
template <class R>
void LaunchQ<R>::kupdate(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                         hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_q_update_a<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity);
  hipLaunchKernelGGL(k_q_update_b<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity);
}
template <class R>
void LaunchQ<R>::gauss(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                       const double2 *rho, double *rows_out, int maxn1, hipStream_t s) {
  if (nitems <= 0) return;
  if (rho)
    hipLaunchKernelGGL(k_q_rho_fft<R>, dim3(nitems), dim3(256), (size_t)maxn1 * sizeof(double2), s,
                       runs, items, const_cast<double2 *>(rho));
  hipLaunchKernelGGL(k_q_gauss<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity, rho,
                     rows_out);
}
template <class R>
void LaunchQ<R>::fft_j(const RunQ<R> *runs, const Item *items, int nitems, int parity, int maxn1,
                       hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_q_fft_j<R>, dim3(nitems), dim3(256),
                     (size_t)maxn1 * sizeof(typename Cplx<R>::T), s, runs, items, parity);
}
template struct LaunchQ<float>;
template struct LaunchQ<double>;

}  // namespace hp
