// kernels.hip -- HIP kernels (gfx950) of the hybrid Yee-FFT PIC step.
//
// Step order (Sec. 2.1): push_deposit (gather + Boris + move + charge-
// conserving deposit), fft_j (FFT of j along x1, current correction of
// Eq. (11) and the low-pass filter of Sec. 4), kupdate (hybrid Maxwell update
// of Eqs. (12)-(17) in (k1, x2) space), ifft_eb (inverse FFT of E and B for
// the next gather).  Every launch is batched over all runs of a handle through
// a work-item list.
#include "hpic_internal.h"

namespace hp {

// =====================================================================
// push + deposit
// =====================================================================

// Momentum-conserving quadratic gather of the six Yee components at a particle
// in cell (i1, i2) with offsets (f1, f2), Appendix A first variant: each
// component uses the quadratic B-spline around its own staggered node.
template <class R>
__device__ __forceinline__ void gather2(const Run<R> &r, int i1, int i2, R f1, R f2, R Ef[3],
                                        R Bf[3]) {
  const int n1 = r.n1, n2 = r.n2, cells = n1 * n2;
  const int up1 = f1 >= R(0.5), up2 = f2 >= R(0.5);
  R wi1[3], wh1[3], wi2[3], wh2[3];
  spline3<R>(f1 - R(up1), wi1);   // integer nodes along x1
  spline3<R>(f1 - R(0.5), wh1);   // half nodes along x1
  spline3<R>(f2 - R(up2), wi2);
  spline3<R>(f2 - R(0.5), wh2);
  int ci[3], ch[3], ri[3], rh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ci[a] = wrap_pow2(i1 + up1 - 1 + a, n1);
    ch[a] = wrap_pow2(i1 - 1 + a, n1);
    ri[a] = wrap_small(i2 + up2 - 1 + a, n2) * n1;
    rh[a] = wrap_small(i2 - 1 + a, n2) * n1;
  }
  const R *F = r.F;
  R e1 = 0, e2 = 0, e3 = 0, b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    R s_e1 = 0, s_e2 = 0, s_e3 = 0, s_b1 = 0, s_b2 = 0, s_b3 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s_e1 += wh1[a] * F[0 * cells + ri[b] + ch[a]];   // E1 (i1+1/2, i2)
      s_e2 += wi1[a] * F[1 * cells + rh[b] + ci[a]];   // E2 (i1, i2+1/2)
      s_e3 += wi1[a] * F[2 * cells + ri[b] + ci[a]];   // E3 (i1, i2)
      s_b1 += wi1[a] * F[3 * cells + rh[b] + ci[a]];   // B1 (i1, i2+1/2)
      s_b2 += wh1[a] * F[4 * cells + ri[b] + ch[a]];   // B2 (i1+1/2, i2)
      s_b3 += wh1[a] * F[5 * cells + rh[b] + ch[a]];   // B3 (i1+1/2, i2+1/2)
    }
    e1 += wi2[b] * s_e1;
    e2 += wh2[b] * s_e2;
    e3 += wi2[b] * s_e3;
    b1 += wh2[b] * s_b1;
    b2 += wi2[b] * s_b2;
    b3 += wh2[b] * s_b3;
  }
  Ef[0] = e1; Ef[1] = e2; Ef[2] = e3;
  Bf[0] = b1; Bf[1] = b2; Bf[2] = b3;
}

// Relativistic Boris rotation: u^{n-1/2} -> u^{n+1/2} with E^n, B^n.
template <class R>
__device__ __forceinline__ void boris(R qmhdt, const R E[3], const R B[3], R u[3]) {
  const R e0 = qmhdt * E[0], e1 = qmhdt * E[1], e2 = qmhdt * E[2];
  const R m0 = u[0] + e0, m1 = u[1] + e1, m2 = u[2] + e2;
  const R ig = R(1) / sqrt(R(1) + m0 * m0 + m1 * m1 + m2 * m2);
  const R t0 = qmhdt * B[0] * ig, t1 = qmhdt * B[1] * ig, t2 = qmhdt * B[2] * ig;
  const R sf = R(2) / (R(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const R s0 = t0 * sf, s1 = t1 * sf, s2 = t2 * sf;
  const R p0 = m0 + (m1 * t2 - m2 * t1);
  const R p1 = m1 + (m2 * t0 - m0 * t2);
  const R p2 = m2 + (m0 * t1 - m1 * t0);
  u[0] = m0 + (p1 * s2 - p2 * s1) + e0;
  u[1] = m1 + (p2 * s0 - p0 * s2) + e1;
  u[2] = m2 + (p0 * s1 - p1 * s0) + e2;
}

// Velocity from momentum, every operation rounded once in this order (the
// out-of-plane velocity enters the fixed-point deposit, which tests reproduce
// bit for bit on the host).
template <class R>
__device__ __forceinline__ void velocity(const R u[3], R v[3]) {
#pragma clang fp contract(off)
  R s = R(1) + u[0] * u[0];
  s = s + u[1] * u[1];
  s = s + u[2] * u[2];
  const R g = sqrt(s);
  v[0] = u[0] / g;
  v[1] = u[1] / g;
  v[2] = u[2] / g;
}

// New offset in [0,1) and cell shift in {-1, 0, 1} after a move d (|d| < 1).
template <class R>
__device__ __forceinline__ int advance(R f, R d, R &g) {
  g = f + d;
  int s = 0;
  if (g >= R(1)) {
    g = g - R(1);  // exact for g in [1, 2)
    s = 1;
  } else if (g < R(0)) {
    g = g + R(1);
    s = -1;
    if (g >= R(1)) {  // rounded up to 1: the position is the next cell edge
      g = R(0);
      s = 0;
    }
  }
  return s;
}

// Place the three stencil values s[] of nearest node m in a 4-node window
// starting at base (offset m - 1 - base in {0, 1}) without dynamic indexing.
template <class T>
__device__ __forceinline__ void place4(const T s[3], int off, T out[4]) {
  out[0] = off ? T(0) : s[0];
  out[1] = off ? s[0] : s[1];
  out[2] = off ? s[1] : s[2];
  out[3] = off ? s[2] : T(0);
}

// Fixed-point Esirkepov deposit of one particle (2D).  Integer shapes with
// exact sum 2^P make 2 (rho_new - rho_old) = div J hold exactly in the
// integers; j3 is FP32 rounded once per node.  The arithmetic is the one of the
// FP32-precision reference deposit, operation for operation.
__device__ __forceinline__ void deposit2_fixed(long long *J, int n1, int n2, int P,
                                               float inv_wunit, float c3, int i1, int i2,
                                               float fa1, float fa2, int d1, int d2, float fb1,
                                               float fb2, float v3, float qw) {
#pragma clang fp contract(off)
  const int cells = n1 * n2;
  int sa1[3], sb1[3], sa2[3], sb2[3];
  const int na1 = fixed_shape(i1, fa1, P, sa1);
  const int nb1 = fixed_shape(i1 + d1, fb1, P, sb1);
  const int na2 = fixed_shape(i2, fa2, P, sa2);
  const int nb2 = fixed_shape(i2 + d2, fb2, P, sb2);
  const int base1 = min(na1, nb1) - 1, base2 = min(na2, nb2) - 1;
  int S0x[4], S1x[4], S0y[4], S1y[4];
  place4(sa1, na1 - 1 - base1, S0x);
  place4(sb1, nb1 - 1 - base1, S1x);
  place4(sa2, na2 - 1 - base2, S0y);
  place4(sb2, nb2 - 1 - base2, S1y);
  const float qs = qw * inv_wunit;
  const long long Q = (long long)rintf(qs);
  int C1[4], C2[4], A1[4], A2[4];
  int acc1 = 0, acc2 = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    acc1 += S1x[a] - S0x[a];
    acc2 += S1y[a] - S0y[a];
    C1[a] = acc1;
    C2[a] = acc2;
    A1[a] = S0x[a] + S1x[a];
    A2[a] = S0y[a] + S1y[a];
  }
  int col[4], row[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    col[a] = wrap_pow2(base1 + a, n1);
    row[a] = wrap_small(base2 + a, n2) * n1;
  }
  unsigned long long *J1 = (unsigned long long *)J;
  unsigned long long *J2 = J1 + cells, *J3 = J1 + 2 * cells;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const long long qc = Q * (long long)C1[a];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long v = qc * (long long)A2[b];
      if (v != 0) atomicAdd(J1 + row[b] + col[a], (unsigned long long)v);
    }
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const long long qc = Q * (long long)C2[b];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const long long v = qc * (long long)A1[a];
      if (v != 0) atomicAdd(J2 + row[b] + col[a], (unsigned long long)v);
    }
  }
  const float hv = qs * v3;
  const float h = hv * c3;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const float B0 = (float)S0y[b], B1 = (float)S1y[b];
    const float t0 = 2.0f * B0 + B1;
    const float t1 = B0 + 2.0f * B1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const float p0 = (float)S0x[a] * t0;
      const float p1 = (float)S1x[a] * t1;
      const float T = p0 + p1;
      const float v = T * h;
      const long long iv = (long long)rintf(v);
      if (iv != 0) atomicAdd(J3 + row[b] + col[a], (unsigned long long)iv);
    }
  }
}

// FP64 Esirkepov deposit of one particle (2D) with FP64 atomics.
__device__ __forceinline__ void deposit2_fp64(double *J, int n1, int n2, double jfx1,
                                              double jfx2, int i1, int i2, double fa1,
                                              double fa2, int d1, int d2, double fb1,
                                              double fb2, double v3, double qw) {
  const int cells = n1 * n2;
  double sa1[3], sb1[3], sa2[3], sb2[3];
  const int ua1 = fa1 >= 0.5, ub1 = fb1 >= 0.5, ua2 = fa2 >= 0.5, ub2 = fb2 >= 0.5;
  spline3<double>(fa1 - ua1, sa1);
  spline3<double>(fb1 - ub1, sb1);
  spline3<double>(fa2 - ua2, sa2);
  spline3<double>(fb2 - ub2, sb2);
  const int na1 = i1 + ua1, nb1 = i1 + d1 + ub1, na2 = i2 + ua2, nb2 = i2 + d2 + ub2;
  const int base1 = min(na1, nb1) - 1, base2 = min(na2, nb2) - 1;
  double S0x[4], S1x[4], S0y[4], S1y[4];
  place4(sa1, na1 - 1 - base1, S0x);
  place4(sb1, nb1 - 1 - base1, S1x);
  place4(sa2, na2 - 1 - base2, S0y);
  place4(sb2, nb2 - 1 - base2, S1y);
  int col[4], row[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    col[a] = wrap_pow2(base1 + a, n1);
    row[a] = wrap_small(base2 + a, n2) * n1;
  }
  double *J1 = J, *J2 = J + cells, *J3 = J + 2 * cells;
  const double f1 = qw * jfx1, f2 = qw * jfx2;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc += f1 * (S1x[a] - S0x[a]) * 0.5 * (S0y[b] + S1y[b]);
      if (acc != 0.0) unsafeAtomicAdd(J1 + row[b] + col[a], acc);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      acc += f2 * (S1y[b] - S0y[b]) * 0.5 * (S0x[a] + S1x[a]);
      if (acc != 0.0) unsafeAtomicAdd(J2 + row[b] + col[a], acc);
    }
  }
  const double g3 = qw * v3;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double W3 = S0x[a] * S0y[b] * (1.0 / 3.0) + S1x[a] * S0y[b] * (1.0 / 6.0) +
                        S0x[a] * S1y[b] * (1.0 / 6.0) + S1x[a] * S1y[b] * (1.0 / 3.0);
      const double v = g3 * W3;
      if (v != 0.0) unsafeAtomicAdd(J3 + row[b] + col[a], v);
    }
  }
}

__device__ __forceinline__ void deposit_one(const Run<float> &r, long long *J, int i1, int i2,
                                            float fa1, float fa2, int d1, int d2, float fb1,
                                            float fb2, float v3, float qw) {
  deposit2_fixed(J, r.n1, r.n2, r.P, r.inv_wunit, r.c3, i1, i2, fa1, fa2, d1, d2, fb1, fb2, v3,
                 qw);
}
__device__ __forceinline__ void deposit_one(const Run<double> &r, double *J, int i1, int i2,
                                            double fa1, double fa2, int d1, int d2, double fb1,
                                            double fb2, double v3, double qw) {
  deposit2_fp64(J, r.n1, r.n2, r.jfx1, r.jfx2, i1, i2, fa1, fa2, d1, d2, fb1, fb2, v3, qw);
}

template <class R>
__device__ __forceinline__ bool finite3(R a, R b, R c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// One thread per particle; item = (run, first particle, count).
template <class R>
__global__ void __launch_bounds__(256) k_push_deposit(const Run<R> *__restrict__ runs,
                                                      const Item *__restrict__ items, int parity,
                                                      unsigned *err) {
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int end = it.a + it.b;
  typename AccOf<R>::T *J = r.J[parity];
  for (int p = it.a + (int)threadIdx.x; p < end; p += blockDim.x) {
    const int cell = r.cell[p];
    const int i1 = cell & (r.n1 - 1), i2 = cell >> r.log2n1;
    const R f1 = r.f1[p], f2 = r.f2[p];
    R u[3] = {r.u1[p], r.u2[p], r.u3[p]};
    R Ef[3], Bf[3];
    gather2<R>(r, i1, i2, f1, f2, Ef, Bf);
    boris<R>(r.qmhdt, Ef, Bf, u);
    R v[3];
    velocity<R>(u, v);
    const R m1 = r.dtdx1 * v[0], m2 = r.dtdx2 * v[1];
    if (!finite3(u[0], u[1], u[2]) || !isfinite(m1) || !isfinite(m2)) {
      atomicOr(err, ERR_NUMERIC);
      continue;
    }
    if (!(fabs(m1) < R(1)) || !(fabs(m2) < R(1))) {
      atomicOr(err, ERR_RANGE);
      continue;
    }
    R g1, g2;
    const int d1 = advance<R>(f1, m1, g1);
    const int d2 = advance<R>(f2, m2, g2);
    deposit_one(r, J, i1, i2, f1, f2, d1, d2, g1, g2, v[2], r.qw[p]);
    const int j1 = wrap_pow2(i1 + d1, r.n1), j2 = wrap_small(i2 + d2, r.n2);
    r.cell[p] = (j2 << r.log2n1) | j1;
    r.f1[p] = g1;
    r.f2[p] = g2;
    r.u1[p] = u[0];
    r.u2[p] = u[1];
    r.u3[p] = u[2];
  }
}

// Deposit alone on given moves (tests of the fixed-point deposit).
__global__ void k_debug_deposit(int n1, int n2, int P, float inv_wunit, float c3, int np,
                                const int *cell0, const float *off0, const int *cell1,
                                const float *off1, const float *v3, const float *qw,
                                long long *J, unsigned *err) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int a1 = cell0[p], a2 = cell0[np + p], b1 = cell1[p], b2 = cell1[np + p];
  int d1 = (b1 - a1) & (n1 - 1);
  d1 = d1 > n1 / 2 ? d1 - n1 : d1;
  int d2 = wrap_small(b2 - a2, n2);
  d2 = d2 > n2 / 2 ? d2 - n2 : d2;
  if (d1 < -1 || d1 > 1 || d2 < -1 || d2 > 1 || a1 < 0 || a1 >= n1 || a2 < 0 || a2 >= n2) {
    atomicOr(err, ERR_RANGE);
    return;
  }
  deposit2_fixed(J, n1, n2, P, inv_wunit, c3, a1, a2, off0[p], off0[np + p], d1, d2, off1[p],
                 off1[np + p], v3[p], qw[p]);
}

// =====================================================================
// FFT of the current along x1, correction and filter
// =====================================================================

template <class R> __device__ __forceinline__ R to_real(long long v) { return (R)v; }
template <class R> __device__ __forceinline__ R to_real(double v) { return (R)v; }

// X[k] for k = 0..M of a length-2M real row from Z = FFT_M(z), z[n] = x[2n] + i x[2n+1]:
// X[k] = (Z[k] + conj Z[M-k])/2 - i W^k (Z[k] - conj Z[M-k])/2, W = exp(-i pi / M).
template <class C>
__device__ __forceinline__ C r2c_post(C Zk, C Zmk, C Wk) {
  const C e = cadd(Zk, cconj(Zmk));
  const C o = csub(Zk, cconj(Zmk));
  const C t = cmul(Wk, o);
  using R = decltype(e.x);
  // (e - i t)/2
  return cmk(R(0.5) * (e.x + t.y), R(0.5) * (e.y - t.x));
}

// Z[k] = Ze[k] + i Zo[k], Ze = (X[k] + conj X[M-k])/2, Zo = (X[k] - conj X[M-k]) conj(W^k)/2.
template <class C>
__device__ __forceinline__ C c2r_pre(C Xk, C Xmk, C Wk) {
  const C e = cadd(Xk, cconj(Xmk));
  const C o = cmul(csub(Xk, cconj(Xmk)), cconj(Wk));
  using R = decltype(e.x);
  // (e + i o)/2
  return cmk(R(0.5) * (e.x - o.y), R(0.5) * (e.y + o.x));
}

// One workgroup per (run, row): the three current components of the row.
template <class R>
__global__ void __launch_bounds__(256) k_fft_j(const Run<R> *__restrict__ runs,
                                               const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int row = it.a;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, cells = n1 * r.n2;
  const auto *Jin = r.J[parity];
  auto *Jz = r.J[parity ^ 1];
  for (int c = 0; c < 3; ++c) {
    const long long base = (long long)c * cells + (long long)row * n1;
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
      const R x0 = to_real<R>(Jin[base + 2 * n]);
      const R x1 = to_real<R>(Jin[base + 2 * n + 1]);
      lds[c * M + n] = cmk(x0, x1);
      Jz[base + 2 * n] = 0;
      Jz[base + 2 * n + 1] = 0;
    }
  }
  __syncthreads();
  lds_fft<C, 6>(lds, M, log2M, 3, r.tw, 2, false);
  const int nk = r.nk;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    const C Wk = r.tw[k], Wmk = r.tw[mk];
    for (int c = 0; c < 3; ++c) {
      const C Zk = lds[c * M + k];
      const C Zmk = lds[c * M + (mk & (M - 1))];
      C Xk = r2c_post(Zk, Zmk, Wk);
      const R fk = r.jfac[k * 3 + c];
      Xk = cscale(Xk, fk);
      if (k == 0) Xk.x += r.jbg0[c];
      C *out = r.Jk + (long long)c * r.n2 * nk + (long long)row * nk;
      out[k] = Xk;
      if (mk != k) {
        C Xm = r2c_post(Zmk, Zk, Wmk);
        Xm = cscale(Xm, r.jfac[mk * 3 + c]);
        out[mk] = Xm;
      }
    }
  }
}

// Forward transform of the six real-space fields of a row into the k-space
// master (initialisation).  Item = (run, row, group): group g covers 3g..3g+2.
template <class R>
__global__ void __launch_bounds__(256) k_fields_to_k(const Run<R> *__restrict__ runs,
                                                     const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int row = it.a, grp = it.b;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, cells = n1 * r.n2, nk = r.nk;
  for (int c = 0; c < 3; ++c) {
    const R *src = r.F + (long long)(3 * grp + c) * cells + (long long)row * n1;
    for (int n = threadIdx.x; n < M; n += blockDim.x) lds[c * M + n] = cmk(src[2 * n], src[2 * n + 1]);
  }
  __syncthreads();
  lds_fft<C, 6>(lds, M, log2M, 3, r.tw, 2, false);
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int c = 0; c < 3; ++c) {
      const C Zk = lds[c * M + k];
      const C Zmk = lds[c * M + (mk & (M - 1))];
      C *out = r.Fk[parity] + (long long)(3 * grp + c) * r.n2 * nk + (long long)row * nk;
      out[k] = r2c_post(Zk, Zmk, r.tw[k]);
      if (mk != k) out[mk] = r2c_post(Zmk, Zk, r.tw[mk]);
    }
  }
}

// =====================================================================
// hybrid Maxwell update in (k1, x2) space
// =====================================================================
//
// Per mode kappa1 the rows i2 are coupled only by the x2 differences.  A thread
// owns one (i2, kappa1) and recomputes the half-step B of the neighbour rows it
// needs, so the update is one pass reading E^n, B^n, j and writing E^{n+1},
// B^{n+1} into the other master buffer:
//   B^{n+1/2} = B^n - (dt/2) C_E E^n
//   E^{n+1}   = E^n + dt (C_B B^{n+1/2} - j~)
//   B^{n+1}   = B^{n+1/2} - (dt/2) C_E E^{n+1}
// with C_E E = (D2+ E3, -D1+ E3, D1+ E2 - D2+ E1), C_B B = (D2- B3, -D1- B3,
// D1- B2 - D2- B1), D1+- = i k1 xi+- (Eq. (18)), D2+- the forward/backward
// differences along x2.
template <class R>
__global__ void __launch_bounds__(256) k_kupdate(const Run<R> *__restrict__ runs,
                                                 const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int nk = r.nk, n2 = r.n2;
  const int e = it.a + threadIdx.x;
  if (e >= n2 * nk) return;
  const int i2 = e / nk, k = e - i2 * nk;
  const long long plane = (long long)n2 * nk;
  const C *Fi = r.Fk[parity];
  C *Fo = r.Fk[parity ^ 1];
  const int rm = wrap_small(i2 - 1, n2), rp = wrap_small(i2 + 1, n2), rpp = wrap_small(i2 + 2, n2);
  auto at = [&](int comp, int row) { return Fi[comp * plane + (long long)row * nk + k]; };
  const C E1m = at(0, rm), E1 = at(0, i2), E1p = at(0, rp), E1pp = at(0, rpp);
  const C E2m = at(1, rm), E2 = at(1, i2), E2p = at(1, rp);
  const C E3m = at(2, rm), E3 = at(2, i2), E3p = at(2, rp), E3pp = at(2, rpp);
  const C B1m = at(3, rm), B1 = at(3, i2), B1p = at(3, rp);
  const C B2 = at(4, i2), B2p = at(4, rp);
  const C B3m = at(5, rm), B3 = at(5, i2), B3p = at(5, rp);
  const C *Jk = r.Jk;
  const C j1 = Jk[(long long)i2 * nk + k], j1p = Jk[(long long)rp * nk + k];
  const C j2 = Jk[plane + (long long)i2 * nk + k];
  const C j3 = Jk[2 * plane + (long long)i2 * nk + k], j3p = Jk[2 * plane + (long long)rp * nk + k];
  const C dp = cmk(r.sym[4 * k + 0], r.sym[4 * k + 1]);
  const C dm = cmk(r.sym[4 * k + 2], r.sym[4 * k + 3]);
  const R hdt = r.hdt, dt = r.dt, i2x = r.idx2;
  // B^{n+1/2} on rows rm, i2, rp
  auto b1h = [&](C B, C Ea, C Eb) { return csub(B, cscale(csub(Eb, Ea), hdt * i2x)); };
  auto b2h = [&](C B, C E) { return cadd(B, cscale(cmul(dp, E), hdt)); };
  auto b3h = [&](C B, C E2x, C E1a, C E1b) {
    return csub(B, cscale(csub(cmul(dp, E2x), cscale(csub(E1b, E1a), i2x)), hdt));
  };
  const C B1h_m = b1h(B1m, E3m, E3), B1h = b1h(B1, E3, E3p), B1h_p = b1h(B1p, E3p, E3pp);
  const C B2h = b2h(B2, E3), B2h_p = b2h(B2p, E3p);
  const C B3h_m = b3h(B3m, E2m, E1m, E1), B3h = b3h(B3, E2, E1, E1p), B3h_p = b3h(B3p, E2p, E1p, E1pp);
  // E^{n+1} on rows i2 (all) and rp (E1, E3)
  auto e1n = [&](C E, C Ba, C Bb, C j) { return cadd(E, cscale(csub(cscale(csub(Bb, Ba), i2x), j), dt)); };
  auto e3n = [&](C E, C B2x, C B1a, C B1b, C j) {
    return cadd(E, cscale(csub(csub(cmul(dm, B2x), cscale(csub(B1b, B1a), i2x)), j), dt));
  };
  const C E1n = e1n(E1, B3h_m, B3h, j1), E1n_p = e1n(E1p, B3h, B3h_p, j1p);
  const C E2n = cadd(E2, cscale(csub(cscale(cmul(dm, B3h), R(-1)), j2), dt));
  const C E3n = e3n(E3, B2h, B1h_m, B1h, j3), E3n_p = e3n(E3p, B2h_p, B1h, B1h_p, j3p);
  // B^{n+1} on row i2
  const C B1n = b1h(B1h, E3n, E3n_p);
  const C B2n = b2h(B2h, E3n);
  const C B3n = b3h(B3h, E2n, E1n, E1n_p);
  const long long o = (long long)i2 * nk + k;
  Fo[o] = E1n;
  Fo[plane + o] = E2n;
  Fo[2 * plane + o] = E3n;
  Fo[3 * plane + o] = B1n;
  Fo[4 * plane + o] = B2n;
  Fo[5 * plane + o] = B3n;
}

// =====================================================================
// inverse FFT of E and B
// =====================================================================
// Item = (run, row, group): components 3g..3g+2 of the master buffer of the
// given parity, written to the real-space fields.
template <class R>
__global__ void __launch_bounds__(256) k_ifft_eb(const Run<R> *__restrict__ runs,
                                                 const Item *__restrict__ items, int parity) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int row = it.a, grp = it.b;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, cells = n1 * r.n2, nk = r.nk;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int c = 0; c < 3; ++c) {
      const C *X = r.Fk[parity] + (long long)(3 * grp + c) * r.n2 * nk + (long long)row * nk;
      const C Xk = X[k], Xmk = X[mk];
      lds[c * M + k] = c2r_pre(Xk, Xmk, r.tw[k]);
      if (k != 0 && mk != k) lds[c * M + mk] = c2r_pre(Xmk, Xk, r.tw[mk]);
    }
  }
  __syncthreads();
  lds_fft<C, 6>(lds, M, log2M, 3, r.tw, 2, true);
  const R s = r.inv_m;
  for (int c = 0; c < 3; ++c) {
    R *dst = r.F + (long long)(3 * grp + c) * cells + (long long)row * n1;
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
      const C z = lds[c * M + n];
      dst[2 * n] = z.x * s;
      dst[2 * n + 1] = z.y * s;
    }
  }
}

// Generic inverse real transform of rows (used to return the corrected current).
template <class R>
__global__ void __launch_bounds__(256) k_inverse_rows(const typename Cplx<R>::T *Xk, int nk, int n1,
                                                      const typename Cplx<R>::T *tw, R scale,
                                                      R *out) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const int row = blockIdx.x;
  const int M = n1 >> 1;
  int log2M = 0;
  while ((1 << log2M) < M) ++log2M;
  const C *X = Xk + (long long)row * nk;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    lds[k] = c2r_pre(X[k], X[mk], tw[k]);
    if (k != 0 && mk != k) lds[mk] = c2r_pre(X[mk], X[k], tw[mk]);
  }
  __syncthreads();
  lds_fft<C, 6>(lds, M, log2M, 1, tw, 2, true);
  for (int n = threadIdx.x; n < M; n += blockDim.x) {
    out[(long long)row * n1 + 2 * n] = lds[n].x * scale;
    out[(long long)row * n1 + 2 * n + 1] = lds[n].y * scale;
  }
}

// =====================================================================
// diagnostics (FP64)
// =====================================================================

__global__ void k_rho_fixed(const Run<float> *run, long long *rho) {
  const Run<float> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const int cell = r.cell[p];
  const int i1 = cell & (r.n1 - 1), i2 = cell >> r.log2n1;
  int s1[3], s2[3];
  const int m1 = fixed_shape(i1, r.f1[p], r.P, s1);
  const int m2 = fixed_shape(i2, r.f2[p], r.P, s2);
  const long long Q = (long long)rintf(r.qw[p] * r.inv_wunit);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int row = wrap_small(m2 - 1 + b, r.n2) * r.n1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const long long v = Q * (long long)s1[a] * (long long)s2[b];
      if (v != 0)
        atomicAdd((unsigned long long *)(rho + row + wrap_pow2(m1 - 1 + a, r.n1)),
                  (unsigned long long)v);
    }
  }
}

__global__ void k_rho_fp64(const Run<double> *run, double *rho) {
  const Run<double> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const int cell = r.cell[p];
  const int i1 = cell & (r.n1 - 1), i2 = cell >> r.log2n1;
  const double f1 = r.f1[p], f2 = r.f2[p];
  const int u1 = f1 >= 0.5, u2 = f2 >= 0.5;
  double s1[3], s2[3];
  spline3<double>(f1 - u1, s1);
  spline3<double>(f2 - u2, s2);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int row = wrap_small(i2 + u2 - 1 + b, r.n2) * r.n1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      unsafeAtomicAdd(rho + row + wrap_pow2(i1 + u1 - 1 + a, r.n1), r.qw[p] * s1[a] * s2[b]);
  }
}

template <class R>
__global__ void k_energy(const R *F, long long cells, double *partial) {
  __shared__ double red[256][6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells;
       i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double v = (double)F[c * cells + i];
      acc[c] += v * v;
    }
  }
  for (int c = 0; c < 6; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 6; ++c) red[threadIdx.x][c] += red[threadIdx.x + w][c];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 6; ++c) partial[blockIdx.x * 6 + c] = red[0][c];
}

template <class R>
__global__ void k_kinetic(const Run<R> *run, double *partial) {
  const Run<R> &r = *run;
  __shared__ double red[256];
  double acc = 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < r.np; p += gridDim.x * blockDim.x) {
    const double u1 = r.u1[p], u2 = r.u2[p], u3 = r.u3[p];
    const double g = sqrt(1.0 + u1 * u1 + u2 * u2 + u3 * u3);
    acc += (double)r.qw[p] * (u1 * u1 + u2 * u2 + u3 * u3) / (g + 1.0);  // qw (gamma - 1)
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Gauss residual (Eq. (27)) of one row in FP64: R = D1- E1 + D2- E2 - f rho.
template <class R>
__global__ void __launch_bounds__(256) k_gauss(const Run<R> *run, int parity, const double *rho,
                                               const double2 *tw64, const double *sym64,
                                               const double *filt, double idx2, double *rows_out) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  double2 *lds = (double2 *)smem_raw;
  __shared__ double red[256][3];
  const Run<R> &r = *run;
  const int row = blockIdx.x;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, nk = r.nk, n2 = r.n2;
  for (int n = threadIdx.x; n < M; n += blockDim.x)
    lds[n] = make_double2(rho[(long long)row * n1 + 2 * n], rho[(long long)row * n1 + 2 * n + 1]);
  __syncthreads();
  lds_fft<double2, 6>(lds, M, log2M, 1, tw64, 2, false);
  const long long plane = (long long)n2 * nk;
  const C *Fk = r.Fk[parity];
  const int rm = wrap_small(row - 1, n2);
  double s2 = 0, smax = 0, sref = 0;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int side = 0; side < 2; ++side) {
      const int kk = side ? mk : k;
      if (side && mk == k) break;
      const double2 Zk = lds[kk & (M - 1)], Zmk = lds[(M - kk) & (M - 1)];
      const double2 rh = r2c_post(Zk, Zmk, tw64[kk]);
      const C e1 = Fk[(long long)row * nk + kk];
      const C e2 = Fk[plane + (long long)row * nk + kk];
      const C e2m = Fk[plane + (long long)rm * nk + kk];
      const double2 dm = make_double2(sym64[4 * kk + 2], sym64[4 * kk + 3]);
      const double2 E1 = make_double2(e1.x, e1.y);
      double2 div = cmul(dm, E1);
      div.x += ((double)e2.x - (double)e2m.x) * idx2;
      div.y += ((double)e2.y - (double)e2m.y) * idx2;
      const double fr_x = filt[kk] * rh.x, fr_y = filt[kk] * rh.y;
      const double rx = div.x - fr_x, ry = div.y - fr_y;
      // the half spectrum stands for both k and -k except at kappa = 0, M
      const double wgt = (kk == 0 || kk == M) ? 1.0 : 2.0;
      const double a2 = rx * rx + ry * ry;
      s2 += wgt * a2;
      smax = fmax(smax, sqrt(a2));
      sref += wgt * (fr_x * fr_x + fr_y * fr_y);
    }
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
    rows_out[3 * row + 0] = red[0][0];
    rows_out[3 * row + 1] = red[0][1];
    rows_out[3 * row + 2] = red[0][2];
  }
}

__global__ void k_cont_fixed(const long long *rn, const long long *ro, const long long *J, int n1,
                             int n2, long long *partial) {
  __shared__ long long red[256];
  const long long cells = (long long)n1 * n2;
  long long m = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells;
       i += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(i % n1), i2 = (int)(i / n1);
    const long long w1 = (long long)i2 * n1 + ((i1 - 1) & (n1 - 1));
    const long long w2 = (long long)wrap_small(i2 - 1, n2) * n1 + i1;
    const long long res = 2 * (rn[i] - ro[i]) - ((J[i] - J[w1]) + (J[cells + i] - J[cells + w2]));
    const long long a = res < 0 ? -res : res;
    m = a > m ? a : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_cont_fp64(const double *rn, const double *ro, const double *J, int n1, int n2,
                            double dt, double idx1, double idx2, double *partial) {
  __shared__ double red[256];
  const long long cells = (long long)n1 * n2;
  double m = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells;
       i += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(i % n1), i2 = (int)(i / n1);
    const long long w1 = (long long)i2 * n1 + ((i1 - 1) & (n1 - 1));
    const long long w2 = (long long)wrap_small(i2 - 1, n2) * n1 + i1;
    const double res = (rn[i] - ro[i]) / dt + (J[i] - J[w1]) * idx1 + (J[cells + i] - J[cells + w2]) * idx2;
    m = fmax(m, fabs(res));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// =====================================================================
// launch wrappers
// =====================================================================
#define HP_CHECK_LAUNCH() (void)hipGetLastError()

template <class R>
void Launch<R>::push_deposit(const Run<R> *runs, const Item *items, int nitems, int parity,
                             unsigned *err, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_push_deposit<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity, err);
}

template <class R>
void Launch<R>::fft_j(const Run<R> *runs, const Item *items, int nitems, int parity, int maxM,
                      hipStream_t s) {
  if (nitems <= 0) return;
  const size_t lds = 3 * (size_t)maxM * sizeof(typename Cplx<R>::T);
  hipLaunchKernelGGL(k_fft_j<R>, dim3(nitems), dim3(256), lds, s, runs, items, parity);
}

template <class R>
void Launch<R>::kupdate(const Run<R> *runs, const Item *items, int nitems, int parity,
                        hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_kupdate<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity);
}

template <class R>
void Launch<R>::ifft_eb(const Run<R> *runs, const Item *items, int nitems, int parity, int maxM,
                        hipStream_t s) {
  if (nitems <= 0) return;
  const size_t lds = 3 * (size_t)maxM * sizeof(typename Cplx<R>::T);
  hipLaunchKernelGGL(k_ifft_eb<R>, dim3(nitems), dim3(256), lds, s, runs, items, parity);
}

template <class R>
void Launch<R>::fields_to_k(const Run<R> *runs, const Item *items, int nitems, int parity,
                            int maxM, hipStream_t s) {
  if (nitems <= 0) return;
  const size_t lds = 3 * (size_t)maxM * sizeof(typename Cplx<R>::T);
  hipLaunchKernelGGL(k_fields_to_k<R>, dim3(nitems), dim3(256), lds, s, runs, items, parity);
}

template struct Launch<float>;
template struct Launch<double>;

void launch_rho_fixed(const Run<float> *run_dev, int np, int, int, long long *rho, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_rho_fixed, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, rho);
}
void launch_rho_fp64(const Run<double> *run_dev, int np, int, int, double *rho, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_rho_fp64, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, rho);
}

template <class R>
void launch_energy(const R *F, long long cells, double *partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_energy<R>, dim3(nblocks), dim3(256), 0, s, F, cells, partial);
}
template void launch_energy<float>(const float *, long long, double *, int, hipStream_t);
template void launch_energy<double>(const double *, long long, double *, int, hipStream_t);

template <class R>
void launch_kinetic(const Run<R> *run_dev, int, double *partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic<R>, dim3(nblocks), dim3(256), 0, s, run_dev, partial);
}
template void launch_kinetic<float>(const Run<float> *, int, double *, int, hipStream_t);
template void launch_kinetic<double>(const Run<double> *, int, double *, int, hipStream_t);

template <class R>
void launch_gauss(const Run<R> *run_dev, int n2, int n1, int parity, const double *rho,
                  const double2 *tw64, const double *sym64, const double *filt, double idx2,
                  double *rows_out, hipStream_t s) {
  const size_t lds = (size_t)(n1 / 2) * sizeof(double2);
  hipLaunchKernelGGL(k_gauss<R>, dim3(n2), dim3(256), lds, s, run_dev, parity, rho, tw64, sym64,
                     filt, idx2, rows_out);
}
template void launch_gauss<float>(const Run<float> *, int, int, int, const double *,
                                  const double2 *, const double *, const double *, double,
                                  double *, hipStream_t);
template void launch_gauss<double>(const Run<double> *, int, int, int, const double *,
                                   const double2 *, const double *, const double *, double,
                                   double *, hipStream_t);

void launch_cont_fixed(const long long *rn, const long long *ro, const long long *J, int n1,
                       int n2, long long *partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_cont_fixed, dim3(nblocks), dim3(256), 0, s, rn, ro, J, n1, n2, partial);
}
void launch_cont_fp64(const double *rn, const double *ro, const double *J, int n1, int n2,
                      double dt, double idx1, double idx2, double *partial, int nblocks,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_cont_fp64, dim3(nblocks), dim3(256), 0, s, rn, ro, J, n1, n2, dt, idx1,
                     idx2, partial);
}

void launch_debug_deposit(int n1, int n2, int P, float inv_wunit, float c3, int np,
                          const int *cell0, const float *off0, const int *cell1,
                          const float *off1, const float *v3, const float *qw, long long *J,
                          unsigned *err, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_debug_deposit, dim3((np + 255) / 256), dim3(256), 0, s, n1, n2, P,
                     inv_wunit, c3, np, cell0, off0, cell1, off1, v3, qw, J, err);
}

template <class R>
void launch_inverse_rows(const typename Cplx<R>::T *Xk, int nk, int n1, int nrows,
                         const typename Cplx<R>::T *tw, R scale, R *out, hipStream_t s) {
  const size_t lds = (size_t)(n1 / 2) * sizeof(typename Cplx<R>::T);
  hipLaunchKernelGGL(k_inverse_rows<R>, dim3(nrows), dim3(256), lds, s, Xk, nk, n1, tw, scale,
                     out);
}
template void launch_inverse_rows<float>(const float2 *, int, int, int, const float2 *, float,
                                         float *, hipStream_t);
template void launch_inverse_rows<double>(const double2 *, int, int, int, const double2 *, double,
                                          double *, hipStream_t);

}  // namespace hp
