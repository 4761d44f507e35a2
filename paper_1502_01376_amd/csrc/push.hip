// push.hip -- particle side of the hybrid Yee-FFT PIC step on gfx950:
// field gather + relativistic Boris push + charge-conserving deposit, the
// particle tile sort, the deposit test hook and the charge density.
//
// The push+deposit kernel runs one workgroup per particle tile (particles are
// counting-sorted by tile every few steps).  The workgroup finds the periodic
// bounding box of its particles' cells, stages the six field components of that
// box (plus the stencil halo) in LDS, pushes its particles gathering from LDS,
// accumulates the current of the box in LDS (64-bit integer atomics in the FP32
// form, so the result does not depend on the order), and adds the box to the
// global accumulators with one atomic per node.  A box too large for LDS falls
// back to gathering and depositing in global memory directly.
#include <type_traits>

#include "hpic_internal.h"

namespace hp {

template <class R> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

// ---------------------------------------------------------------- field sources
// Fields as seen by the gather: rows/cols are offsets returned by row()/col()
// for (possibly out-of-range) node indices; pairs share a stencil:
// p0 = (E1, B2) on (i1+1/2, i2), p1 = (E2, B1) on (i1, i2+1/2),
// e3 on (i1, i2), b3 on (i1+1/2, i2+1/2).
template <class R>
struct GlobalFields {
  gptr<const R> F;
  int n1, n2, cells;
  __device__ int col(int i) const { return wrap_pow2(i, n1); }
  __device__ int row(int j) const { return wrap_small(j, n2) * n1; }
  __device__ typename V2<R>::T p0(int r, int c) const {
    typename V2<R>::T v;
    v.x = F[r + c];
    v.y = F[4 * cells + r + c];
    return v;
  }
  __device__ typename V2<R>::T p1(int r, int c) const {
    typename V2<R>::T v;
    v.x = F[cells + r + c];
    v.y = F[3 * cells + r + c];
    return v;
  }
  __device__ R e3(int r, int c) const { return F[2 * cells + r + c]; }
  __device__ R b3(int r, int c) const { return F[5 * cells + r + c]; }
};

template <class R>
struct LdsFields {
  const typename V2<R>::T *P0, *P1;
  const R *E3, *B3;
  int W;
  __device__ int col(int i) const { return i; }
  __device__ int row(int j) const { return __mul24(j, W); }
  __device__ typename V2<R>::T p0(int r, int c) const { return P0[r + c]; }
  __device__ typename V2<R>::T p1(int r, int c) const { return P1[r + c]; }
  __device__ R e3(int r, int c) const { return E3[r + c]; }
  __device__ R b3(int r, int c) const { return B3[r + c]; }
};

// Quadratic gather (Appendix A): momentum-conserving (every component uses the
// quadratic B-spline around its own staggered node) or, with ec, energy-
// conserving (linear weights along the component's staggered directions).
template <class R, class Src>
__device__ __forceinline__ void gather2(const Src &S, int i1, int i2, R f1, R f2, R Ef[3],
                                        R Bf[3], bool ec) {
  const int up1 = f1 >= R(0.5), up2 = f2 >= R(0.5);
  R wi1[3], wh1[3], wi2[3], wh2[3];
  spline3<R>(f1 - R(up1), wi1);   // integer nodes along x1
  half3<R>(f1 - R(0.5), wh1, ec);  // half nodes along x1
  spline3<R>(f2 - R(up2), wi2);
  half3<R>(f2 - R(0.5), wh2, ec);
  int ci[3], ch[3], ri[3], rh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ci[a] = S.col(i1 + up1 - 1 + a);
    ch[a] = S.col(i1 - 1 + a);
    ri[a] = S.row(i2 + up2 - 1 + a);
    rh[a] = S.row(i2 - 1 + a);
  }
  R e1 = 0, e2 = 0, e3 = 0, b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    R s_e1 = 0, s_e2 = 0, s_e3 = 0, s_b1 = 0, s_b2 = 0, s_b3 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const auto q0 = S.p0(ri[b], ch[a]);  // E1, B2 at (i1+1/2, i2)
      const auto q1 = S.p1(rh[b], ci[a]);  // E2, B1 at (i1, i2+1/2)
      s_e1 += wh1[a] * q0.x;
      s_b2 += wh1[a] * q0.y;
      s_e2 += wi1[a] * q1.x;
      s_b1 += wi1[a] * q1.y;
      s_e3 += wi1[a] * S.e3(ri[b], ci[a]);
      s_b3 += wh1[a] * S.b3(rh[b], ch[a]);
    }
    e1 += wi2[b] * s_e1;
    b2 += wi2[b] * s_b2;
    e2 += wh2[b] * s_e2;
    b1 += wh2[b] * s_b1;
    e3 += wi2[b] * s_e3;
    b3 += wh2[b] * s_b3;
  }
  Ef[0] = e1; Ef[1] = e2; Ef[2] = e3;
  Bf[0] = b1; Bf[1] = b2; Bf[2] = b3;
}

// 1/sqrt(x) and 1/x: hardware approximations (~1 ulp) in FP32, IEEE in FP64.
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }

// Relativistic Boris rotation: u^{n-1/2} -> u^{n+1/2} with E^n, B^n.
template <class R>
__device__ __forceinline__ void boris(R qmhdt, const R E[3], const R B[3], R u[3]) {
  const R e0 = qmhdt * E[0], e1 = qmhdt * E[1], e2 = qmhdt * E[2];
  const R m0 = u[0] + e0, m1 = u[1] + e1, m2 = u[2] + e2;
  const R ig = rsqrt_(R(1) + m0 * m0 + m1 * m1 + m2 * m2);
  const R t0 = qmhdt * B[0] * ig, t1 = qmhdt * B[1] * ig, t2 = qmhdt * B[2] * ig;
  const R sf = R(2) * rcp_(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
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
// bit for bit on the host): g = sqrt(((1 + u1 u1) + u2 u2) + u3 u3) and
// v = u * (1/g), square root and reciprocal correctly rounded.
template <class R>
__device__ __forceinline__ void velocity(const R u[3], R v[3]) {
#pragma clang fp contract(off)
  R s = R(1) + u[0] * u[0];
  s = s + u[1] * u[1];
  s = s + u[2] * u[2];
  const R g = sqrt(s);
  const R ig = R(1) / g;
  v[0] = u[0] * ig;
  v[1] = u[1] * ig;
  v[2] = u[2] * ig;
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

// ---------------------------------------------------------------- current sinks
// A sink maps node indices (in the frame of the cell indices given to the
// deposit) to offsets with row(j) + col(i) and adds a value to component c at
// an offset.
struct GlobalFixed {
  gptr<unsigned long long> J;
  int n1, n2, cells;
  __device__ int row(int j) const { return wrap_small(j, n2) * n1; }
  __device__ int col(int i) const { return wrap_pow2(i, n1); }
  __device__ void add(int c, int off, long long v) const {
    if (v != 0)
      __scoped_atomic_fetch_add(J + c * cells + off, (unsigned long long)v, __ATOMIC_RELAXED,
                                __MEMORY_SCOPE_DEVICE);
  }
};
struct LdsFixed {
  unsigned long long *J;
  int W, plane;
  __device__ int row(int j) const { return __mul24(j, W); }
  __device__ int col(int i) const { return i; }
  __device__ void add(int c, int off, long long v) const {
    // nodes a particle does not reach hold zero: skipping them saves LDS traffic
    if (v != 0) atomicAdd(J + c * plane + off, (unsigned long long)v);
  }
};
struct GlobalFp64 {
  double *J;
  int n1, n2, cells;
  __device__ int row(int j) const { return wrap_small(j, n2) * n1; }
  __device__ int col(int i) const { return wrap_pow2(i, n1); }
  __device__ void add(int c, int off, double v) const {
    if (v != 0.0) unsafeAtomicAdd(J + c * cells + off, v);
  }
};
struct LdsFp64 {
  double *J;
  int W, plane;
  __device__ int row(int j) const { return __mul24(j, W); }
  __device__ int col(int i) const { return i; }
  __device__ void add(int c, int off, double v) const {
    if (v != 0.0) unsafeAtomicAdd(J + c * plane + off, v);
  }
};

// Fixed-point Esirkepov deposit of one particle (2D).  Integer shapes with
// exact sum 2^P make 2 (rho_new - rho_old) = div J hold exactly in the
// integers; j3 is FP32 rounded once per node.  The arithmetic is the one of the
// FP32-precision reference deposit, operation for operation.
//
// UNIT (|charge| 2^P < 2^23, so Q C1 and Q C2 fit 24 signed bits) selects the
// full-rate 24-bit integer products; it is a template parameter so that the
// general 64-bit products are not compiled into the common kernel.
template <bool UNIT, class Sink>
__device__ __forceinline__ void deposit2_fixed(const Sink &K, int P, float inv_wunit, float c3,
                                               int i1, int i2, float fa1, float fa2, int d1,
                                               int d2, float fb1, float fb2, float v3, float qw) {
#pragma clang fp contract(off)
  int sa1[3], sb1[3], sa2[3], sb2[3];
  const int na1 = fixed_shape<UNIT>(i1, fa1, P, sa1);
  const int nb1 = fixed_shape<UNIT>(i1 + d1, fb1, P, sb1);
  const int na2 = fixed_shape<UNIT>(i2, fa2, P, sa2);
  const int nb2 = fixed_shape<UNIT>(i2 + d2, fb2, P, sb2);
  const int base1 = min(na1, nb1) - 1, base2 = min(na2, nb2) - 1;
  int S0x[4], S1x[4], S0y[4], S1y[4];
  place4(sa1, na1 - 1 - base1, S0x);
  place4(sb1, nb1 - 1 - base1, S1x);
  place4(sa2, na2 - 1 - base2, S0y);
  place4(sb2, nb2 - 1 - base2, S1y);
  const float qs = qw * inv_wunit;
  const int Q = (int)rintf(qs);
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
  int ro[4], co[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    ro[a] = K.row(base2 + a);
    co[a] = K.col(base1 + a);
  }
  // J1 = Q C1[a] A2[b], J2 = Q C2[b] A1[a]: exact integer products.  With
  // |Q C| <= 2^22 and A <= 1.5 2^P both factors fit 24 signed bits, so the
  // 48-bit product is one pair of full-rate 24-bit multiplies.
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int qc = UNIT ? mul24_lo(Q, C1[a]) : 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      long long v;
      if (UNIT) v = mul24_wide(qc, A2[b]);
      else v = ((long long)Q * (long long)C1[a]) * (long long)A2[b];
      K.add(0, ro[b] + co[a], v);
    }
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int qc = UNIT ? mul24_lo(Q, C2[b]) : 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      long long v;
      if (UNIT) v = mul24_wide(qc, A1[a]);
      else v = ((long long)Q * (long long)C2[b]) * (long long)A1[a];
      K.add(1, ro[b] + co[a], v);
    }
  }
  // j3 = rint(x0[a] t0[b] + x1[a] t1[b]) with x = S h, t0 = 2 S0y + S1y,
  // t1 = S0y + 2 S1y: the product x1 t1 rounded, then one fused multiply-add.
  // |value| < 2^31 by the choice of c3, so it fits 32 bits.
  const float hv = qs * v3;
  const float h = hv * c3;
  float x0[4], x1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    x0[a] = (float)S0x[a] * h;
    x1[a] = (float)S1x[a] * h;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const float B0 = (float)S0y[b], B1 = (float)S1y[b];
    const float t0 = 2.0f * B0 + B1;
    const float t1 = B0 + 2.0f * B1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const float p1 = x1[a] * t1;
      const float v = __builtin_fmaf(x0[a], t0, p1);
      K.add(2, ro[b] + co[a], (long long)(int)rintf(v));
    }
  }
}

// FP64 Esirkepov deposit of one particle (2D).
template <class Sink>
__device__ __forceinline__ void deposit2_fp64(const Sink &K, double jfx1, double jfx2, int i1,
                                              int i2, double fa1, double fa2, int d1, int d2,
                                              double fb1, double fb2, double v3, double qw) {
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
  int ro[4], co[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    ro[a] = K.row(base2 + a);
    co[a] = K.col(base1 + a);
  }
  const double f1 = qw * jfx1, f2 = qw * jfx2;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc += f1 * (S1x[a] - S0x[a]) * 0.5 * (S0y[b] + S1y[b]);
      K.add(0, ro[b] + co[a], acc);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      acc += f2 * (S1y[b] - S0y[b]) * 0.5 * (S0x[a] + S1x[a]);
      K.add(1, ro[b] + co[a], acc);
    }
  }
  const double g3 = qw * v3;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double W3 = S0x[a] * S0y[b] * (1.0 / 3.0) + S1x[a] * S0y[b] * (1.0 / 6.0) +
                        S0x[a] * S1y[b] * (1.0 / 6.0) + S1x[a] * S1y[b] * (1.0 / 3.0);
      K.add(2, ro[b] + co[a], g3 * W3);
    }
  }
}

template <class T> using lptr = T __attribute__((address_space(3))) *;

// The same deposit into a workgroup's LDS box, giving the same integers bit for
// bit; only the addressing and which zero contributions are left out differ.
// In the window (first node min(nearest node before, after) - 1 per axis) both
// shapes cover nodes 0..2 unless the particle changes its nearest node along
// that axis, so apart from offsets exactly on a stencil edge the zero
// contributions are: along x1, column 3 of j2 and j3 and the running sum C1[2]
// of j1 (zero unless the lane switches nodes along x1); along x2, row 3 of j1
// and j3 and C2[2] of j2; all of j1 (j2) for a particle that does not move
// along x1 (x2) by a quantisation step; all of j3 when |h| is too small for
// any value to round away from zero.  The x1 column is skipped per lane; the
// x2 row for the whole wave when no lane switches along x2 (the common case
// for plasmas drifting along x1); a component for the lanes that do not move
// along its axis, and for the whole wave when none does (a cold drift along x1
// has no j2 and j3 outside the laser).  Every other node is added without a
// test (adding an exact zero changes nothing).  Each window row is one LDS
// pointer, so the nodes of a row are immediate offsets of the atomics.
template <bool UNIT>
__device__ __forceinline__ void deposit2_fixed_lds(const LdsFixed &K, int P, float inv_wunit,
                                                   float c3, int i1, int i2, float fa1, float fa2,
                                                   int d1, int d2, float fb1, float fb2, float v3,
                                                   float qw) {
#pragma clang fp contract(off)
  int sa1[3], sb1[3], sa2[3], sb2[3];
  const int na1 = fixed_shape<UNIT>(i1, fa1, P, sa1);
  const int nb1 = fixed_shape<UNIT>(i1 + d1, fb1, P, sb1);
  const int na2 = fixed_shape<UNIT>(i2, fa2, P, sa2);
  const int nb2 = fixed_shape<UNIT>(i2 + d2, fb2, P, sb2);
  const int base1 = min(na1, nb1) - 1, base2 = min(na2, nb2) - 1;
  int S0x[4], S1x[4], S0y[4], S1y[4];
  place4(sa1, na1 - 1 - base1, S0x);
  place4(sb1, nb1 - 1 - base1, S1x);
  place4(sa2, na2 - 1 - base2, S0y);
  place4(sb2, nb2 - 1 - base2, S1y);
  const float qs = qw * inv_wunit;
  const int Q = (int)rintf(qs);
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
  const bool sw1 = na1 != nb1;                      // per lane
  const bool row3 = __ballot(na2 != nb2) != 0;     // wave-uniform
  // j1 (j2) vanishes when the quantised x1 (x2) shapes are the same before
  // and after the move (three integers summing to 2^P: two of them decide)
  const bool mv1 = (na1 != nb1) | (sa1[0] != sb1[0]) | (sa1[2] != sb1[2]);
  const bool mv2 = (na2 != nb2) | (sa2[0] != sb2[0]) | (sa2[2] != sb2[2]);
  const int W = K.W;
  const lptr<unsigned long long> J1 = (lptr<unsigned long long>)K.J + (__mul24(base2, W) + base1);
  const lptr<unsigned long long> J2 = J1 + K.plane, J3 = J2 + K.plane;
  auto add = [](lptr<unsigned long long> q, long long v) {
    __hip_atomic_fetch_add(q, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto prod = [&](int qc, int c, int f) -> long long {
    if (UNIT) return mul24_wide(qc, f);
    return ((long long)Q * (long long)c) * (long long)f;
  };
  // j1 = Q C1[a] A2[b], a = 0..2 (C1[3] = 0)
  if (__ballot(mv1) != 0 && mv1) {
    int qc1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) qc1[a] = UNIT ? mul24_lo(Q, C1[a]) : 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b == 3 && !row3) break;
      const lptr<unsigned long long> row = J1 + __mul24(b, W);
      add(row, prod(qc1[0], C1[0], A2[b]));
      add(row + 1, prod(qc1[1], C1[1], A2[b]));
      if (sw1) add(row + 2, prod(qc1[2], C1[2], A2[b]));
    }
  }
  // j2 = Q C2[b] A1[a], b = 0..2 (C2[3] = 0)
  if (__ballot(mv2) != 0 && mv2) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (b == 2 && !row3) break;
      const lptr<unsigned long long> row = J2 + __mul24(b, W);
      const int qc = UNIT ? mul24_lo(Q, C2[b]) : 0;
      add(row, prod(qc, C2[b], A1[0]));
      add(row + 1, prod(qc, C2[b], A1[1]));
      add(row + 2, prod(qc, C2[b], A1[2]));
      if (sw1) add(row + 3, prod(qc, C2[b], A1[3]));
    }
  }
  // j3 = rint(x0[a] t0[b] + x1[a] t1[b]) with the operation order of deposit2_fixed
  const float hv = qs * v3;
  const float h = hv * c3;
  // every j3 value rounds to zero when |h| (S0x t0 + S1x t1) stays below 1/2:
  // the bracket is at most 2 (3/4)(9/4) 2^(2P) = 3.375 2^(2P), and 0.45 leaves
  // room for the FP32 rounding of the products
  const bool z3 = fabsf(h) * (3.375f * (float)(1 << P) * (float)(1 << P)) < 0.45f;
  if (__ballot(!z3) == 0 || z3) return;
  float x0[4], x1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    x0[a] = (float)S0x[a] * h;
    x1[a] = (float)S1x[a] * h;
  }
  auto j3v = [&](int a, float t0, float t1) -> long long {
    const float p1 = x1[a] * t1;
    const float v = __builtin_fmaf(x0[a], t0, p1);
    return (long long)(int)rintf(v);
  };
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (b == 3 && !row3) break;
    const float B0 = (float)S0y[b], B1 = (float)S1y[b];
    const float t0 = 2.0f * B0 + B1;
    const float t1 = B0 + 2.0f * B1;
    const lptr<unsigned long long> row = J3 + __mul24(b, W);
    add(row, j3v(0, t0, t1));
    add(row + 1, j3v(1, t0, t1));
    add(row + 2, j3v(2, t0, t1));
    if (sw1) add(row + 3, j3v(3, t0, t1));
  }
}

template <bool UNIT, class Sink>
__device__ __forceinline__ void deposit_one(const Run<float> &r, const Sink &K, int i1, int i2,
                                            float fa1, float fa2, int d1, int d2, float fb1,
                                            float fb2, float v3, float qw) {
  deposit2_fixed<UNIT>(K, r.P, r.inv_wunit, r.c3, i1, i2, fa1, fa2, d1, d2, fb1, fb2, v3, qw);
}
template <bool UNIT>
__device__ __forceinline__ void deposit_one(const Run<float> &r, const LdsFixed &K, int i1, int i2,
                                            float fa1, float fa2, int d1, int d2, float fb1,
                                            float fb2, float v3, float qw) {
  deposit2_fixed_lds<UNIT>(K, r.P, r.inv_wunit, r.c3, i1, i2, fa1, fa2, d1, d2, fb1, fb2, v3, qw);
}
template <bool UNIT, class Sink>
__device__ __forceinline__ void deposit_one(const Run<double> &r, const Sink &K, int i1, int i2,
                                            double fa1, double fa2, int d1, int d2, double fb1,
                                            double fb2, double v3, double qw) {
  deposit2_fp64(K, r.jfx1, r.jfx2, i1, i2, fa1, fa2, d1, d2, fb1, fb2, v3, qw);
}

template <class R> struct Sinks;
template <> struct Sinks<float> { using G = GlobalFixed; using L = LdsFixed; using T = unsigned long long; };
template <> struct Sinks<double> { using G = GlobalFp64; using L = LdsFp64; using T = double; };

// State of one particle as loaded from the buffers.
template <class R>
struct PState {
  int cell;
  R f1, f2, u1, u2, u3, qw;
};

template <class R>
__device__ __forceinline__ PState<R> load_state(const Parts<R> &P, int p) {
  PState<R> s;
  s.cell = G(P.cell)[p];
  s.f1 = G(P.f1)[p];
  s.f2 = G(P.f2)[p];
  s.u1 = G(P.u1)[p];
  s.u2 = G(P.u2)[p];
  s.u3 = G(P.u3)[p];
  s.qw = G(P.qw)[p];
  return s;
}

// Push one particle (state s, index p of buffer P): gather from S at the
// particle's cell (li1, li2) in S's frame, Boris, move, deposit into K in the
// same frame, store.  (gi1, gi2) is the global cell.  Returns the global cell
// after the step (unchanged if the particle was rejected: a non-finite or a
// too-long move leaves it as it was and sets the error word).
template <class R, bool UNIT, bool EC, class Src, class Sink>
__device__ __forceinline__ int push_one(const Run<R> &r, const Parts<R> &P, int p,
                                        const PState<R> &s, int gi1, int gi2, int li1, int li2,
                                        const Src &S, const Sink &K, unsigned *err) {
  R u[3] = {s.u1, s.u2, s.u3};
  R Ef[3], Bf[3];
  gather2<R>(S, li1, li2, s.f1, s.f2, Ef, Bf, EC);
  boris<R>(r.qmhdt, Ef, Bf, u);
  R v[3];
  velocity<R>(u, v);
  const R m1 = r.dtdx1 * v[0], m2 = r.dtdx2 * v[1];
  if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(m1) && isfinite(m2))) {
    atomicOr(err, ERR_NUMERIC);
    return s.cell;
  }
  if (!(fabs(m1) < R(1)) || !(fabs(m2) < R(1))) {
    atomicOr(err, ERR_RANGE);
    return s.cell;
  }
  R g1, g2;
  const int d1 = advance<R>(s.f1, m1, g1);
  const int d2 = advance<R>(s.f2, m2, g2);
  deposit_one<UNIT>(r, K, li1, li2, s.f1, s.f2, d1, d2, g1, g2, v[2], s.qw);
  const int j1 = wrap_pow2(gi1 + d1, r.n1), j2 = wrap_small(gi2 + d2, r.n2);
  const int cell = (j2 << r.log2n1) | j1;
  G(P.cell)[p] = cell;
  G(P.f1)[p] = g1;
  G(P.f2)[p] = g2;
  G(P.u1)[p] = u[0];
  G(P.u2)[p] = u[1];
  G(P.u3)[p] = u[2];
  return cell;
}

__device__ __forceinline__ int wrap_delta_pow2(int d, int n) { return ((d + (n >> 1)) & (n - 1)) - (n >> 1); }
__device__ __forceinline__ int wrap_delta(int d, int n) {
  d += (d < -(n >> 1)) ? n : 0;
  d -= (d >= n - (n >> 1)) ? n : 0;
  return d;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// One workgroup per (run, tile).  The tile's bounding box (from the previous
// push, or the tile itself right after a sort) sizes the LDS staging; the new
// box of the pushed particles is written back for the next step.
template <class R, bool UNIT, bool EC>
__global__ void __launch_bounds__(PUSH_THREADS)
k_push_deposit(const Run<R> *__restrict__ runs, const Item *__restrict__ items, int parity, int pp,
               int lds_bytes, unsigned *err, unsigned *stats) {
  using T2 = typename V2<R>::T;
  using SK = Sinks<R>;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int nbox[4];
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const Parts<R> P = r.pt[pp];
  const int t = it.a;
  const int start = r.tile_start[t], end = r.tile_start[t + 1];
  if (start >= end) return;
  const int n1 = r.n1, n2 = r.n2, cells = n1 * n2;
  const int t2 = t / r.nt1, t1 = t - t2 * r.nt1;
  const int ref1 = t1 * r.T1, ref2 = t2 * r.T2;  // tile origin
  const int *box = r.tile_box + 6 * t;
  const int lo1 = box[0], hi1 = box[1], lo2 = box[2], hi2 = box[3];
  if (threadIdx.x == 0) {
    nbox[0] = 1 << 30; nbox[1] = -(1 << 30); nbox[2] = 1 << 30; nbox[3] = -(1 << 30);
    atomicAdd(&stats[STAT_TILES], 1u);
  }
  // field box: cells lo-1 .. hi+2; current box: lo-2 .. hi+3
  const int FW = hi1 - lo1 + 4, FH = hi2 - lo2 + 4;
  const int W = hi1 - lo1 + 6, H = hi2 - lo2 + 6;
  const int fnodes = FW * FH, jnodes = W * H;
  const size_t jbytes = ((size_t)3 * jnodes * sizeof(typename SK::T) + 15) & ~(size_t)15;
  const size_t need = jbytes + (size_t)fnodes * (2 * sizeof(T2) + 2 * sizeof(R));
  int blo1 = 1 << 30, bhi1 = -(1 << 30), blo2 = 1 << 30, bhi2 = -(1 << 30);
  auto track = [&](int cell) {
    const int d1 = wrap_delta_pow2((cell & (n1 - 1)) - ref1, n1);
    const int d2 = wrap_delta((cell >> r.log2n1) - ref2, n2);
    blo1 = min(blo1, d1); bhi1 = max(bhi1, d1);
    blo2 = min(blo2, d2); bhi2 = max(bhi2, d2);
  };
  if (need > (size_t)lds_bytes) {
    // fallback: gather and deposit in global memory.  The barrier orders the
    // box initialisation above before every wave's min/max at the end (the
    // LDS branch has its own barrier after the staging).
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&stats[STAT_FALLBACK], 1u);
    const GlobalFields<R> S{G((const R *)r.F), n1, n2, cells};
    const typename SK::G K{(decltype(SK::G::J))G((typename SK::T *)r.J[parity]), n1, n2, cells};
    for (int p = start + threadIdx.x; p < end; p += PUSH_THREADS) {
      const PState<R> s = load_state(P, p);
      const int i1 = s.cell & (n1 - 1), i2 = s.cell >> r.log2n1;
      track(push_one<R, UNIT, EC>(r, P, p, s, i1, i2, i1, i2, S, K, err));
    }
  } else {
    // LDS layout: current accumulators first, then the fields (16-byte aligned)
    typename SK::T *lj = (typename SK::T *)smem_raw;
    T2 *lp0 = (T2 *)(smem_raw + jbytes);
    T2 *lp1 = lp0 + fnodes;
    R *le3 = (R *)(lp1 + fnodes);
    R *lb3 = le3 + fnodes;
    const gptr<const R> F = G((const R *)r.F);
    const int o1 = ref1 + lo1 - 1, o2 = ref2 + lo2 - 1;  // global cell of the field-box origin
    for (int q = threadIdx.x; q < fnodes; q += PUSH_THREADS) {
      const int b = q / FW, a = q - b * FW;
      int g2 = (o2 + b) % n2;
      g2 += g2 < 0 ? n2 : 0;
      const int g = g2 * n1 + wrap_pow2(o1 + a, n1);
      T2 v0, v1;
      v0.x = F[g];             // E1
      v0.y = F[4 * cells + g]; // B2
      v1.x = F[cells + g];     // E2
      v1.y = F[3 * cells + g]; // B1
      lp0[q] = v0;
      lp1[q] = v1;
      le3[q] = F[2 * cells + g];
      lb3[q] = F[5 * cells + g];
    }
    for (int q = threadIdx.x; q < 3 * jnodes; q += PUSH_THREADS) lj[q] = 0;
    __syncthreads();
    // Particles use field-box coordinates (origin: cell lo-1).  The current box
    // starts one cell earlier, so its sink is shifted by one row and one column.
    const LdsFields<R> S{lp0, lp1, le3, lb3, FW};
    const typename SK::L K{lj + W + 1, W, jnodes};
    // each thread loads a batch of PUSH_BATCH particles (strided by the block,
    // so every load stays coalesced) before pushing them: more bytes in flight
    for (int p0 = start + threadIdx.x; p0 < end; p0 += PUSH_BATCH * PUSH_THREADS) {
      PState<R> st[PUSH_BATCH];
#pragma unroll
      for (int k = 0; k < PUSH_BATCH; ++k) {
        const int p = p0 + k * PUSH_THREADS;
        if (p < end) st[k] = load_state(P, p);
      }
#pragma unroll
      for (int k = 0; k < PUSH_BATCH; ++k) {
        const int p = p0 + k * PUSH_THREADS;
        if (p < end) {
          const int i1 = st[k].cell & (n1 - 1), i2 = st[k].cell >> r.log2n1;
          const int d1 = wrap_delta_pow2(i1 - ref1, n1), d2 = wrap_delta(i2 - ref2, n2);
          track(push_one<R, UNIT, EC>(r, P, p, st[k], i1, i2, d1 - lo1 + 1, d2 - lo2 + 1, S, K, err));
        }
      }
    }
    __syncthreads();
    // add the box to the global accumulators
    const auto J = G((typename SK::T *)r.J[parity]);
    const int c1 = ref1 + lo1 - 2, c2 = ref2 + lo2 - 2;
    for (int q = threadIdx.x; q < jnodes; q += PUSH_THREADS) {
      const int b = q / W, a = q - b * W;
      int g2 = (c2 + b) % n2;
      g2 += g2 < 0 ? n2 : 0;
      const int g = g2 * n1 + wrap_pow2(c1 + a, n1);
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const typename SK::T v = lj[comp * jnodes + q];
        if (v != 0)
          __scoped_atomic_fetch_add(J + comp * cells + g, v, __ATOMIC_RELAXED, __MEMORY_SCOPE_DEVICE);
      }
    }
  }
  // new bounding box of the tile's particles
  blo1 = wave_min(blo1); bhi1 = wave_max(bhi1); blo2 = wave_min(blo2); bhi2 = wave_max(bhi2);
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&nbox[0], blo1); atomicMax(&nbox[1], bhi1);
    atomicMin(&nbox[2], blo2); atomicMax(&nbox[3], bhi2);
  }
  __syncthreads();
  if (threadIdx.x < 4) r.tile_box[6 * t + threadIdx.x] = nbox[threadIdx.x];
}

// ---------------------------------------------------------------- tile sort
// Counting sort of the particles of every run by tile of their current cell:
// count, exclusive scan (one workgroup per run), scatter into the other
// particle buffer.  The order inside a tile is whatever the atomics give; the
// step's results do not depend on it.
template <class R>
__device__ __forceinline__ int tile_of(const Run<R> &r, int cell) {
  const int i1 = cell & (r.n1 - 1);
  if (r.dim == 3) {
    const int i2 = (cell >> r.log2n1) & ((1 << (r.sh3 - r.log2n1)) - 1), i3 = cell >> r.sh3;
    return ((i3 / r.T3) * r.nt2 + i2 / r.T2) * r.nt1 + i1 / r.T1;
  }
  const int i2 = cell >> r.log2n1;
  return (i2 / r.T2) * r.nt1 + i1 / r.T1;
}

template <class R>
__global__ void k_sort_clear(const Run<R> *runs, const Item *per_run) {
  const Run<R> &r = runs[per_run[blockIdx.x].run];
  for (int t = threadIdx.x; t < r.ntiles; t += blockDim.x) r.tile_cnt[t] = 0;
}

template <class R>
__global__ void k_sort_count(const Run<R> *runs, const Item *chunks, int pp) {
  const Item it = chunks[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const bool active = threadIdx.x < (unsigned)it.b;
  const int key = active ? tile_of(r, r.pt[pp].cell[it.a + threadIdx.x]) : 0;
  wave_atomic_inc(r.tile_cnt, key, active);
}

// exclusive scan of tile_cnt into tile_start (and back into tile_cnt as the
// scatter cursor); one 1024-thread workgroup per run
template <class R>
__global__ void __launch_bounds__(1024) k_sort_scan(const Run<R> *runs, const Item *per_run) {
  __shared__ int part[1024];
  const Run<R> &r = runs[per_run[blockIdx.x].run];
  const int nt = r.ntiles;
  const int per = (nt + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int t = b0; t < min(b0 + per, nt); ++t) s += r.tile_cnt[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;  // exclusive prefix of this thread's block
  for (int t = b0; t < min(b0 + per, nt); ++t) {
    const int c = r.tile_cnt[t];
    r.tile_start[t] = run;
    r.tile_cnt[t] = run;
    run += c;
    // right after the sort every particle of tile t lies in the tile; the box
    // is expressed in the frame the push uses (cell minus tile origin, wrapped
    // into [-n/2, n - n/2)), so a tile wider than half the grid covers the
    // whole wrapped range
    const int t3 = t / (r.nt1 * r.nt2), t12 = t - t3 * r.nt1 * r.nt2;
    const int t2 = t12 / r.nt1, t1 = t12 - t2 * r.nt1;
    const int w[3] = {min(r.T1, r.n1 - t1 * r.T1), min(r.T2, r.n2 - t2 * r.T2),
                      min(r.T3, r.n3 - t3 * r.T3)};
    const int nn[3] = {r.n1, r.n2, r.n3};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool full = w[d] > nn[d] - (nn[d] >> 1);
      r.tile_box[6 * t + 2 * d] = full ? -(nn[d] >> 1) : 0;
      r.tile_box[6 * t + 2 * d + 1] = full ? nn[d] - (nn[d] >> 1) - 1 : w[d] - 1;
    }
  }
  if (threadIdx.x == 1023) r.tile_start[nt] = part[1023];
}

// Scatter.  With `scramble`, a particle's rank within its tile (arrival order)
// is transposed (a bijection, below) so that consecutive slots of a tile hold
// particles of different cells: the lanes of a push wave then do not hit the
// same LDS accumulator, and their addresses fall in different banks.  That is
// needed once, for input in cell order; later sorts keep the arrival order
// (already spread), so lanes of one wave with the same tile write consecutive
// slots.
template <class R>
__global__ void k_sort_scatter(const Run<R> *runs, const Item *chunks, int pp, int scramble) {
  const Item it = chunks[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const bool active = threadIdx.x < (unsigned)it.b;
  const int p = it.a + threadIdx.x;
  const Parts<R> &A = r.pt[pp];
  const Parts<R> &B = r.pt[pp ^ 1];
  const int c = active ? A.cell[p] : 0;
  const int t = tile_of(r, c);
  const int q = wave_atomic_inc(r.tile_cnt, t, active);
  if (!active) return;
  const int t0 = r.tile_start[t], cnt = r.tile_start[t + 1] - t0;
  const int rank = q - t0;
  int slot = t0 + rank;
  if (scramble) {
    // ragged transpose by the tile's mean particles per cell m: arrival rank
    // r = m j + k (loaded particles arrive in cell order) goes to column k,
    // row j, so consecutive slots, the lanes of a wave, hold particles of
    // different cells
    const int area = (r.dim == 3) ? r.T1 * r.T2 * r.T3 : r.T1 * r.T2;
    const int m = max(1, cnt / area);
    const int rows = cnt / m, rem = cnt - rows * m;
    const int k = rank % m, j = rank / m;
    slot = t0 + k * rows + min(k, rem) + j;
  }
  B.cell[slot] = c;
  B.id[slot] = A.id[p];
  B.f1[slot] = A.f1[p];
  B.f2[slot] = A.f2[p];
  if (r.dim == 3) B.f3[slot] = A.f3[p];
  B.u1[slot] = A.u1[p];
  B.u2[slot] = A.u2[p];
  B.u3[slot] = A.u3[p];
  B.qw[slot] = A.qw[p];
}

// ---------------------------------------------------------------- test hook
// Deposit alone on given moves (tests of the fixed-point deposit).
__global__ void k_debug_deposit(int n1, int n2, int P, float inv_wunit, float c3, int np,
                                const int *cell0, const float *off0, const int *cell1,
                                const float *off1, const float *v3, const float *qw,
                                long long *J, unsigned *err) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int a1 = cell0[p], a2 = cell0[np + p], b1 = cell1[p], b2 = cell1[np + p];
  const int d1 = wrap_delta_pow2(b1 - a1, n1);
  const int d2 = wrap_delta(b2 - a2, n2);
  if (d1 < -1 || d1 > 1 || d2 < -1 || d2 > 1 || a1 < 0 || a1 >= n1 || a2 < 0 || a2 >= n2) {
    atomicOr(err, ERR_RANGE);
    return;
  }
  const GlobalFixed K{G((unsigned long long *)J), n1, n2, n1 * n2};
  deposit2_fixed<false>(K, P, inv_wunit, c3, a1, a2, off0[p], off0[np + p], d1, d2, off1[p],
                 off1[np + p], v3[p], qw[p]);
}

// ---------------------------------------------------------------- charge density
__global__ void k_rho_fixed(const Run<float> *run, int pp, long long *rho) {
  const Run<float> &r = *run;
  const Parts<float> &P = r.pt[pp];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const int cell = P.cell[p];
  const int i1 = cell & (r.n1 - 1), i2 = cell >> r.log2n1;
  int s1[3], s2[3];
  const int m1 = fixed_shape<false>(i1, P.f1[p], r.P, s1);
  const int m2 = fixed_shape<false>(i2, P.f2[p], r.P, s2);
  const long long Q = (long long)rintf(P.qw[p] * r.inv_wunit);
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

__global__ void k_rho_fp64(const Run<double> *run, int pp, double *rho) {
  const Run<double> &r = *run;
  const Parts<double> &P = r.pt[pp];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const int cell = P.cell[p];
  const int i1 = cell & (r.n1 - 1), i2 = cell >> r.log2n1;
  const double f1 = P.f1[p], f2 = P.f2[p];
  const int u1 = f1 >= 0.5, u2 = f2 >= 0.5;
  double s1[3], s2[3];
  spline3<double>(f1 - u1, s1);
  spline3<double>(f2 - u2, s2);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int row = wrap_small(i2 + u2 - 1 + b, r.n2) * r.n1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      unsafeAtomicAdd(rho + row + wrap_pow2(i1 + u1 - 1 + a, r.n1), P.qw[p] * s1[a] * s2[b]);
  }
}

template <class R>
__global__ void k_kinetic(const Run<R> *run, int pp, double *partial) {
  const Run<R> &r = *run;
  const Parts<R> &P = r.pt[pp];
  __shared__ double red[256];
  double acc = 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < r.np; p += gridDim.x * blockDim.x) {
    const double u1 = P.u1[p], u2 = P.u2[p], u3 = P.u3[p];
    const double uu = u1 * u1 + u2 * u2 + u3 * u3;
    acc += (double)P.qw[p] * uu / (sqrt(1.0 + uu) + 1.0);  // qw (gamma - 1)
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- launches
template <class R>
void Launch<R>::push_deposit(const Run<R> *runs, const Item *items, int nitems, int parity, int pp,
                             int lds_bytes, bool unit, bool ec, unsigned *err, unsigned *stats,
                             hipStream_t s) {
  if (nitems <= 0) return;
  if constexpr (std::is_same<R, float>::value) {
    if (unit) {
      if (ec)
        hipLaunchKernelGGL((k_push_deposit<R, true, true>), dim3(nitems), dim3(PUSH_THREADS),
                           lds_bytes, s, runs, items, parity, pp, lds_bytes, err, stats);
      else
        hipLaunchKernelGGL((k_push_deposit<R, true, false>), dim3(nitems), dim3(PUSH_THREADS),
                           lds_bytes, s, runs, items, parity, pp, lds_bytes, err, stats);
      return;
    }
  }
  if (ec)
    hipLaunchKernelGGL((k_push_deposit<R, false, true>), dim3(nitems), dim3(PUSH_THREADS),
                       lds_bytes, s, runs, items, parity, pp, lds_bytes, err, stats);
  else
    hipLaunchKernelGGL((k_push_deposit<R, false, false>), dim3(nitems), dim3(PUSH_THREADS),
                       lds_bytes, s, runs, items, parity, pp, lds_bytes, err, stats);
}

template <class R>
void Launch<R>::sort(const Run<R> *runs, const Item *chunks, int nchunks, const Item *per_run,
                     int nruns, int pp, bool scramble, hipStream_t s) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(k_sort_clear<R>, dim3(nruns), dim3(256), 0, s, runs, per_run);
  hipLaunchKernelGGL(k_sort_count<R>, dim3(nchunks), dim3(256), 0, s, runs, chunks, pp);
  hipLaunchKernelGGL(k_sort_scan<R>, dim3(nruns), dim3(1024), 0, s, runs, per_run);
  hipLaunchKernelGGL(k_sort_scatter<R>, dim3(nchunks), dim3(256), 0, s, runs, chunks, pp,
                     scramble ? 1 : 0);
}

template struct Launch<float>;
template struct Launch<double>;

void launch_rho_fixed(const Run<float> *run_dev, int pp, int np, long long *rho, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_rho_fixed, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, pp, rho);
}
void launch_rho_fp64(const Run<double> *run_dev, int pp, int np, double *rho, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_rho_fp64, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, pp, rho);
}

template <class R>
void launch_kinetic(const Run<R> *run_dev, int pp, double *partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic<R>, dim3(nblocks), dim3(256), 0, s, run_dev, pp, partial);
}
template void launch_kinetic<float>(const Run<float> *, int, double *, int, hipStream_t);
template void launch_kinetic<double>(const Run<double> *, int, double *, int, hipStream_t);

void launch_debug_deposit(int n1, int n2, int P, float inv_wunit, float c3, int np,
                          const int *cell0, const float *off0, const int *cell1,
                          const float *off1, const float *v3, const float *qw, long long *J,
                          unsigned *err, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_debug_deposit, dim3((np + 255) / 256), dim3(256), 0, s, n1, n2, P,
                     inv_wunit, c3, np, cell0, off0, cell1, off1, v3, qw, J, err);
}

}  // namespace hp
