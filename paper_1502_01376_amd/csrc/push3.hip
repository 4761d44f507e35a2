// push3.hip -- particle side of the 3D hybrid Yee-FFT PIC step on gfx950:
// field gather + relativistic Boris push + Esirkepov current deposit in 3D,
// and the 3D charge density of the diagnostics.
//
// One workgroup per particle tile (T1 x T2 x T3 cells).  The tile's particles
// gather the 27-node quadratic stencil of each field component, in the FP32
// form from a copy of the tile's field box staged in LDS when it fits next to
// the current box (else, and in the FP64 form, through the cache), and deposit
// into an LDS copy of the current box that is added to the global accumulators
// with one atomic per touched node.  Too large a box falls back to depositing
// with global atomics.
//
// FP32 form: the Esirkepov weights of the FP32 offsets are computed in FP64
// and each node's contribution is rounded once to an integer, accumulated in
// 64 bits: the result does not depend on the order of the atomics.  (An exact
// integer scheme as in 2D would need products of three shape factors plus the
// charge, more than 64 bits for general charges.)
#include "hpic_internal.h"

namespace hp {

__device__ __forceinline__ int wrap_delta_pow2_3(int d, int n) { return ((d + (n >> 1)) & (n - 1)) - (n >> 1); }
__device__ __forceinline__ int wrap_delta_3(int d, int n) {
  d += (d < -(n >> 1)) ? n : 0;
  d -= (d >= n - (n >> 1)) ? n : 0;
  return d;
}
// i mod n for any i (a loop of corrections: boxes that fit the LDS reach at
// most a few periods of a small grid)
__device__ __forceinline__ int wrap_any3(int i, int n) {
  while (i >= n) i -= n;
  while (i < 0) i += n;
  return i;
}

__device__ __forceinline__ int wave_min3(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max3(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ float rsqrt3(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt3(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp3(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp3(double x) { return 1.0 / x; }

// Momentum-conserving quadratic gather of one staggered component: the
// weights along each axis are those of the integer (h = 0) or half (h = 1)
// node stencil; o_d[3] are the node offsets (already wrapped and scaled).
template <class R, class PT>
__device__ __forceinline__ R gather_comp(PT F, const R w1[3], const int o1[3], const R w2[3],
                                         const int o2[3], const R w3[3], const int o3[3]) {
  R acc = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R s2 = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const PT row = F + o3[c] + o2[b];
      const R s1 = w1[0] * row[o1[0]] + w1[1] * row[o1[1]] + w1[2] * row[o1[2]];
      s2 += w2[b] * s1;
    }
    acc += w3[c] * s2;
  }
  return acc;
}

template <class R>
__device__ __forceinline__ void boris3(R qmhdt, const R E[3], const R B[3], R u[3]) {
  const R e0 = qmhdt * E[0], e1 = qmhdt * E[1], e2 = qmhdt * E[2];
  const R m0 = u[0] + e0, m1 = u[1] + e1, m2 = u[2] + e2;
  const R ig = rsqrt3(R(1) + m0 * m0 + m1 * m1 + m2 * m2);
  const R t0 = qmhdt * B[0] * ig, t1 = qmhdt * B[1] * ig, t2 = qmhdt * B[2] * ig;
  const R sf = R(2) * rcp3(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const R s0 = t0 * sf, s1 = t1 * sf, s2 = t2 * sf;
  const R p0 = m0 + (m1 * t2 - m2 * t1);
  const R p1 = m1 + (m2 * t0 - m0 * t2);
  const R p2 = m2 + (m0 * t1 - m1 * t0);
  u[0] = m0 + (p1 * s2 - p2 * s1) + e0;
  u[1] = m1 + (p2 * s0 - p0 * s2) + e1;
  u[2] = m2 + (p0 * s1 - p1 * s0) + e2;
}

// v = u / sqrt(((1 + u1 u1) + u2 u2) + u3 u3), one correctly rounded square
// root and reciprocal.
template <class R>
__device__ __forceinline__ void velocity3(const R u[3], R v[3]) {
#pragma clang fp contract(off)
  R s = R(1) + u[0] * u[0];
  s = s + u[1] * u[1];
  s = s + u[2] * u[2];
  const R ig = R(1) / sqrt(s);
  v[0] = u[0] * ig;
  v[1] = u[1] * ig;
  v[2] = u[2] * ig;
}

template <class R>
__device__ __forceinline__ int advance3(R f, R d, R &g) {
  g = f + d;
  int s = 0;
  if (g >= R(1)) {
    g = g - R(1);
    s = 1;
  } else if (g < R(0)) {
    g = g + R(1);
    s = -1;
    if (g >= R(1)) {
      g = R(0);
      s = 0;
    }
  }
  return s;
}

// FP64 shape factors of one coordinate at the nodes m-1, m, m+1 around the
// nearest node m = cell + (f >= 1/2); d = offset from m (exact).  No
// contraction: the FP32 form's integer deposit is defined operation by
// operation.
__device__ __forceinline__ int dshape3(int cell, double f, double s[3]) {
#pragma clang fp contract(off)
  const int up = (f >= 0.5) ? 1 : 0;
  const double d = up ? (f - 1.0) : f;
  const double a = 0.5 - d, b = 0.5 + d;
  s[0] = 0.5 * (a * a);
  s[1] = 0.75 - d * d;
  s[2] = 0.5 * (b * b);
  return cell + up;
}

template <class T>
__device__ __forceinline__ void place4_3(const T s[3], int off, T out[4]) {
  out[0] = off ? T(0) : s[0];
  out[1] = off ? s[0] : s[1];
  out[2] = off ? s[1] : s[2];
  out[3] = off ? s[2] : T(0);
}

// Current sinks: node offset = o1[a] + o2[b] + o3[c] (from offs()), add().
// (FP32 form: node offsets in bytes, so that an address is one add; the LDS
// atomic is issued for zero contributions too: adding an exact zero changes
// nothing, and it costs less than the test)
struct Sink3Lds {
  unsigned char __attribute__((address_space(3))) *J;
  int W8, WH8, vol8;
  static __device__ Sink3Lds make(void *lj, int W, int WH, int vol) {
    return Sink3Lds{(unsigned char __attribute__((address_space(3))) *)lj, 8 * W, 8 * WH, 8 * vol};
  }
  __device__ int offs(int axis, int i) const { return axis == 0 ? 8 * i : (axis == 1 ? i * W8 : i * WH8); }
  using Base = unsigned char __attribute__((address_space(3))) *;
  __device__ Base base(int c, int off) const { return J + c * vol8 + off; }
  __device__ void put(Base b, int off, long long v) const {
    __hip_atomic_fetch_add((unsigned long long __attribute__((address_space(3))) *)(b + off),
                           (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};
struct Sink3Global {
  gptr<unsigned long long> J;
  int n1, n2, n3, n12, cells;
  __device__ int offs(int axis, int i) const {
    return axis == 0 ? wrap_pow2(i, n1) : (axis == 1 ? wrap_small(i, n2) * n1 : wrap_small(i, n3) * n12);
  }
  using Base = gptr<unsigned long long>;
  __device__ Base base(int c, int off) const { return J + c * cells + off; }
  __device__ void put(Base b, int off, long long v) const {
    if (v != 0)
      __scoped_atomic_fetch_add(b + off, (unsigned long long)v, __ATOMIC_RELAXED,
                                __MEMORY_SCOPE_DEVICE);
  }
};
struct Sink3LdsF64 {
  double *J;
  int W, WH, vol;
  static __device__ Sink3LdsF64 make(void *lj, int W, int WH, int vol) {
    return Sink3LdsF64{(double *)lj, W, WH, vol};
  }
  __device__ int offs(int axis, int i) const { return axis == 0 ? i : (axis == 1 ? i * W : i * WH); }
  __device__ void add(int c, int off, double v) const {
    if (v != 0.0) unsafeAtomicAdd(J + c * vol + off, v);
  }
};
struct Sink3GlobalF64 {
  double *J;
  int n1, n2, n3, n12, cells;
  __device__ int offs(int axis, int i) const {
    return axis == 0 ? wrap_pow2(i, n1) : (axis == 1 ? wrap_small(i, n2) * n1 : wrap_small(i, n3) * n12);
  }
  __device__ void add(int c, int off, double v) const {
    if (v != 0.0) unsafeAtomicAdd(J + c * cells + off, v);
  }
};

// Esirkepov deposit of one particle in 3D.  l[] is the particle's cell in the
// sink's frame, fa[] the old offsets, dd[] the cell moves, fb[] the new
// offsets.  For component d, with (e, f) the other axes in cyclic order:
//   T[i][j] = S0e[i] (2 S0f[j] + S1f[j]) + S1e[i] (S0f[j] + 2 S1f[j])
//           (6 times the Esirkepov bracket), C[k] = running sum of S1d - S0d,
//   J_d[k][i][j] += C[k] g T[i][j],  k = 0..2.
// FP32 form: the weights of the FP32 offsets in FP64, g = (qw inv_wunit) cj
// with cj = 2^40, every FP64 operation rounded once in the order written, the
// node value rounded to a 64-bit integer (j_d = -(dx_d/dt) J / (6 inv_wunit
// cj)): the sums are independent of the order of the atomics and continuity
// holds to about 2^-41 of a particle's charge per node and step (with FP32
// weights and a 2^28 scale, long drifting-beam runs grew a spurious k1 = 0
// mode).  FP64 form: g = qw (-dx_d/dt) / 6, physical current.
// Where no particle of the wave changes its nearest node along an axis, the
// stencil is three nodes wide there (the fourth row of S0 and S1 is zero, the
// last running sum C[2] along that axis only the rounding of 1 - 1) and both
// blocks of terms are skipped for the whole wave.  In the FP32 form the skip
// is exact: the skipped rows add exact zeros, and |C[2]| is a few units of
// 2^-53, so |C[2] g T| < 2^-53 x 8 x 2^40 x 3.4 stays far below the half
// unit that would round away from zero.  The FP32 form walks the nodes (i, j)
// of the two other axes outside the three running sums, so only one bracket
// T is live at a time (the whole 4 x 4 block of brackets spilled registers).
template <class Sink>
__device__ __forceinline__ void deposit3_fixed(const Sink &K, float inv_wunit, float cj,
                                               const int l[3], const float fa[3], const int dd[3],
                                               const float fb[3], float qw) {
#pragma clang fp contract(off)
  double S0[3][4], S1[3][4], C[3][4];
  int o[3][4];
  bool w4[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double sa[3], sb[3];
    const int na = dshape3(l[d], (double)fa[d], sa);
    const int nb = dshape3(l[d] + dd[d], (double)fb[d], sb);
    const int base = min(na, nb) - 1;
    w4[d] = __ballot(na != nb) != 0;
    place4_3(sa, na - 1 - base, S0[d]);
    place4_3(sb, nb - 1 - base, S1[d]);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      acc = acc + (S1[d][k] - S0[d][k]);
      C[d][k] = acc;
      o[d][k] = K.offs(d, base + k);
    }
  }
  const double gq = ((double)qw * (double)inv_wunit) * (double)cj;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    double u0[4], u1[4], cg[3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u0[j] = 2.0 * S0[f][j] + S1[f][j];
      u1[j] = S0[f][j] + 2.0 * S1[f][j];
    }
    typename Sink::Base bk[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cg[k] = C[d][k] * gq;
      bk[k] = K.base(d, o[d][k]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i == 3 && !w4[e]) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j == 3 && !w4[f]) continue;
        const double T = S0[e][i] * u0[j] + S1[e][i] * u1[j];
        const int oij = o[e][i] + o[f][j];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (k == 2 && !w4[d]) continue;
          K.put(bk[k], oij, rint_i64(cg[k] * T));
        }
      }
    }
  }
}

template <class Sink>
__device__ __forceinline__ void deposit3_fp64(const Sink &K, const double jf[3], const int l[3],
                                              const double fa[3], const int dd[3],
                                              const double fb[3], double qw) {
  double S0[3][4], S1[3][4], C[3][4];
  int o[3][4];
  bool w4[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double sa[3], sb[3];
    const int na = dshape3(l[d], fa[d], sa);
    const int nb = dshape3(l[d] + dd[d], fb[d], sb);
    const int base = min(na, nb) - 1;
    w4[d] = __ballot(na != nb) != 0;
    place4_3(sa, na - 1 - base, S0[d]);
    place4_3(sb, nb - 1 - base, S1[d]);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      acc += S1[d][k] - S0[d][k];
      C[d][k] = acc;
      o[d][k] = K.offs(d, base + k);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    const double g = qw * jf[d] * (1.0 / 6.0);
    double u0[4], u1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u0[j] = 2.0 * S0[f][j] + S1[f][j];
      u1[j] = S0[f][j] + 2.0 * S1[f][j];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == 2 && !w4[d]) continue;  // three-node stencil along d
      const double cg = C[d][k] * g;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i == 3 && !w4[e]) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j == 3 && !w4[f]) continue;
          K.add(d, o[d][k] + o[e][i] + o[f][j], cg * (S0[e][i] * u0[j] + S1[e][i] * u1[j]));
        }
      }
    }
  }
}

template <class R> struct Sinks3;
template <> struct Sinks3<float> { using G = Sink3Global; using L = Sink3Lds; using T = unsigned long long; };
template <> struct Sinks3<double> { using G = Sink3GlobalF64; using L = Sink3LdsF64; using T = double; };

template <class Sink>
__device__ __forceinline__ void deposit3_one(const Run<float> &r, const Sink &K, const int l[3],
                                             const float fa[3], const int dd[3], const float fb[3],
                                             float qw) {
  deposit3_fixed(K, r.inv_wunit, r.cj, l, fa, dd, fb, qw);
}
template <class Sink>
__device__ __forceinline__ void deposit3_one(const Run<double> &r, const Sink &K, const int l[3],
                                             const double fa[3], const int dd[3],
                                             const double fb[3], double qw) {
  const double jf[3] = {r.jfx1, r.jfx2, r.jfx3};
  deposit3_fp64(K, jf, l, fa, dd, fb, qw);
}

__device__ __forceinline__ void unpack3(int cell, int log2n1, int sh3, int n1, int &i1, int &i2,
                                        int &i3) {
  i1 = cell & (n1 - 1);
  i2 = (cell >> log2n1) & ((1 << (sh3 - log2n1)) - 1);
  i3 = cell >> sh3;
}

template <class T> using lptr3 = T __attribute__((address_space(3))) *;

// Field sources of the gather: the whole grid in global memory, or the tile's
// field box in LDS ([6][FD][FH][FW], origin one cell below the tile's particle
// box, i.e. sink-frame cell - 1 along each axis; FP32 form only).
template <class R> struct GlobalF3 {
  static constexpr bool local = false;
};
template <class R> struct LdsF3 {
  static constexpr bool local = true;
  lptr3<R> F;
  int FW, FWH, plane;
};

// State of one particle as loaded: offsets, momenta, charge.
template <class R> struct PState3 {
  R f[3], u[3], qw;
};
template <class R>
__device__ __forceinline__ PState3<R> load_state3(const Parts<R> &P, int p) {
  PState3<R> s;
  s.f[0] = G(P.f1)[p];
  s.f[1] = G(P.f2)[p];
  s.f[2] = G(P.f3)[p];
  s.u[0] = G(P.u1)[p];
  s.u[1] = G(P.u2)[p];
  s.u[2] = G(P.u3)[p];
  s.qw = G(P.qw)[p];
  return s;
}

// Push particle p (loaded state st, packed cell `cell`): gather at global
// cell (g1, g2, g3) (from the field box when S is local), Boris, move, deposit
// into K in the sink's frame (cell l[]), store.  Returns the new packed cell
// (the old one if the particle was rejected).
template <class R, class Src, class Sink>
__device__ __forceinline__ int push_one3(const Run<R> &r, const Parts<R> &P, int p, int cell,
                                         const PState3<R> &st, int g1, int g2, int g3,
                                         const int l[3], const Src &S, const Sink &K,
                                         unsigned *err) {
  const R f[3] = {st.f[0], st.f[1], st.f[2]};
  R u[3] = {st.u[0], st.u[1], st.u[2]};
  const R qw = st.qw;
  const int n1 = r.n1, n2 = r.n2, n3 = r.n3, n12 = n1 * n2, cells = r.cells;
  // stencil weights and offsets, integer (i) and half (h) nodes per axis
  R wi[3][3], wh[3][3];
  int oi[3][3], oh[3][3];
  const int gc[3] = {g1, g2, g3};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int up = f[d] >= R(0.5);
    spline3<R>(f[d] - R(up), wi[d]);
    half3<R>(f[d] - R(0.5), wh[d], r.interp != 0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if constexpr (Src::local) {
        // box-local nodes: sink-frame cell - 1, then the stencil
        const int ni = l[d] - 1 + up - 1 + a, nh = l[d] - 1 - 1 + a;
        const int sc = d == 0 ? 1 : (d == 1 ? S.FW : S.FWH);
        oi[d][a] = ni * sc;
        oh[d][a] = nh * sc;
      } else {
        const int ni = gc[d] + up - 1 + a, nh = gc[d] - 1 + a;
        if (d == 0) {
          oi[0][a] = wrap_pow2(ni, n1);
          oh[0][a] = wrap_pow2(nh, n1);
        } else if (d == 1) {
          oi[1][a] = wrap_small(ni, n2) * n1;
          oh[1][a] = wrap_small(nh, n2) * n1;
        } else {
          oi[2][a] = wrap_small(ni, n3) * n12;
          oh[2][a] = wrap_small(nh, n3) * n12;
        }
      }
    }
  }
  R E[3], B[3];
  auto gather6 = [&](auto F, int stride) {
    E[0] = gather_comp<R>(F, wh[0], oh[0], wi[1], oi[1], wi[2], oi[2]);
    E[1] = gather_comp<R>(F + stride, wi[0], oi[0], wh[1], oh[1], wi[2], oi[2]);
    E[2] = gather_comp<R>(F + 2 * stride, wi[0], oi[0], wi[1], oi[1], wh[2], oh[2]);
    B[0] = gather_comp<R>(F + 3 * stride, wi[0], oi[0], wh[1], oh[1], wh[2], oh[2]);
    B[1] = gather_comp<R>(F + 4 * stride, wh[0], oh[0], wi[1], oi[1], wh[2], oh[2]);
    B[2] = gather_comp<R>(F + 5 * stride, wh[0], oh[0], wh[1], oh[1], wi[2], oi[2]);
  };
  if constexpr (Src::local)
    gather6(S.F, S.plane);
  else
    gather6((const R *)r.F, cells);
  boris3<R>(r.qmhdt, E, B, u);
  R v[3];
  velocity3<R>(u, v);
  const R m[3] = {r.dtdx1 * v[0], r.dtdx2 * v[1], r.dtdx3 * v[2]};
  if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(m[0]) && isfinite(m[1]) &&
        isfinite(m[2]))) {
    atomicOr(err, ERR_NUMERIC);
    return cell;
  }
  if (!(fabs(m[0]) < R(1)) || !(fabs(m[1]) < R(1)) || !(fabs(m[2]) < R(1))) {
    atomicOr(err, ERR_RANGE);
    return cell;
  }
  R g[3];
  int dd[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) dd[d] = advance3<R>(f[d], m[d], g[d]);
  deposit3_one(r, K, l, f, dd, g, qw);
  const int j1 = wrap_pow2(g1 + dd[0], n1), j2 = wrap_small(g2 + dd[1], n2),
            j3 = wrap_small(g3 + dd[2], n3);
  const int nc = (j3 << r.sh3) | (j2 << r.log2n1) | j1;
  G(P.cell)[p] = nc;
  G(P.f1)[p] = g[0];
  G(P.f2)[p] = g[1];
  G(P.f3)[p] = g[2];
  G(P.u1)[p] = u[0];
  G(P.u2)[p] = u[1];
  G(P.u3)[p] = u[2];
  return nc;
}

template <class R>
__global__ void __launch_bounds__(256, Push3Occupancy<R>::WAVES_PER_SIMD)
k_push_deposit3(const Run<R> *__restrict__ runs, const Item *__restrict__ items, int parity, int pp,
                int lds_bytes, unsigned *err, unsigned *stats) {
  using SK = Sinks3<R>;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int nbox[6];
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const Parts<R> P = r.pt[pp];
  const int t = it.a;
  const int start = r.tile_start[t], end = r.tile_start[t + 1];
  if (start >= end) return;
  const int n1 = r.n1, n2 = r.n2, n3 = r.n3;
  const int t3 = t / (r.nt1 * r.nt2), t12 = t - t3 * r.nt1 * r.nt2;
  const int t2 = t12 / r.nt1, t1 = t12 - t2 * r.nt1;
  const int ref[3] = {t1 * r.T1, t2 * r.T2, t3 * r.T3};
  const int *box = r.tile_box + 6 * t;
  int lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = box[2 * d];
    hi[d] = box[2 * d + 1];
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      nbox[2 * d] = 1 << 30;
      nbox[2 * d + 1] = -(1 << 30);
    }
    atomicAdd(&stats[STAT_TILES], 1u);
  }
  // current box: cells lo-2 .. hi+3 per axis
  const int W = hi[0] - lo[0] + 6, H = hi[1] - lo[1] + 6, D = hi[2] - lo[2] + 6;
  const long long jn = (long long)W * H * D;
  const size_t need = (size_t)3 * jn * sizeof(typename SK::T);
  int bl[3] = {1 << 30, 1 << 30, 1 << 30}, bh[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  auto track = [&](int cell) {
    int i1, i2, i3;
    unpack3(cell, r.log2n1, r.sh3, n1, i1, i2, i3);
    const int dl[3] = {wrap_delta_pow2_3(i1 - ref[0], n1), wrap_delta_3(i2 - ref[1], n2),
                       wrap_delta_3(i3 - ref[2], n3)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      bl[d] = min(bl[d], dl[d]);
      bh[d] = max(bh[d], dl[d]);
    }
  };
  if (need > (size_t)lds_bytes) {
    // the barrier orders the box initialisation above before every wave's
    // min/max at the end (the LDS branch has its own after the staging)
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&stats[STAT_FALLBACK], 1u);
    const typename SK::G K{(decltype(SK::G::J))G((typename SK::T *)r.J[parity]), n1, n2, n3,
                           n1 * n2, r.cells};
    for (int p = start + threadIdx.x; p < end; p += 256) {
      const int cell = G(P.cell)[p];
      int i1, i2, i3;
      unpack3(cell, r.log2n1, r.sh3, n1, i1, i2, i3);
      const int l[3] = {i1, i2, i3};
      track(push_one3<R>(r, P, p, cell, load_state3(P, p), i1, i2, i3, l, GlobalF3<R>{}, K, err));
    }
  } else {
    typename SK::T *lj = (typename SK::T *)smem_raw;
    const int vol = (int)jn;
    // field box: cells lo-1 .. hi+2 per axis, after the current box when both fit
    const int FW = hi[0] - lo[0] + 4, FH = hi[1] - lo[1] + 4, FD = hi[2] - lo[2] + 4;
    const int fplane = FW * FH * FD;
    const size_t jbytes = (need + 15) & ~(size_t)15;
    const bool use_fl =
        sizeof(R) == 4 && jbytes + (size_t)6 * fplane * sizeof(R) <= (size_t)lds_bytes;
    const lptr3<R> fl = (lptr3<R>)(smem_raw + jbytes);
    // FP32 form: the thread's first particle is loaded before the staging, so
    // that its loads wait out the memory latency together with the staging's
    const int p0 = start + (int)threadIdx.x;
    constexpr bool pre = sizeof(R) == 4;
    int cell0 = 0;
    PState3<R> st0{};
    if (pre && p0 < end) {
      cell0 = G(P.cell)[p0];
      st0 = load_state3(P, p0);
    }
    for (int q = threadIdx.x; q < 3 * vol; q += 256) lj[q] = 0;
    if (use_fl) {
      const gptr<const R> F = G((const R *)r.F);
      const long long cells = r.cells;
      const int o1 = ref[0] + lo[0] - 1, o2 = ref[1] + lo[1] - 1, o3 = ref[2] + lo[2] - 1;
      // one node's six components per pass, all six loads in flight before
      // their LDS stores (a tile stages about 13 values per thread, which one
      // at a time would wait out the memory latency in turn)
      for (int e = threadIdx.x; e < fplane; e += 256) {
        const int k = e / (FW * FH), rem = e - k * FW * FH;
        const int b = rem / FW, a = rem - b * FW;
        const int g3 = wrap_any3(o3 + k, n3), g2 = wrap_any3(o2 + b, n2);
        const long long g = ((long long)g3 * n2 + g2) * n1 + wrap_pow2(o1 + a, n1);
        R v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = F[c * cells + g];
#pragma unroll
        for (int c = 0; c < 6; ++c) fl[c * fplane + e] = v[c];
      }
    }
    __syncthreads();
    const typename SK::L K = SK::L::make(lj, W, W * H, vol);
    const LdsF3<R> SL{fl, FW, FW * FH, fplane};
    for (int p = p0; p < end; p += 256) {
      int cell;
      PState3<R> st;
      if (pre && p == p0) {
        cell = cell0;
        st = st0;
      } else {
        cell = G(P.cell)[p];
        st = load_state3(P, p);
      }
      int i1, i2, i3;
      unpack3(cell, r.log2n1, r.sh3, n1, i1, i2, i3);
      const int l[3] = {wrap_delta_pow2_3(i1 - ref[0], n1) - lo[0] + 2,
                        wrap_delta_3(i2 - ref[1], n2) - lo[1] + 2,
                        wrap_delta_3(i3 - ref[2], n3) - lo[2] + 2};
      if (use_fl)
        track(push_one3<R>(r, P, p, cell, st, i1, i2, i3, l, SL, K, err));
      else
        track(push_one3<R>(r, P, p, cell, st, i1, i2, i3, l, GlobalF3<R>{}, K, err));
    }
    __syncthreads();
    const auto J = G((typename SK::T *)r.J[parity]);
    const int c1 = ref[0] + lo[0] - 2, c2 = ref[1] + lo[1] - 2, c3 = ref[2] + lo[2] - 2;
    auto flush = [&](int q, long long g) {
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const typename SK::T v = lj[comp * vol + q];
        if (v != 0)
          __scoped_atomic_fetch_add(J + comp * (long long)r.cells + g, v, __ATOMIC_RELAXED,
                                    __MEMORY_SCOPE_DEVICE);
      }
    };
    if (W <= 256) {
      // each thread keeps one column a of the box and walks the rows
      // (k, b) = rr, rr + rpp, ... with rpp = 256 / W rows per pass
      const int rpp = 256 / W, rr = (int)threadIdx.x / W, a = (int)threadIdx.x - rr * W;
      if (rr < rpp) {
        const int col = wrap_pow2(c1 + a, n1);
        int k = rr / H, b = rr - k * H;
        for (int row = rr; row < H * D; row += rpp) {
          const int g3 = wrap_any3(c3 + k, n3), g2 = wrap_any3(c2 + b, n2);
          flush(row * W + a, ((long long)g3 * n2 + g2) * n1 + col);
          b += rpp;
          while (b >= H) {
            b -= H;
            ++k;
          }
        }
      }
    } else {
      for (int q = threadIdx.x; q < vol; q += 256) {
        const int k = q / (W * H), rem = q - k * W * H;
        const int b = rem / W, a = rem - b * W;
        const int g3 = wrap_any3(c3 + k, n3), g2 = wrap_any3(c2 + b, n2);
        flush(q, ((long long)g3 * n2 + g2) * n1 + wrap_pow2(c1 + a, n1));
      }
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    bl[d] = wave_min3(bl[d]);
    bh[d] = wave_max3(bh[d]);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicMin(&nbox[2 * d], bl[d]);
      atomicMax(&nbox[2 * d + 1], bh[d]);
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) r.tile_box[6 * t + threadIdx.x] = nbox[threadIdx.x];
}

template <class R>
void Launch<R>::push_deposit3(const Run<R> *runs, const Item *items, int nitems, int parity,
                              int pp, int lds_bytes, unsigned *err, unsigned *stats,
                              hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_push_deposit3<R>, dim3(nitems), dim3(256), lds_bytes, s, runs, items,
                     parity, pp, lds_bytes, err, stats);
}
template void Launch<float>::push_deposit3(const Run<float> *, const Item *, int, int, int, int,
                                           unsigned *, unsigned *, hipStream_t);
template void Launch<double>::push_deposit3(const Run<double> *, const Item *, int, int, int, int,
                                            unsigned *, unsigned *, hipStream_t);

// Charge density in FP64 (diagnostics): rho = qw S1 S2 S3 on the integer
// nodes, from the particles' cells and offsets (either form).
template <class R>
__global__ void k_rho3(const Run<R> *run, int pp, double *rho) {
  const Run<R> &r = *run;
  const Parts<R> &P = r.pt[pp];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  int i1, i2, i3;
  unpack3(P.cell[p], r.log2n1, r.sh3, r.n1, i1, i2, i3);
  double s1[3], s2[3], s3[3];
  const int m1 = dshape3(i1, (double)P.f1[p], s1);
  const int m2 = dshape3(i2, (double)P.f2[p], s2);
  const int m3 = dshape3(i3, (double)P.f3[p], s3);
  const double q = (double)P.qw[p];
  for (int c = 0; c < 3; ++c) {
    const long long pl = (long long)wrap_small(m3 - 1 + c, r.n3) * r.n2;
    for (int b = 0; b < 3; ++b) {
      const long long row = (pl + wrap_small(m2 - 1 + b, r.n2)) * r.n1;
      for (int a = 0; a < 3; ++a)
        unsafeAtomicAdd(rho + row + wrap_pow2(m1 - 1 + a, r.n1), q * s1[a] * s2[b] * s3[c]);
    }
  }
}

template <class R>
void launch_rho3(const Run<R> *run_dev, int pp, int np, double *rho, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_rho3<R>, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, pp, rho);
}
template void launch_rho3<float>(const Run<float> *, int, int, double *, hipStream_t);
template void launch_rho3<double>(const Run<double> *, int, int, double *, hipStream_t);

}  // namespace hp
