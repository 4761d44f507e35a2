// pushc.hip -- 2D push with the cubic particle shape on gfx950: quadratic or
// cubic B-spline form factors of order l (Appendix A; Sec. 4 uses cubic
// shapes against the NCI modes the quadratic shape leaves), here l = 3:
// gather over 4 x 4 nodes (the energy-conserving variant drops to the
// quadratic shape along a component's staggered directions), relativistic
// Boris push, and the Esirkepov deposit over a 5 x 5 window.
//
// One workgroup per particle tile of the periodic tile sort.  The workgroup
// bounds its tile's particle cells, accumulates the current of all of them
// into one LDS box (a move is under a cell: columns and rows -2 .. +3 around
// the cells) and adds the box to the global accumulators at the end; a box
// too large for LDS falls back to global atomics.  FP32 form: integer cubic
// weights with exact sum 2^P and the integer Esirkepov products of the
// quadratic kernel, so 2 (rho_new - rho_old) = div J holds exactly in the
// integers and the sums do not depend on the order; FP64 form: physical
// current in FP64.
#include "hpic_internal.h"

namespace hp {

namespace {

constexpr int CLDS_BYTES = 64512;

template <class T> using lptrc = T __attribute__((address_space(3))) *;

__device__ __forceinline__ int wminc(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wmaxc(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float rsqrtc(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrtc(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcpc(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpc(double x) { return 1.0 / x; }

// Cubic B-spline weights of the nodes m-1, m, m+1, m+2 for a position m + d,
// d in [0, 1): S3 at the distances 1 + d, d, 1 - d, 2 - d.
template <class R>
__device__ __forceinline__ void cubic4(R d, R w[4]) {
  const R e = R(1) - d;
  w[0] = e * e * e * R(1.0 / 6.0);
  w[1] = (R(4) - R(6) * d * d + R(3) * d * d * d) * R(1.0 / 6.0);
  w[2] = (R(4) - R(6) * e * e + R(3) * e * e * e) * R(1.0 / 6.0);
  w[3] = d * d * d * R(1.0 / 6.0);
}
// Quadratic weights on the same four nodes (m-1 .. m+2) for m + d: the nearest
// node is m (d < 1/2) or m + 1.
template <class R>
__device__ __forceinline__ void quad4(R d, R w[4]) {
  const bool up = d >= R(0.5);
  const R q = up ? d - R(1) : d;
  const R a = R(0.5) - q, b = R(0.5) + q;
  const R s0 = R(0.5) * a * a, s1 = R(0.75) - q * q, s2 = R(0.5) * b * b;
  w[0] = up ? R(0) : s0;
  w[1] = up ? s0 : s1;
  w[2] = up ? s1 : s2;
  w[3] = up ? s2 : R(0);
}
// Stencil along one axis for a component with staggering h (0 or 1/2 cell) at
// cell i with offset f: first node and four weights.
template <class R>
__device__ __forceinline__ int stencil4(int i, R f, bool half, bool lower, R w[4]) {
  int m = i;
  R d = f;
  if (half) {
    if (f >= R(0.5)) {
      d = f - R(0.5);
    } else {
      d = f + R(0.5);
      m = i - 1;
    }
  }
  if (lower)
    quad4<R>(d, w);
  else
    cubic4<R>(d, w);
  return m - 1;
}

template <class R>
__device__ __forceinline__ void borisc(R qmhdt, const R E[3], const R B[3], R u[3]) {
  const R e0 = qmhdt * E[0], e1 = qmhdt * E[1], e2 = qmhdt * E[2];
  const R m0 = u[0] + e0, m1 = u[1] + e1, m2 = u[2] + e2;
  const R ig = rsqrtc(R(1) + m0 * m0 + m1 * m1 + m2 * m2);
  const R t0 = qmhdt * B[0] * ig, t1 = qmhdt * B[1] * ig, t2 = qmhdt * B[2] * ig;
  const R sf = R(2) * rcpc(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const R s0 = t0 * sf, s1 = t1 * sf, s2 = t2 * sf;
  const R p0 = m0 + (m1 * t2 - m2 * t1);
  const R p1 = m1 + (m2 * t0 - m0 * t2);
  const R p2 = m2 + (m0 * t1 - m1 * t0);
  u[0] = m0 + (p1 * s2 - p2 * s1) + e0;
  u[1] = m1 + (p2 * s0 - p0 * s2) + e1;
  u[2] = m2 + (p0 * s1 - p1 * s0) + e2;
}

template <class R>
__device__ __forceinline__ int advc(R f, R d, R &g) {
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

// One staggered component: 4 x 4 nodes, stencil origins (c0, r0), weights.
template <class R>
__device__ __forceinline__ R gather_c(const R *__restrict__ F, int n1, int n2, int c0, const R w1[4],
                                      int r0, const R w2[4]) {
  R acc = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const R *row = F + (long long)wrap_small(r0 + b, n2) * n1;
    R s = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) s += w1[a] * row[wrap_pow2(c0 + a, n1)];
    acc += w2[b] * s;
  }
  return acc;
}

// The same from the tile's field box in LDS (row stride FW, box-local first
// nodes c0, r0).
template <class R>
__device__ __forceinline__ R gather_cl(const lptrc<R> Fl, int FW, int c0, const R w1[4], int r0,
                                       const R w2[4]) {
  R acc = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const lptrc<R> row = Fl + (r0 + b) * FW + c0;
    R s = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) s += w1[a] * row[a];
    acc += w2[b] * s;
  }
  return acc;
}

// Integer cubic weights of the nodes m-1 .. m+2 for a position m + d: the
// spline values in FP32 (no contraction, so every call site computes the same
// integers from the same offset) scaled by 2^P and rounded, the node m+1
// taking the remainder, so the four sum to 2^P exactly.  |error| of each is a
// few units of 2^-P.
__device__ __forceinline__ void cubic_fixed(float d, int P, int s[4]) {
#pragma clang fp contract(off)
  const float e = 1.0f - d;
  const float sc = (float)(1 << P) * (1.0f / 6.0f);
  s[0] = (int)rintf(e * e * e * sc);
  s[1] = (int)rintf((4.0f - 6.0f * d * d + 3.0f * d * d * d) * sc);
  s[3] = (int)rintf(d * d * d * sc);
  s[2] = (1 << P) - s[0] - s[1] - s[3];
}

// deposit targets (values already in the accumulator's type)
template <class A>
struct SinkLdsC {
  lptrc<A> box;
  int H, W, c0, r0;  // window origin in the box
  __device__ __forceinline__ void operator()(int comp, int b, int a, A v) const {
    if (v != A(0))
      __hip_atomic_fetch_add(box + (comp * H + (r0 + b)) * W + (c0 + a), v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};
template <class A>
struct SinkGlobC {
  A *J;
  long long cells;
  int n1, n2, c0, r0;  // window origin (global, unwrapped)
  __device__ __forceinline__ void operator()(int comp, int b, int a, A v) const {
    if (v != A(0))
      __hip_atomic_fetch_add(G(J) + comp * cells + (long long)wrap_small(r0 + b, n2) * n1 +
                                 wrap_pow2(c0 + a, n1),
                             v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// FP64 Esirkepov deposit over the 5 x 5 window: J1 = C1 T2 g1, J2 = C2 T1 g2
// (C the running sums of S1 - S0, T = (S0 + S1)/2), J3 = W3 g3.
template <class R, class Sink>
__device__ __forceinline__ void deposit_c(const Sink &put, const R S0x[5], const R S1x[5],
                                          const R S0y[5], const R S1y[5], R g1, R g2, R g3) {
  R C1[5], C2[5], T1[5], T2[5];
  R a1 = 0, a2 = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    a1 = a1 + (S1x[k] - S0x[k]);
    a2 = a2 + (S1y[k] - S0y[k]);
    C1[k] = a1;
    C2[k] = a2;
    T1[k] = R(0.5) * (S0x[k] + S1x[k]);
    T2[k] = R(0.5) * (S0y[k] + S1y[k]);
  }
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (T2[b] == R(0)) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) put(0, b, a, C1[a] * T2[b] * g1);
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    if (T1[a] == R(0)) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) put(1, b, a, C2[b] * T1[a] * g2);
  }
#pragma unroll
  for (int b = 0; b < 5; ++b) {
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const R W3 = S0x[a] * S0y[b] * R(1.0 / 3.0) + S1x[a] * S0y[b] * R(1.0 / 6.0) +
                   S0x[a] * S1y[b] * R(1.0 / 6.0) + S1x[a] * S1y[b] * R(1.0 / 3.0);
      if (W3 != R(0)) put(2, b, a, W3 * g3);
    }
  }
}

// Fixed-point Esirkepov deposit over the 5 x 5 window from integer weights
// with exact sum 2^P: J1 = Q C1[a] A2[b], J2 = Q C2[b] A1[a] (C the running
// sums of S1 - S0, A = S0 + S1) as exact integer products, so the integer
// divergence equals twice the integer change of Q S_x S_y node by node; J3 as
// the quadratic kernel's: rint(x0 t0 + x1 t1), x = S h, t0 = 2 S0y + S1y,
// t1 = S0y + 2 S1y (|value| < 2^31 by the choice of c3).  UNIT: |Q C| and A
// fit 24 signed bits, so each product is one full-rate 24-bit pair.
template <bool UNIT, class Sink>
__device__ __forceinline__ void deposit_cf(const Sink &put, const int S0x[5], const int S1x[5],
                                           const int S0y[5], const int S1y[5], int Q, float h) {
#pragma clang fp contract(off)
  int C1[5], C2[5], A1[5], A2[5];
  int a1 = 0, a2 = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    a1 += S1x[k] - S0x[k];
    a2 += S1y[k] - S0y[k];
    C1[k] = a1;
    C2[k] = a2;
    A1[k] = S0x[k] + S1x[k];
    A2[k] = S0y[k] + S1y[k];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (C1[a] == 0) continue;
    const int qc = UNIT ? mul24_lo(Q, C1[a]) : 0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const long long v = UNIT ? mul24_wide(qc, A2[b])
                               : ((long long)Q * (long long)C1[a]) * (long long)A2[b];
      put(0, b, a, v);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (C2[b] == 0) continue;
    const int qc = UNIT ? mul24_lo(Q, C2[b]) : 0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const long long v = UNIT ? mul24_wide(qc, A1[a])
                               : ((long long)Q * (long long)C2[b]) * (long long)A1[a];
      put(1, b, a, v);
    }
  }
  float x0[5], x1[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    x0[a] = (float)S0x[a] * h;
    x1[a] = (float)S1x[a] * h;
  }
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const float B0 = (float)S0y[b], B1 = (float)S1y[b];
    if (B0 == 0.0f && B1 == 0.0f) continue;
    const float t0 = 2.0f * B0 + B1;
    const float t1 = B0 + 2.0f * B1;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const float p1 = x1[a] * t1;
      const float v = __builtin_fmaf(x0[a], t0, p1);
      put(2, b, a, (long long)(int)rintf(v));
    }
  }
}

template <class R>
__device__ __forceinline__ void place5(const R s[4], int off, R out[5]) {
  out[0] = off ? R(0) : s[0];
  out[1] = off ? s[0] : s[1];
  out[2] = off ? s[1] : s[2];
  out[3] = off ? s[2] : s[3];
  out[4] = off ? s[3] : R(0);
}

}  // namespace

// One workgroup per particle tile (items: run, tile).  The tile's particles
// are bounded first (cells relative to the tile origin, periodic), the
// current box (bounds -2 .. +3) is accumulated in LDS by all of them and added
// to the global accumulators at the end; a box too large for LDS falls back to
// global atomics.  The FP32 form is built for 5 waves per SIMD (96 VGPRs;
// it held 103, i.e. 4 waves, and spills three values off the hot path); the
// FP64 form keeps its registers.
template <class R, bool UNIT, bool EC>
__global__ void __launch_bounds__(256, sizeof(R) == 4 ? 5 : 1) k_push_deposit_cubic(const Run<R> *__restrict__ runs,
                                                            const Item *__restrict__ items,
                                                            int parity, int pp, int lds_bytes,
                                                            unsigned *err) {
  using A = typename AccOf<R>::T;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int red[4][4];
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int t = it.a;
  const int start = r.tile_start[t], end = r.tile_start[t + 1];
  if (start >= end) return;  // the whole workgroup
  const Parts<R> P = r.pt[pp];
  const int n1 = r.n1, n2 = r.n2;
  const int t2i = t / r.nt1, t1i = t - t2i * r.nt1;
  const int ref1 = t1i * r.T1, ref2 = t2i * r.T2;
  auto rel = [&](int c, int &a, int &b) {
    const int i1 = c & (n1 - 1), i2 = c >> r.log2n1;
    a = ((i1 - ref1 + (n1 >> 1)) & (n1 - 1)) - (n1 >> 1);
    int d = i2 - ref2;
    d += d < -(n2 >> 1) ? n2 : 0;
    d -= d >= n2 - (n2 >> 1) ? n2 : 0;
    b = d;
  };
  // ---- bounds of the tile's particle cells
  int lo1 = 1 << 29, hi1 = -(1 << 29), lo2 = 1 << 29, hi2 = -(1 << 29);
  for (int p = start + (int)threadIdx.x; p < end; p += 256) {
    int a, b;
    rel(G(P.cell)[p], a, b);
    lo1 = min(lo1, a);
    hi1 = max(hi1, a);
    lo2 = min(lo2, b);
    hi2 = max(hi2, b);
  }
  lo1 = wminc(lo1);
  hi1 = wmaxc(hi1);
  lo2 = wminc(lo2);
  hi2 = wmaxc(hi2);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[wave][0] = lo1;
    red[wave][1] = hi1;
    red[wave][2] = lo2;
    red[wave][3] = hi2;
  }
  __syncthreads();
  lo1 = min(min(red[0][0], red[1][0]), min(red[2][0], red[3][0])) - 2;
  hi1 = max(max(red[0][1], red[1][1]), max(red[2][1], red[3][1])) + 3;
  lo2 = min(min(red[0][2], red[1][2]), min(red[2][2], red[3][2])) - 2;
  hi2 = max(max(red[0][3], red[1][3]), max(red[2][3], red[3][3])) + 3;
  const int W = hi1 - lo1 + 1, H = hi2 - lo2 + 1;
  // field box: relative cells lo1 .. hi1 - 1 (a stencil reaches cell - 2 .. cell + 2)
  const int FW = W - 1, FH = H - 1;
  const long long jbytes = (3LL * W * H * (long long)sizeof(A) + 15) & ~15LL;
  const bool use_lds = W <= n1 && H <= n2 && jbytes <= lds_bytes;
  const bool use_fl = use_lds && jbytes + 6LL * FW * FH * (long long)sizeof(R) <= lds_bytes;
  const lptrc<A> box = (lptrc<A>)smem_raw;
  const lptrc<R> fl = (lptrc<R>)(smem_raw + jbytes);
  const long long cells = r.cells;
  const R *F = r.F;
  if (use_lds)
    for (int e = threadIdx.x; e < 3 * W * H; e += 256) box[e] = 0;
  if (use_fl) {
    const int plane = FW * FH;
    for (int e = threadIdx.x; e < 6 * plane; e += 256) {
      const int comp = e / plane, q = e - comp * plane;
      const int b = q / FW, a = q - b * FW;
      int g2 = (ref2 + lo2 + b) % n2;
      g2 += g2 < 0 ? n2 : 0;
      fl[e] = G(F)[comp * cells + (long long)g2 * n1 + wrap_pow2(ref1 + lo1 + a, n1)];
    }
  }
  __syncthreads();
  for (int p = start + (int)threadIdx.x; p < end; p += 256) {
    const int cell = G(P.cell)[p];
    const int i1 = cell & (n1 - 1), i2 = cell >> r.log2n1;
    int rel1, rel2;
    rel(cell, rel1, rel2);
    const R f1 = G(P.f1)[p], f2 = G(P.f2)[p];
    R u[3] = {G(P.u1)[p], G(P.u2)[p], G(P.u3)[p]};
    const R qw = G(P.qw)[p];
    // ---- gather: integer (i) and half (h) stencils; EC lowers the order
    // along the staggered directions
    R wi1[4], wh1[4], wi2[4], wh2[4];
    const int ci = stencil4<R>(i1, f1, false, false, wi1);
    const int ch = stencil4<R>(i1, f1, true, EC, wh1);
    const int ri = stencil4<R>(i2, f2, false, false, wi2);
    const int rh = stencil4<R>(i2, f2, true, EC, wh2);
    R E[3], B[3];
    if (use_fl) {
      // box-local first nodes: the stencil starts 1 or 2 cells before the cell
      const int lci = rel1 - lo1 + (ci - i1), lch = rel1 - lo1 + (ch - i1);
      const int lri = rel2 - lo2 + (ri - i2), lrh = rel2 - lo2 + (rh - i2);
      const int plane = FW * FH;
      E[0] = gather_cl<R>(fl, FW, lch, wh1, lri, wi2);
      E[1] = gather_cl<R>(fl + plane, FW, lci, wi1, lrh, wh2);
      E[2] = gather_cl<R>(fl + 2 * plane, FW, lci, wi1, lri, wi2);
      B[0] = gather_cl<R>(fl + 3 * plane, FW, lci, wi1, lrh, wh2);
      B[1] = gather_cl<R>(fl + 4 * plane, FW, lch, wh1, lri, wi2);
      B[2] = gather_cl<R>(fl + 5 * plane, FW, lch, wh1, lrh, wh2);
    } else {
      E[0] = gather_c<R>(F, n1, n2, ch, wh1, ri, wi2);
      E[1] = gather_c<R>(F + cells, n1, n2, ci, wi1, rh, wh2);
      E[2] = gather_c<R>(F + 2 * cells, n1, n2, ci, wi1, ri, wi2);
      B[0] = gather_c<R>(F + 3 * cells, n1, n2, ci, wi1, rh, wh2);
      B[1] = gather_c<R>(F + 4 * cells, n1, n2, ch, wh1, ri, wi2);
      B[2] = gather_c<R>(F + 5 * cells, n1, n2, ch, wh1, rh, wh2);
    }
    borisc<R>(r.qmhdt, E, B, u);
    R v[3];
    {
#pragma clang fp contract(off)
      R s = R(1) + u[0] * u[0];
      s = s + u[1] * u[1];
      s = s + u[2] * u[2];
      const R ig = R(1) / sqrt(s);
      v[0] = u[0] * ig;
      v[1] = u[1] * ig;
      v[2] = u[2] * ig;
    }
    const R m1 = r.dtdx1 * v[0], m2 = r.dtdx2 * v[1];
    if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(m1) && isfinite(m2))) {
      atomicOr(err, ERR_NUMERIC);
      continue;
    }
    if (!(fabs(m1) < R(1)) || !(fabs(m2) < R(1))) {
      atomicOr(err, ERR_RANGE);
      continue;
    }
    R g1, g2;
    const int d1 = advc<R>(f1, m1, g1);
    const int d2 = advc<R>(f2, m2, g2);
    // window: nodes from min(cell_old, cell_new) - 1, five per axis
    const int o1 = min(0, d1), o2 = min(0, d2);  // window origin relative to i - 1
    auto deposit = [&](const auto &K) {
      if constexpr (sizeof(R) == 4) {
        int sa[4], sb[4], S0x[5], S1x[5], S0y[5], S1y[5];
        cubic_fixed(f1, r.P, sa);
        cubic_fixed(g1, r.P, sb);
        place5<int>(sa, 0 - o1, S0x);
        place5<int>(sb, d1 - o1, S1x);
        cubic_fixed(f2, r.P, sa);
        cubic_fixed(g2, r.P, sb);
        place5<int>(sa, 0 - o2, S0y);
        place5<int>(sb, d2 - o2, S1y);
        const float qs = qw * r.inv_wunit;
        const float hv = qs * v[2];
        deposit_cf<UNIT>(K, S0x, S1x, S0y, S1y, (int)rintf(qs), hv * r.c3);
      } else {
        R sa[4], sb[4], S0x[5], S1x[5], S0y[5], S1y[5];
        cubic4<R>(f1, sa);
        cubic4<R>(g1, sb);
        place5<R>(sa, 0 - o1, S0x);
        place5<R>(sb, d1 - o1, S1x);
        cubic4<R>(f2, sa);
        cubic4<R>(g2, sb);
        place5<R>(sa, 0 - o2, S0y);
        place5<R>(sb, d2 - o2, S1y);
        deposit_c<R>(K, S0x, S1x, S0y, S1y, qw * r.jfx1, qw * r.jfx2, qw * v[2]);
      }
    };
    if (use_lds)
      deposit(SinkLdsC<A>{box, H, W, rel1 - 1 + o1 - lo1, rel2 - 1 + o2 - lo2});
    else
      deposit(SinkGlobC<A>{r.J[parity], cells, n1, n2, i1 - 1 + o1, i2 - 1 + o2});
    const int j1 = wrap_pow2(i1 + d1, n1), j2 = wrap_small(i2 + d2, n2);
    G(P.cell)[p] = (j2 << r.log2n1) | j1;
    G(P.f1)[p] = g1;
    G(P.f2)[p] = g2;
    G(P.u1)[p] = u[0];
    G(P.u2)[p] = u[1];
    G(P.u3)[p] = u[2];
  }
  __syncthreads();
  if (use_lds) {
    A *J = r.J[parity];
    for (int e = threadIdx.x; e < 3 * W * H; e += 256) {
      const A v = box[e];
      if (v == A(0)) continue;
      const int cc = e % W, rest = e / W;
      const int rr = rest % H, comp = rest / H;
      const int col = wrap_pow2(ref1 + lo1 + cc, n1);
      int row = (ref2 + lo2 + rr) % n2;
      row += row < 0 ? n2 : 0;
      __hip_atomic_fetch_add(G(J) + comp * cells + (long long)row * n1 + col, v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Charge density of a run's particles with the cubic shape in the deposit's
// units: FP32 form Q S_x S_y with the integer weights of the deposit (so the
// integer continuity check is exact), FP64 form q w S_x S_y.
template <class R>
__global__ void __launch_bounds__(256) k_rho_cubic(const Run<R> *__restrict__ run, int pp,
                                                   typename AccOf<R>::T *rho) {
  const Run<R> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const Parts<R> P = r.pt[pp];
  const int cell = P.cell[p];
  const int i1 = cell & (r.n1 - 1), i2 = cell >> r.log2n1;
  if constexpr (sizeof(R) == 4) {
    int w1[4], w2[4];
    cubic_fixed(P.f1[p], r.P, w1);
    cubic_fixed(P.f2[p], r.P, w2);
    const long long Q = (long long)rintf(P.qw[p] * r.inv_wunit);
    for (int b = 0; b < 4; ++b) {
      const long long row = (long long)wrap_small(i2 - 1 + b, r.n2) * r.n1;
      for (int a = 0; a < 4; ++a) {
        const long long v = Q * (long long)w1[a] * (long long)w2[b];
        if (v != 0)
          atomicAdd((unsigned long long *)(rho + row + wrap_pow2(i1 - 1 + a, r.n1)),
                    (unsigned long long)v);
      }
    }
  } else {
    double w1[4], w2[4];
    cubic4<double>(P.f1[p], w1);
    cubic4<double>(P.f2[p], w2);
    const double q = P.qw[p];
    for (int b = 0; b < 4; ++b) {
      const long long row = (long long)wrap_small(i2 - 1 + b, r.n2) * r.n1;
      for (int a = 0; a < 4; ++a)
        unsafeAtomicAdd(rho + row + wrap_pow2(i1 - 1 + a, r.n1), q * w1[a] * w2[b]);
    }
  }
}

template <class R>
void launch_push_cubic(const Run<R> *runs, const Item *items, int nitems, int parity, int pp,
                       int lds_bytes, bool unit, bool ec, unsigned *err, hipStream_t s) {
  if (nitems <= 0) return;
  lds_bytes = min(lds_bytes, CLDS_BYTES);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(nitems), dim3(256), (size_t)lds_bytes, s, runs, items, parity,
                       pp, lds_bytes, err);
  };
  // UNIT selects the 24-bit integer products of the FP32 form; the FP64 form
  // has no integer products and is instantiated without it
  constexpr bool U = sizeof(R) == 4;
  if (U && unit) {
    if (ec) go(k_push_deposit_cubic<R, U, true>);
    else go(k_push_deposit_cubic<R, U, false>);
  } else {
    if (ec) go(k_push_deposit_cubic<R, false, true>);
    else go(k_push_deposit_cubic<R, false, false>);
  }
}
template <class R>
void launch_rho_cubic(const Run<R> *run_dev, int pp, int np, typename AccOf<R>::T *rho,
                      hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_rho_cubic<R>, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, pp, rho);
}
template void launch_push_cubic<float>(const Run<float> *, const Item *, int, int, int, int, bool,
                                       bool, unsigned *, hipStream_t);
template void launch_push_cubic<double>(const Run<double> *, const Item *, int, int, int, int,
                                        bool, bool, unsigned *, hipStream_t);
template void launch_rho_cubic<float>(const Run<float> *, int, int, long long *, hipStream_t);
template void launch_rho_cubic<double>(const Run<double> *, int, int, double *, hipStream_t);

}  // namespace hp
