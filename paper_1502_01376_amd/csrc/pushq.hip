// pushq.hip -- particle side of the quasi-3D (r-z with azimuthal modes) step
// on gfx950: field gather from the modes, relativistic Boris push in Cartesian
// momenta, and the per-mode charge-conserving deposit (Sec. 5 runs the hybrid
// solver per mode; the particle scheme is that of the cited quasi-3D method).
//
// Mode convention F(z, r, th) = sum_m Re(F_m(z, r) e^{i m th}); the phase of a
// particle is P_m = e^{-i m th} = ((x - i y)/r)^m.  Node weights are quadratic
// B-spline products in (z, r) cell units.  The stencil row below the axis
// (row -1) is the mirror point of row 1 (integer-r nodes) or row 0 (half-r
// nodes): z components and scalars of mode m carry (-1)^m there, r and th
// components -(-1)^m.
//
// Deposit of one move (W^0, P^0) -> (W^1, P^1), per mode, with c_0 = 1 and
// c_m = 2: W^1 P^1 - W^0 P^0 = (W^1 - W^0)(P^0 + P^1)/2 + (W^0 + W^1)/2 (P^1 - P^0).
// The first part is split into z and r face fluxes by the Esirkepov
// decomposition in (z, r) index space with the mean phase (separable: the
// running sum of the shape change along one axis times the mean shape along
// the other), the second is an azimuthal flux i c_m q w Wbar (P^1 - P^0) / m.
// Where continuity sets no azimuthal current (m = 0, and m = 1 on the axis
// node) the azimuthal current is deposited directly from the azimuthal
// velocity with the time-averaged weight W3.  Ghost-row fold factors:
// (-1)^m for the z and azimuthal fluxes, -(-1)^m for the flux through the face
// at -dr/2 (it lands on the face at +dr/2) and for the direct azimuthal
// current.  The accumulators hold charge per step (flux times dt), scaled by
// wscale; the row-transform kernel converts them to current densities with
// the face areas and node volumes.
//
// One thread per particle; each wave accumulates into an LDS box (global
// atomics if its particles spread too far), then adds the box to the global
// accumulators.  The deposit's arithmetic (shapes, phases and fluxes of the
// stored positions, their radius and direction in R) is FP64 in both forms;
// the FP32 form rounds each contribution once to a 64-bit integer on a fine
// scale (2^40 per unit charge), so the sums do not depend on the order and
// continuity holds to about 2^-41 of a particle's charge per node and step.  (With FP32 weights and a 2^28 scale, long
// drifting-beam runs grew a spurious k1 = 0 mode.)
#include "hpic_q3d.h"

namespace hp {

namespace {

__device__ __forceinline__ float rsqrtq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrtq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcpq(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpq(double x) { return 1.0 / x; }

template <class R>
__device__ __forceinline__ void splineq(R d, R w[3]) {
  const R a = R(0.5) - d, b = R(0.5) + d;
  w[0] = R(0.5) * a * a;
  w[1] = R(0.75) - d * d;
  w[2] = R(0.5) * b * b;
}

// Floor for the small non-negative arguments used here (r/dr + 1/2 >= 0).
template <class R> __device__ __forceinline__ int ifloorq(R x) { return (int)floor(x); }

// r / dr of a transverse position given as cells + offsets, as its nearest
// integer node m and the offset d = r/dr - m, and the direction (c, s).  The
// offset is formed from the exact integer part of (r/dr)^2 - m^2, so it keeps
// the resolution of the stored offsets anywhere in the column: with
// S = (ix + fx)^2 + (iy + fy)^2, d = (S - m^2) / (r/dr + m).
template <class R>
__device__ __forceinline__ void radial(int ix, R fx, int iy, R fy, int &m, R &d, R &c, R &s) {
#pragma clang fp contract(off)
  const int si = ix * ix + iy * iy;
  const R sf = fx * (R(2 * ix) + fx) + fy * (R(2 * iy) + fy);
  const R rho0 = sqrt(fmax(R(si) + sf, R(0)));
  m = (int)floor(rho0 + R(0.5));
  const R X = R(ix) + fx, Y = R(iy) + fy;
  // within half a cell of the axis ix, iy are 0 or -1 and X, Y are exact
  d = m == 0 ? sqrt(X * X + Y * Y) : (R(si - m * m) + sf) / (rho0 + R(m));
  const R rho = R(m) + d;
  c = rho > R(0) ? X / rho : R(1);
  s = rho > R(0) ? Y / rho : R(0);
}

// New offset in [0,1) and cell shift in {-1, 0, 1} after a move d (|d| < 1).
template <class R>
__device__ __forceinline__ int advq(R f, R d, R &g) {
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

template <class R>
__device__ __forceinline__ void borisq(R qmhdt, const R E[3], const R B[3], R u[3]) {
  const R e0 = qmhdt * E[0], e1 = qmhdt * E[1], e2 = qmhdt * E[2];
  const R m0 = u[0] + e0, m1 = u[1] + e1, m2 = u[2] + e2;
  const R ig = rsqrtq(R(1) + m0 * m0 + m1 * m1 + m2 * m2);
  const R t0 = qmhdt * B[0] * ig, t1 = qmhdt * B[1] * ig, t2 = qmhdt * B[2] * ig;
  const R sf = R(2) * rcpq(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const R s0 = t0 * sf, s1 = t1 * sf, s2 = t2 * sf;
  const R p0 = m0 + (m1 * t2 - m2 * t1);
  const R p1 = m1 + (m2 * t0 - m0 * t2);
  const R p2 = m2 + (m0 * t1 - m1 * t0);
  u[0] = m0 + (p1 * s2 - p2 * s1) + e0;
  u[1] = m1 + (p2 * s0 - p0 * s2) + e1;
  u[2] = m2 + (p0 * s1 - p1 * s0) + e2;
}

// Quadratic shape of a coordinate given as cell + offset f in [0,1) along z:
// nodes n-1, n, n+1 around the nearest node n = cell + (f >= 1/2).
template <class R>
__device__ __forceinline__ int zshape(int cell, R f, R s[3]) {
  const int up = f >= R(0.5);
  splineq<R>(f - R(up), s);
  return cell + up;
}
// The same along r for rho = r/dr >= 0 (integer-r nodes).
template <class R>
__device__ __forceinline__ int rshape(R rho, R s[3]) {
  const int n = ifloorq<R>(rho + R(0.5));
  splineq<R>(rho - R(n), s);
  return n;
}
template <class R>
__device__ __forceinline__ void place4(const R s[3], int off, R out[4]) {
  out[0] = off ? R(0) : s[0];
  out[1] = off ? s[0] : s[1];
  out[2] = off ? s[1] : s[2];
  out[3] = off ? s[2] : R(0);
}

// One mode of one staggered component at the particle: the complex
// interpolated value (vx, vy) from weights wz/wr, node columns oz[3] and rows
// rr[3] (a ghost row already mirrored; ghost0: row 0 of the stencil is the
// ghost, whose sign depends on the mode parity and on whether the component is
// a z component or a transverse one).  F points at the mode's plane of the
// component, in global memory (row stride n1) or in a wave's LDS copy of the
// fields around its particles (row stride the box width, columns relative to
// the box).
template <class R, class PC, class I>
__device__ __forceinline__ void gather_q(PC F, const R wz[3], const int oz[3], const R wr[3],
                                         const int rr[3], bool ghost0, bool odd, bool vec,
                                         I rowstride, R &vx, R &vy) {
  vx = 0;
  vy = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const PC row = F + rr[b] * rowstride;
    R sx = 0, sy = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const auto v = row[oz[a]];
      sx += wz[a] * v.x;
      sy += wz[a] * v.y;
    }
    R w = wr[b];
    if (b == 0 && ghost0 && odd != vec) w = -w;  // (-1)^m for z components, -(-1)^m for r, th
    vx += w * sx;
    vy += w * sy;
  }
}

// LDS of one push workgroup: a private region per wave of WAVE_CAP 64-bit
// accumulators (the wave's particles are consecutive, hence close together).
// FP32 form: three workgroups per compute unit (3 waves per SIMD, the register
// budget 168); FP64 form: two.
template <class R> struct QPush;
template <> struct QPush<float> {
  static constexpr int LDS = 53248;
  static constexpr int WAVES_PER_SIMD = 3;
};
template <> struct QPush<double> {
  static constexpr int LDS = 64512;
  static constexpr int WAVES_PER_SIMD = 2;
};

__device__ __forceinline__ int wmin(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wmax(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
template <class T> using lptr = T __attribute__((address_space(3))) *;
// A complex value as a clang vector (copyable to and from LDS).
template <class R> struct LdsC;
template <> struct LdsC<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct LdsC<double> { typedef double T __attribute__((ext_vector_type(2))); };

// One FP64 contribution in the accumulator's type: FP32 form the nearest 64-bit
// integer (|v| < 2^44: charges are scaled to at most 2^40 and every weight
// factor is at most 4 in magnitude), FP64 form the value.
template <class A> __device__ __forceinline__ A to_acc(double v);
template <> __device__ __forceinline__ long long to_acc<long long>(double v) {
  return rint_i64(v);
}
template <> __device__ __forceinline__ double to_acc<double>(double v) { return v; }

// Deposit targets: the wave's LDS box, or the global accumulators.
template <class A>
struct SinkLdsQ {
  lptr<A> box;
  int H, W, rlo, z0, per;  // z0: box column of global column 0 of the window frame
  int bzrel;               // box column of the window's first column
  __device__ __forceinline__ void window(int bz) { bzrel = bz + z0; }
  // the window's first node in row `row` of accumulator (c, m, part); the
  // nodes of the row are then immediate offsets
  using Row = lptr<A>;
  __device__ __forceinline__ Row row(int c, int m, int part, int row) const {
    const int slot = c * per + (m == 0 ? 0 : 2 * m - 1 + part);
    return box + (__mul24(__mul24(slot, H) + (row - rlo), W) + bzrel);
  }
  __device__ __forceinline__ void put(Row r, int a, double v) const {
    const A q = to_acc<A>(v);
    if (q != A(0)) __hip_atomic_fetch_add(r + a, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};
template <class A>
struct SinkGlobQ {
  A *J;
  long long plane;
  int n1, col[4];
  __device__ __forceinline__ void window(int bz) {
#pragma unroll
    for (int a = 0; a < 4; ++a) col[a] = wrap_pow2(bz + a, n1);
  }
  using Row = gptr<A>;
  __device__ __forceinline__ Row row(int c, int m, int part, int row) const {
    return G(J) + ((long long)(m * 3 + c) * plane + (long long)row * n1) * 2 + part;
  }
  __device__ __forceinline__ void put(Row r, int a, double v) const {
    const A q = to_acc<A>(v);
    if (q != A(0))
      __hip_atomic_fetch_add(r + 2 * col[a], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};
__device__ __forceinline__ void glob_add(gptr<long long> p, long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void glob_add(gptr<double> p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-mode deposit of one move (see the file header): window shapes S0/S1
// along z and r, their running sums C and means T, window row base br, the
// old and new directions (cta, sta), (ctb, stb) (phases P_m = (c - i s)^m by
// the same recurrence for both, so the new phase of one step is bit for bit
// the old phase of the next), scaled charge g and v_th dt.
template <int MC, class R, class Sink>
__device__ __forceinline__ void deposit_q(const Sink &put, int M, const R S0z[4], const R S1z[4],
                                          const R S0r[4], const R S1r[4], const R Cz[4],
                                          const R Tz[4], const R Cr[4], const R Tr[4], int br,
                                          R cta, R sta, R ctb, R stb, R g, R vthdt) {
#pragma clang fp contract(off)
  R P0r = 1, P0i = 0;  // phase at the old position
  R P1r = 1, P1i = 0;  // phase at the new position
  if (MC > 0) M = MC;
  for (int m = 0; m < M; ++m) {
    if (m > 0) {
      const R t0 = P0r * cta + P0i * sta;
      P0i = P0i * cta - P0r * sta;
      P0r = t0;
      const R t = P1r * ctb + P1i * stb;
      P1i = P1i * ctb - P1r * stb;
      P1r = t;
    }
    const R cm = m == 0 ? R(1) : R(2);
    const bool odd = m & 1;
    const R Pmr = R(0.5) * (P0r + P1r), Pmi = R(0.5) * (P0i + P1i);
    const R qr = -cm * g * Pmr, qi = -cm * g * Pmi;
    // z faces
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int row = br + b;
      R f = Tr[b];
      if (row < 0) {
        row = -row;
        if (odd) f = -f;
      }
      if (f == R(0)) continue;
      const auto r0 = put.row(0, m, 0, row), r1 = put.row(0, m, 1, row);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R w = Cz[a] * f;
        put.put(r0, a, qr * w);
        if (m > 0) put.put(r1, a, qi * w);
      }
    }
    // r faces (face j at (j + 1/2) dr; face -1 lands on face 0)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      int face = br + b;
      R f = Cr[b];
      if (face < 0) {
        face = 0;
        if (!odd) f = -f;
      }
      if (f == R(0)) continue;
      const auto r0 = put.row(1, m, 0, face), r1 = put.row(1, m, 1, face);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const R w = Tz[a] * f;
        if (w == R(0)) continue;
        put.put(r0, a, qr * w);
        if (m > 0) put.put(r1, a, qi * w);
      }
    }
    // azimuthal current
    const R dPr = P1r - P0r, dPi = P1i - P0i;
    const R inv_m = m > 0 ? R(1) / R(m) : R(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int row = br + b;
      const bool ghost = row < 0;
      if (ghost) row = -row;
      const bool direct = m == 0 || (m == 1 && row == 0);
      if (!direct && row == 0) continue;
      const auto r0 = put.row(2, m, 0, row), r1 = put.row(2, m, 1, row);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (direct) {
          const R W3 = S0z[a] * S0r[b] * R(1.0 / 3.0) + S1z[a] * S0r[b] * R(1.0 / 6.0) +
                       S0z[a] * S1r[b] * R(1.0 / 6.0) + S1z[a] * S1r[b] * R(1.0 / 3.0);
          if (W3 == R(0)) continue;
          R sv = cm * g * W3 * vthdt;
          if (ghost && !odd) sv = -sv;  // -(-1)^m
          put.put(r0, a, sv * Pmr);
          if (m > 0) put.put(r1, a, sv * Pmi);
        } else {
          const R Wb = R(0.5) * (S0z[a] * S0r[b] + S1z[a] * S1r[b]);
          if (Wb == R(0)) continue;
          R sv = cm * g * Wb * inv_m;
          if (ghost && odd) sv = -sv;  // (-1)^m
          // i sv dP
          put.put(r0, a, -sv * dPi);
          put.put(r1, a, sv * dPr);
        }
      }
    }
  }
}

// Deposit of one move from the particle's old and new positions: cell cz
// with z offset fz, moved by dz cells to offset gz; radial nodes mri, mrb with
// offsets dri, drb; old and new directions; scaled charge g; v_th dt.  Builds
// the 4-node windows along z and r holding both stencils, their running sums
// and means, and deposits through K (whose column origin follows the window).
template <int MC, class Sink>
__device__ __forceinline__ void deposit_move(Sink K, int M, int cz, double fz, int dz, double gz,
                                             int mri, double dri, int mrb, double drb, double ct,
                                             double st, double ctb, double stb, double g,
                                             double vthdt) {
  using D = double;
  D S0z[4], S1z[4], S0r[4], S1r[4];
  int bz, br;
  {
    D sa[3], sb[3];
    const int na = zshape<D>(cz, fz, sa);
    const int nb = zshape<D>(cz + dz, gz, sb);
    bz = min(na, nb) - 1;
    place4<D>(sa, na - 1 - bz, S0z);
    place4<D>(sb, nb - 1 - bz, S1z);
    splineq<D>(dri, sa);
    splineq<D>(drb, sb);
    br = min(mri, mrb) - 1;
    place4<D>(sa, mri - 1 - br, S0r);
    place4<D>(sb, mrb - 1 - br, S1r);
  }
  D Cz[4], Tz[4], Cr[4], Tr[4];
  {
    D az = 0, ar = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      az = az + (S1z[k] - S0z[k]);
      ar = ar + (S1r[k] - S0r[k]);
      Cz[k] = az;
      Cr[k] = ar;
      Tz[k] = 0.5 * (S0z[k] + S1z[k]);
      Tr[k] = 0.5 * (S0r[k] + S1r[k]);
    }
  }
  K.window(bz);
  deposit_q<MC, D>(K, M, S0z, S1z, S0r, S1r, Cz, Tz, Cr, Tr, br, ct, st, ctb, stb, g, vthdt);
}

// The rare global-atomic path out of line, with plain arguments (no array
// whose address is taken), so that it adds neither registers nor scratch
// memory to the LDS path.
template <class A>
__device__ __noinline__ void deposit_move_global(A *J, long long plane, int n1, int M, int cz,
                                                 double fz, int dz, double gz, int mri, double dri,
                                                 int mrb, double drb, double ct, double st,
                                                 double ctb, double stb, double g, double vthdt) {
  SinkGlobQ<A> K;
  K.J = J;
  K.plane = plane;
  K.n1 = n1;
  deposit_move<0>(K, M, cz, fz, dz, gz, mri, dri, mrb, drb, ct, st, ctb, stb, g, vthdt);
}

}  // namespace

// One thread per particle (items: run, first particle of 256).  Each wave
// bounds the deposit footprint of its 64 particles before the push (a move is
// less than a cell: columns cz-2 .. cz+3, rows m-2 .. m+2 around the nearest
// integer-r node m, ghost rows folded onto rows 0 and 1).  In the FP32 form
// its LDS region first holds a copy of the fields its particles gather; then,
// if the box fits, the region is its current box, added to the global
// accumulators at the end; otherwise the wave deposits with global atomics.
// MC: the mode count when every run of the launch has it (the gather's mode
// loop is then unrolled and the deposit's has a constant trip count), or 0.
template <class R, int MC>
__global__ void __launch_bounds__(256, QPush<R>::WAVES_PER_SIMD)
    k_q_push_deposit(const RunQ<R> *__restrict__ runs, const Item *__restrict__ items, int parity,
                     unsigned *err) {
  using C = typename Cplx<R>::T;
  using A = typename AccQ<R>::T;
  extern __shared__ unsigned char smem_raw[];
  constexpr int WAVE_CAP = QPush<R>::LDS / 4 / 8;
  const Item it = items[blockIdx.x];
  const RunQ<R> &r = runs[it.run];
  const int p0 = it.a + threadIdx.x;
  const bool active = p0 < r.np;
  // inactive lanes shadow the run's last particle, which lies in their wave's
  // box whenever the wave has an active lane
  const int p = active ? p0 : r.np - 1;
  const PartsQ<R> P = r.pt;
  const int n1 = r.n1, M = MC > 0 ? MC : r.M;
  const long long plane = r.plane;
  const int cz = G(P.cell)[p], ix = G(P.ix)[p], iy = G(P.iy)[p];
  const R fz = G(P.fz)[p], fx = G(P.fx)[p], fy = G(P.fy)[p];
  R u[3] = {G(P.uz)[p], G(P.ux)[p], G(P.uy)[p]};
  const R qw = G(P.qw)[p];
  // nearest integer-r node mri with offset dri, nearest half-r node (j + 1/2)
  // mrh with offset drh, direction (ct, st)
  int mri;
  R dri, ct, st;
  radial<R>(ix, fx, iy, fy, mri, dri, ct, st);
  const int mrh = dri >= R(0) ? mri : mri - 1;
  const R drh = dri >= R(0) ? dri - R(0.5) : dri + R(0.5);
  // ---- the wave's deposit box (relative z columns, absolute rows)
  const int NS = 3 * (2 * M - 1);  // accumulator slots per node
  const int cz0 = __shfl(cz, 0);
  const int relz = ((cz - cz0 + (n1 >> 1)) & (n1 - 1)) - (n1 >> 1);
  const int zlo = wmin(active ? relz : (1 << 29)) - 2;
  const int zhi = wmax(active ? relz : -(1 << 29)) + 3;
  const int rlo = max(0, wmin(active ? mri : (1 << 29)) - 2);
  const int rhi = wmax(active ? mri : -(1 << 29)) + 2;
  const int W = zhi - zlo + 1, H = rhi - rlo + 1;
  const bool any = zhi >= zlo;
  const bool use_lds = any && W <= n1 && (long long)W * H * NS <= WAVE_CAP;
  const lptr<A> box = (lptr<A>)smem_raw + (threadIdx.x >> 6) * WAVE_CAP;
  const int lane = threadIdx.x & 63;
  const C *F = r.F;
  // FP32 form: before the push the wave's LDS region holds a copy of the
  // fields its particles gather (all modes and components over columns
  // relz - 1 .. relz + 2 and rows rlo .. rhi - 1), laid out
  // [mode][component][row][column]
  constexpr bool STAGE = sizeof(R) == 4;
  const int fzlo = zlo + 1, Wf = W - 2, Hf = H - 1;
  const bool use_fl = STAGE && any && Wf <= 64 &&
                      (long long)6 * M * Wf * Hf * (long long)sizeof(C) <=
                          (long long)WAVE_CAP * (long long)sizeof(A);
  using V2 = typename LdsC<R>::T;
  const lptr<V2> fbox =
      (lptr<V2>)smem_raw + (threadIdx.x >> 6) * (int)(WAVE_CAP * sizeof(A) / sizeof(V2));
  if constexpr (STAGE) {
    if (use_fl) {
      // lane -> (row in a group of rpi rows, column)
      const int rpi = 64 / Wf, sub = lane / Wf, cc = lane - sub * Wf;
      const int col = wrap_pow2(cz0 + fzlo + cc, n1);
      // a mode's six components per pass, all six loads in flight before
      // their LDS stores
      if (sub < rpi)
        for (int r0 = sub; r0 < Hf; r0 += rpi) {
          const long long ro = (long long)(rlo + r0) * n1 + col;
          for (int m = 0; m < M; ++m) {
            C v[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] = F[(long long)(6 * m + c) * plane + ro];
#pragma unroll
            for (int c = 0; c < 6; ++c) fbox[((6 * m + c) * Hf + r0) * Wf + cc] = V2{v[c].x, v[c].y};
          }
        }
    }
  } else {
    if (use_lds)
      for (int e = lane; e < W * H * NS; e += 64) box[e] = 0;
  }
  __syncthreads();
  // ---- gather: integer (i) and half (h) stencils along z and r
  R wzi[3], wzh[3], wri[3], wrh[3];
  int ozi[3], ozh[3], rri[3], rrh[3];
  const int upz = fz >= R(0.5);
  splineq<R>(fz - R(upz), wzi);
  half3<R>(fz - R(0.5), wzh, r.interp != 0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ozi[a] = wrap_pow2(cz + upz - 1 + a, n1);
    ozh[a] = wrap_pow2(cz - 1 + a, n1);
  }
  splineq<R>(dri, wri);
  half3<R>(drh, wrh, r.interp != 0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int ji = mri - 1 + b, jh = mrh - 1 + b;
    rri[b] = ji < 0 ? -ji : ji;
    rrh[b] = jh < 0 ? -jh - 1 : jh;
  }
  const bool gi = mri == 0, gh = mrh == 0;  // ghost row in the stencil
  // sum over the modes of Re(F_m e^{i m th}), with P_m = (ct - i st)^m by
  // recurrence
  R Ec[3] = {0, 0, 0}, Bc[3] = {0, 0, 0};
  R Pr = 1, Pi = 0;
  constexpr int MU = MC > 0 ? MC : 1;
#pragma unroll MU
  for (int m = 0; m < M; ++m) {
    if (m > 0) {
      const R t = Pr * ct + Pi * st;
      Pi = Pi * ct - Pr * st;
      Pr = t;
    }
    const bool odd = m & 1;
    R vx[6], vy[6];
    if (use_fl) {
      // the same stencils in box coordinates
      int lzi[3], lzh[3], lri[3], lrh[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lzi[a] = relz - fzlo + upz - 1 + a;
        lzh[a] = relz - fzlo - 1 + a;
        lri[a] = rri[a] - rlo;
        lrh[a] = rrh[a] - rlo;
      }
      const int fp = Wf * Hf;
      const lptr<V2> fb = fbox + 6 * m * fp;
      gather_q<R>(fb, wzh, lzh, wri, lri, gi, odd, false, Wf, vx[0], vy[0]);
      gather_q<R>(fb + fp, wzi, lzi, wrh, lrh, gh, odd, true, Wf, vx[1], vy[1]);
      gather_q<R>(fb + 2 * fp, wzi, lzi, wri, lri, gi, odd, true, Wf, vx[2], vy[2]);
      gather_q<R>(fb + 3 * fp, wzi, lzi, wrh, lrh, gh, odd, false, Wf, vx[3], vy[3]);
      gather_q<R>(fb + 4 * fp, wzh, lzh, wri, lri, gi, odd, true, Wf, vx[4], vy[4]);
      gather_q<R>(fb + 5 * fp, wzh, lzh, wrh, lrh, gh, odd, true, Wf, vx[5], vy[5]);
    } else {
      const long long rs = n1;
      const C *Fm = F + 6 * m * plane;
      gather_q<R>(Fm, wzh, ozh, wri, rri, gi, odd, false, rs, vx[0], vy[0]);
      gather_q<R>(Fm + plane, wzi, ozi, wrh, rrh, gh, odd, true, rs, vx[1], vy[1]);
      gather_q<R>(Fm + 2 * plane, wzi, ozi, wri, rri, gi, odd, true, rs, vx[2], vy[2]);
      gather_q<R>(Fm + 3 * plane, wzi, ozi, wrh, rrh, gh, odd, false, rs, vx[3], vy[3]);
      gather_q<R>(Fm + 4 * plane, wzh, ozh, wri, rri, gi, odd, true, rs, vx[4], vy[4]);
      gather_q<R>(Fm + 5 * plane, wzh, ozh, wrh, rrh, gh, odd, true, rs, vx[5], vy[5]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Ec[c] += vx[c] * Pr + vy[c] * Pi;  // Re(v e^{i m th}) with P = e^{-i m th}
      Bc[c] += vx[c + 3] * Pr + vy[c + 3] * Pi;
    }
  }
  if constexpr (STAGE) {
    // the region becomes the wave's current box
    __syncthreads();
    if (use_lds)
      for (int e = lane; e < W * H * NS; e += 64) box[e] = 0;
    __syncthreads();
  }
  const R E[3] = {Ec[0], Ec[1] * ct - Ec[2] * st, Ec[1] * st + Ec[2] * ct};
  const R B[3] = {Bc[0], Bc[1] * ct - Bc[2] * st, Bc[1] * st + Bc[2] * ct};
  borisq<R>(r.qmhdt, E, B, u);
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
  // moves in cells
  const R mz = r.dtdz * v[0], mx = r.dtdr * v[1], my = r.dtdr * v[2];
  bool ok = active;
  if (ok && !(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(mz) && isfinite(mx) &&
              isfinite(my))) {
    atomicOr(err, ERR_NUMERIC);
    ok = false;
  }
  R gz = fz, gx = fx, gy = fy;
  int dz = 0, dx = 0, dy = 0, mrb = mri;
  R drb = dri, ctb = ct, stb = st;
  if (ok) {
    if (!(fabs(mz) < R(1)) || !(fabs(mx) < R(1)) || !(fabs(my) < R(1))) {
      atomicOr(err, ERR_RANGE);
      ok = false;
    } else {
      dz = advq<R>(fz, mz, gz);
      dx = advq<R>(fx, mx, gx);
      dy = advq<R>(fy, my, gy);
      radial<R>(ix + dx, gx, iy + dy, gy, mrb, drb, ctb, stb);
      // within the wall margin, and less than a cell in r (the deposit window
      // and the wave's box assume it)
      const R dmove = R(mrb - mri) + (drb - dri);
      if (!(R(mrb) + drb < r.rmax) || !(fabs(dmove) < R(1)) || abs(mrb - mri) > 1) {
        atomicOr(err, ERR_RANGE);
        ok = false;
      }
    }
  }
  if (ok) {
    // the new state first (fewer values live across the deposit)
    G(P.cell)[p] = wrap_pow2(cz + dz, n1);
    G(P.fz)[p] = gz;
    G(P.ix)[p] = ix + dx;
    G(P.fx)[p] = gx;
    G(P.iy)[p] = iy + dy;
    G(P.fy)[p] = gy;
    G(P.uz)[p] = u[0];
    G(P.ux)[p] = u[1];
    G(P.uy)[p] = u[2];
    // ---- deposit (FP64)
    using D = double;
    // azimuthal velocity at the mid point times dt: the move (mx, my) dr
    // projected on the azimuthal direction of the mid point
    const D xmid = D(ix) + (D)fx + 0.5 * (D)mx, ymid = D(iy) + (D)fy + 0.5 * (D)my;
    const D rmid = sqrt(xmid * xmid + ymid * ymid);
    const D vthdt = rmid > 0.0 ? (xmid * (D)my - ymid * (D)mx) / rmid * (D)r.dr : 0.0;
    const D g = (D)qw * (D)r.wscale;
    if (use_lds) {
      SinkLdsQ<A> K{box, H, W, rlo, relz - cz - zlo, 2 * M - 1, 0};
      deposit_move<MC>(K, M, cz, (D)fz, dz, (D)gz, mri, (D)dri, mrb, (D)drb, (D)ct, (D)st, (D)ctb,
                   (D)stb, g, vthdt);
    } else {
      deposit_move_global<A>(r.J[parity], plane, n1, M, cz, (D)fz, dz, (D)gz, mri, (D)dri, mrb,
                             (D)drb, (D)ct, (D)st, (D)ctb, (D)stb, g, vthdt);
    }
  }
  __syncthreads();
  if (use_lds) {
    A *J = r.J[parity];
    const int per = 2 * M - 1;
    if (W <= 64) {
      // each lane keeps one column of the box and walks its rows, slot by
      // slot (box layout [slot][row][column])
      const int rpi = 64 / W, sub = lane / W, cc = lane - sub * W;
      if (sub < rpi) {
        const int col = wrap_pow2(cz0 + zlo + cc, n1);
        for (int slot = 0; slot < NS; ++slot) {
          const int c = slot / per, s2 = slot - c * per;
          const int m = (s2 + 1) >> 1, part = s2 == 0 ? 0 : (s2 - 1) & 1;
          const auto Jb = G(J) + (long long)(m * 3 + c) * plane * 2 + part;
          for (int r0 = sub; r0 < H; r0 += rpi) {
            const A v = box[(slot * H + r0) * W + cc];
            if (v != A(0)) glob_add(Jb + ((long long)(rlo + r0) * n1 + col) * 2, v);
          }
        }
      }
    } else {
      for (int e = lane; e < W * H * NS; e += 64) {
        const A v = box[e];
        if (v == A(0)) continue;
        const int cc = e % W, rest = e / W;
        const int row = rlo + rest % H, slot = rest / H;
        const int c = slot / per, s2 = slot - c * per;
        const int m = (s2 + 1) >> 1, part = s2 == 0 ? 0 : (s2 - 1) & 1;
        const int col = wrap_pow2(cz0 + zlo + cc, n1);
        glob_add(G(J) + ((long long)(m * 3 + c) * plane + (long long)row * n1 + col) * 2 + part, v);
      }
    }
  }
}

// FP64 charge density of a run's particles (any form), added into rho.
template <class R>
__global__ void __launch_bounds__(256) k_q_rho(const RunQ<R> *__restrict__ run, int M,
                                               double2 *rho) {
  const RunQ<R> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const PartsQ<R> P = r.pt;
  const int n1 = r.n1;
  const double f = G(P.fz)[p], qw = G(P.qw)[p];
  const double x = (double)G(P.ix)[p] + (double)G(P.fx)[p];
  const double y = (double)G(P.iy)[p] + (double)G(P.fy)[p];
  const int cz = G(P.cell)[p];
  const double rr = sqrt(x * x + y * y);  // r / dr
  const double ct = rr > 0 ? x / rr : 1.0, st = rr > 0 ? y / rr : 0.0;
  double wz[3], wr[3];
  const int nz = zshape<double>(cz, f, wz);
  const int nr0 = rshape<double>(rr, wr);
  const double PI_ = 3.14159265358979323846;
  double Pr = 1, Pi = 0;
  for (int m = 0; m < M; ++m) {
    if (m > 0) {
      const double t = Pr * ct + Pi * st;
      Pi = Pi * ct - Pr * st;
      Pr = t;
    }
    const double cm = m == 0 ? 1.0 : 2.0;
    for (int b = 0; b < 3; ++b) {
      int row = nr0 - 1 + b;
      double s = cm * qw * wr[b];
      if (row < 0) {
        row = -row;
        if (m & 1) s = -s;
      }
      const double V = row == 0 ? 0.25 * PI_ * r.dr * r.dr * r.dz : 2.0 * PI_ * row * r.dr * r.dr * r.dz;
      for (int a = 0; a < 3; ++a) {
        double *o = (double *)(rho + (long long)m * r.plane + (long long)row * n1 +
                               wrap_pow2(nz - 1 + a, n1));
        const double w = s * wz[a] / V;
        atomicAdd(o, w * Pr);
        if (m > 0) atomicAdd(o + 1, w * Pi);
      }
    }
  }
}

// Co-drifting background current: jbg[j] -= q w v_z S_r / (n1 dz A_j).
template <class R>
__global__ void __launch_bounds__(256) k_q_jbg(const RunQ<R> *__restrict__ run, double *jbg) {
  const RunQ<R> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const PartsQ<R> P = r.pt;
  const double qw = G(P.qw)[p];
  const double x = (double)G(P.ix)[p] + (double)G(P.fx)[p];
  const double y = (double)G(P.iy)[p] + (double)G(P.fy)[p];
  const double uz = G(P.uz)[p], ux = G(P.ux)[p], uy = G(P.uy)[p];
  const double vz = uz / sqrt(1.0 + uz * uz + ux * ux + uy * uy);
  const double rr = sqrt(x * x + y * y);  // r / dr
  double wr[3];
  const int n0 = rshape<double>(rr, wr);
  const double PI_ = 3.14159265358979323846;
  for (int b = 0; b < 3; ++b) {
    int row = n0 - 1 + b;
    if (row < 0) row = -row;
    const double A = row == 0 ? 0.25 * PI_ * r.dr * r.dr : 2.0 * PI_ * row * r.dr * r.dr;
    atomicAdd(jbg + row, -qw * vz * wr[b] / ((double)r.n1 * r.dz * A));
  }
}

// ---------------------------------------------------------------- sort
// The particles of a wave come from consecutive storage slots; the loader
// stores them by (z column, radial row), and a periodic counting sort by bins
// of sbz columns x sbr rows keeps a wave's particles, and so its field copy
// and its current box, compact as they move.  Order within a bin is the
// order of the atomics: the FP32 form's integer deposit does not depend on it.
template <class R>
__device__ __forceinline__ int q_sort_bin(const RunQ<R> &r, const PartsQ<R> &P, int p) {
  const float x = (float)G(P.ix)[p] + (float)G(P.fx)[p];
  const float y = (float)G(P.iy)[p] + (float)G(P.fy)[p];
  const int j = min(max((int)sqrtf(x * x + y * y), 0), r.n2 - 1);
  return (G(P.cell)[p] / r.sbz) * r.nbr + j / r.sbr;
}

template <class R>
__global__ void k_q_sort_clear(const RunQ<R> *__restrict__ run) {
  const RunQ<R> &r = *run;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= r.nbins; i += gridDim.x * blockDim.x)
    r.sbin[i] = 0;
}

template <class R>
__global__ void __launch_bounds__(256) k_q_sort_count(const RunQ<R> *__restrict__ run) {
  const RunQ<R> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = p < r.np;
  // neighbours in storage share bins: one atomic per distinct bin of a wave
  const int b = active ? q_sort_bin<R>(r, r.pt, p) : 0;
  const int rank = wave_atomic_inc(r.sbin, b, active);
  if (!active) return;
  r.skey[p] = b;
  r.srank[p] = rank;
}

// Exclusive prefix sum of the bin counts in three launches: each block of
// 1024 threads scans its 1024 bins in LDS and records their sum; one block
// scans the block sums (a contiguous chunk per thread, then across threads);
// every block adds its offset.
__device__ __forceinline__ int block_scan_incl(int v, int *part) {
  const int t = threadIdx.x;
  part[t] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int w = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += w;
    __syncthreads();
  }
  return part[t];
}

template <class R>
__global__ void __launch_bounds__(1024) k_q_scan_local(const RunQ<R> *__restrict__ run) {
  __shared__ int part[1024];
  const RunQ<R> &r = *run;
  const int i = blockIdx.x * 1024 + threadIdx.x;
  const int v = i < r.nbins ? r.sbin[i] : 0;
  const int inc = block_scan_incl(v, part);
  if (i < r.nbins) r.sbin[i] = inc - v;
  if (threadIdx.x == 1023) r.ssum[blockIdx.x] = inc;
}

template <class R>
__global__ void __launch_bounds__(1024) k_q_scan_sums(const RunQ<R> *__restrict__ run) {
  __shared__ int part[1024];
  const RunQ<R> &r = *run;
  const int n = (r.nbins + 1023) / 1024, t = threadIdx.x;
  const int chunk = (n + 1023) / 1024, lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += r.ssum[i];
  int run_sum = block_scan_incl(sum, part) - sum;  // exclusive prefix of this chunk
  for (int i = lo; i < hi; ++i) {
    const int c = r.ssum[i];
    r.ssum[i] = run_sum;
    run_sum += c;
  }
  if (t == 1023) r.sbin[r.nbins] = part[1023];
}

template <class R>
__global__ void __launch_bounds__(1024) k_q_scan_add(const RunQ<R> *__restrict__ run) {
  const RunQ<R> &r = *run;
  const int i = blockIdx.x * 1024 + threadIdx.x;
  if (i < r.nbins) r.sbin[i] += r.ssum[blockIdx.x];
}

template <class R>
__global__ void __launch_bounds__(256) k_q_sort_scatter(const RunQ<R> *__restrict__ run) {
  const RunQ<R> &r = *run;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.np) return;
  const int d = r.sbin[r.skey[p]] + r.srank[p];
  const PartsQ<R> &A = r.pt, &B = r.pt2;
  G(B.cell)[d] = G(A.cell)[p];
  G(B.ix)[d] = G(A.ix)[p];
  G(B.iy)[d] = G(A.iy)[p];
  G(B.id)[d] = G(A.id)[p];
  G(B.fz)[d] = G(A.fz)[p];
  G(B.fx)[d] = G(A.fx)[p];
  G(B.fy)[d] = G(A.fy)[p];
  G(B.uz)[d] = G(A.uz)[p];
  G(B.ux)[d] = G(A.ux)[p];
  G(B.uy)[d] = G(A.uy)[p];
  G(B.qw)[d] = G(A.qw)[p];
}

template <class R>
__global__ void k_q_sort_swap(RunQ<R> *run) {
  const PartsQ<R> t = run->pt;
  run->pt = run->pt2;
  run->pt2 = t;
}

template <class R>
void LaunchQ<R>::sort(RunQ<R> *run_dev, int np, int nbins, hipStream_t s) {
  if (np <= 0 || nbins <= 0) return;
  const int pb = (np + 255) / 256;
  hipLaunchKernelGGL(k_q_sort_clear<R>, dim3(std::min((nbins + 256) / 256, 1024)), dim3(256), 0, s,
                     run_dev);
  hipLaunchKernelGGL(k_q_sort_count<R>, dim3(pb), dim3(256), 0, s, run_dev);
  const int sb = (nbins + 1023) / 1024;
  hipLaunchKernelGGL(k_q_scan_local<R>, dim3(sb), dim3(1024), 0, s, run_dev);
  hipLaunchKernelGGL(k_q_scan_sums<R>, dim3(1), dim3(1024), 0, s, run_dev);
  hipLaunchKernelGGL(k_q_scan_add<R>, dim3(sb), dim3(1024), 0, s, run_dev);
  hipLaunchKernelGGL(k_q_sort_scatter<R>, dim3(pb), dim3(256), 0, s, run_dev);
  hipLaunchKernelGGL(k_q_sort_swap<R>, dim3(1), dim3(1), 0, s, run_dev);
}

template <class R>
void LaunchQ<R>::push_deposit(const RunQ<R> *runs, const Item *items, int nitems, int parity,
                              int modes, unsigned *err, hipStream_t s) {
  if (nitems <= 0) return;
  // kernels with the mode loops unrolled for the common mode counts
  auto k = modes == 2 ? k_q_push_deposit<R, 2> : modes == 3 ? k_q_push_deposit<R, 3>
                                                            : k_q_push_deposit<R, 0>;
  hipLaunchKernelGGL(k, dim3(nitems), dim3(256), (size_t)QPush<R>::LDS, s, runs, items, parity, err);
}
template <class R>
void LaunchQ<R>::rho(const RunQ<R> *run_dev, int np, int M, double2 *rho, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_q_rho<R>, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, M, rho);
}
template <class R>
void LaunchQ<R>::jbg(const RunQ<R> *run_dev, int np, double *jbg, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_q_jbg<R>, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, jbg);
}

template void LaunchQ<float>::push_deposit(const RunQ<float> *, const Item *, int, int, int,
                                           unsigned *, hipStream_t);
template void LaunchQ<double>::push_deposit(const RunQ<double> *, const Item *, int, int, int,
                                            unsigned *, hipStream_t);
template void LaunchQ<float>::sort(RunQ<float> *, int, int, hipStream_t);
template void LaunchQ<double>::sort(RunQ<double> *, int, int, hipStream_t);
template void LaunchQ<float>::rho(const RunQ<float> *, int, int, double2 *, hipStream_t);
template void LaunchQ<double>::rho(const RunQ<double> *, int, int, double2 *, hipStream_t);
template void LaunchQ<float>::jbg(const RunQ<float> *, int, double *, hipStream_t);
template void LaunchQ<double>::jbg(const RunQ<double> *, int, double *, hipStream_t);

}  // namespace hp
