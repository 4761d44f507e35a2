// hpic_internal.h -- device-side data layout and helpers of the MI355X hybrid
// Yee-FFT PIC library.  Shared by the kernels (kernels.hip) and the host
// runtime (runtime.cpp); not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hp {

// ---------------------------------------------------------------- types
template <class R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

// Deposit accumulator: 64-bit fixed point for the FP32 form, FP64 otherwise.
template <class R> struct AccOf;
template <> struct AccOf<float> { using T = long long; };
template <> struct AccOf<double> { using T = double; };

// One work item of a batched launch: run index and two item-specific ints.
struct Item {
  int run;
  int a;
  int b;
};

// Particle state (structure of arrays): cell[np] packed cell index
// i1 | i2 << log2n1 | i3 << sh3 (2D: i3 = 0, so the packed index is the
// linear one), f1/f2/f3[np] offsets in [0,1) (f3 only in 3D), u1..u3[np]
// momenta u = gamma v, qw[np] charge times weight, id[np] load index.
template <class R>
struct Parts {
  int *cell, *id;
  R *f1, *f2, *f3, *u1, *u2, *u3, *qw;
};

// Device-side description of one 2D run.  Arrays are owned by the host runtime.
//   pt:  particle buffers, ping-pong for the tile sort (index = particle parity)
//   tiles: T1 x T2 cells each, nt1 x nt2 of them; tile_start[ntiles + 1] is the
//        first particle of each tile after the last sort, tile_cnt[ntiles] the
//        histogram / scatter cursor of the sort; tile_box the bounding box of
//        the cells of each tile's particles (they drift out of the tile
//        between sorts)
//   F:   real-space fields [6][n2][n1] (E1 E2 E3 B1 B2 B3) for the gather
//   Fk:  k-space master copy [6][n2][nk] in FP64 for both forms (ping-pong,
//        index = step parity): the state that carries the field from step to
//        step, so its rounding does not accumulate into a phase drift
//        (FP32 storage of a mode rotated 1000 times drifts by ~1e-5)
//   J:   deposit accumulators [3][n2][n1] (ping-pong, index = step parity)
//   Jk:  corrected, filtered current [3][n2][nk]
template <class R>
struct Run {
  using C = typename Cplx<R>::T;
  using Acc = typename AccOf<R>::T;
  int dim;           // 2 or 3
  int interp;        // 0 momentum-conserving gather, 1 energy-conserving (3D
                     // kernel; the 2D kernel takes it as a template argument)
  int shape;         // particle shape order: 2 quadratic, 3 cubic (2D only)
  int n1, n2, n3, log2n1, nk;
  int sh3;           // 3D: shift of i3 in the packed cell index
  int rows;          // n2 * n3: rows of the x1 transforms
  int cells;         // n1 * rows
  int np;
  int P;             // fixed point: shape factors in units of 2^-P
  float inv_wunit;   // fixed point: integer charge = rint(qw * inv_wunit)
  float c3;          // fixed point: scale of the out-of-plane current
  int unit_charge;   // fixed point: |charge| * 2^P < 2^31, so Q*C products fit 32 bits
  R dt, hdt, idx2;   // dt, dt/2, 1/dx2
  R dtdx1, dtdx2;    // dt/dx1, dt/dx2 (position advance in cells per unit velocity)
  R qmhdt;           // (q/m) dt/2
  R jfx1, jfx2;      // FP64 form: -dx1/dt, -dx2/dt (current of a unit-charge move)
  R idx3, dtdx3, jfx3;  // 3D: 1/dx3, dt/dx3, -dx3/dt
  float cj;          // 3D FP32 form: integer scale of the per-node contributions
  R inv_m;           // 1/M, M = n1/2 (inverse real FFT normalisation)
  double jbgu[3];    // j_bg in accumulator units, added to every node before the
                     // row transform (so the transform sees the drift-free current)
  Parts<R> pt[2];
  int T1, T2, T3, nt1, nt2, nt3, ntiles;
  int *tile_start, *tile_cnt;
  int *tile_box;     // [ntiles][6]: lo1, hi1, lo2, hi2, lo3, hi3 of the tile's particle cells
                     // relative to the tile origin (updated by every push)
  R *F;
  double2 *Fk[2];
  Acc *J[2];
  C *Jk;
  const C *tw;       // [n1]: exp(-2 pi i m / n1)
  const double *sym; // [nk][4]: i k1 xi+ (re, im), i k1 xi- (re, im)
  double mdt, mhdt, midx2, midx3;  // dt, dt/2, 1/dx2, 1/dx3 of the FP64 field update
  const R *jfac;     // [nk][3]: factor on the transformed accumulator per component
};

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cmk(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ double2 cmk(double x, double y) { return make_double2(x, y); }
template <class C> __device__ __forceinline__ C cadd(C a, C b) { return cmk(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return cmk(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class C> __device__ __forceinline__ C cconj(C a) { return cmk(a.x, -a.y); }
template <class C, class R> __device__ __forceinline__ C cscale(C a, R s) { return cmk(a.x * s, a.y * s); }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
template <class C> __device__ __forceinline__ C from_d2(double2 a);
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
// multiply by +i (inv = true) or -i
template <class C> __device__ __forceinline__ C cmuli(C a, bool plus) {
  return plus ? cmk(-a.y, a.x) : cmk(a.y, -a.x);
}

// ---------------------------------------------------------------- LDS FFT
// NF independent complex transforms of length M = 2^log2M stored back to back
// in LDS (buf[f*M + j]), computed by the whole workgroup with Stockham
// auto-sort radix-4 passes and, for odd log2M, a final radix-2 pass.
// tw[m * tws] = exp(-2 pi i m / M); inverse = true uses the conjugate twiddles
// (no 1/M).  MAXB bounds the radix-4 butterflies per thread per pass.
template <class C, int MAXB>
__device__ __forceinline__ void lds_fft(C *buf, int M, int log2M, int NF, const C *__restrict__ tw, int tws,
                        bool inverse, int s0 = 0) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Q = M >> 2;
  const int log2Q = log2M - 2;
  int s = s0;  // log2 of the span Ns already transformed
  for (; s + 2 <= log2M; s += 2) {
    const int Ns = 1 << s;
    C v[MAXB][4];
    int ob[MAXB];
    int cnt = 0;
    const int total = NF * Q;
#pragma unroll
    for (int it = 0; it < MAXB; ++it) {
      const int g = tid + it * nthr;
      if (g < total) {
        const int f = g >> log2Q;
        const int j = g & (Q - 1);
        C *x = buf + f * M;
        const int k = j & (Ns - 1);
        C a0 = x[j], a1 = x[j + Q], a2 = x[j + 2 * Q], a3 = x[j + 3 * Q];
        if (s > 0) {
          // twiddle w^(r k), w = exp(-+2 pi i / (4 Ns)) -> table index r k M / (4 Ns)
          const int e = k << (log2Q - s);
          C t1 = tw[(e)*tws], t2 = tw[(2 * e) * tws], t3 = tw[(3 * e) * tws];
          if (inverse) { t1 = cconj(t1); t2 = cconj(t2); t3 = cconj(t3); }
          a1 = cmul(a1, t1);
          a2 = cmul(a2, t2);
          a3 = cmul(a3, t3);
        }
        const C b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3);
        const C b3 = cmuli(csub(a1, a3), inverse);
        v[it][0] = cadd(b0, b2);
        v[it][1] = cadd(b1, b3);
        v[it][2] = csub(b0, b2);
        v[it][3] = csub(b1, b3);
        ob[it] = f * M + ((j >> s) << (s + 2)) + k;
        cnt = it + 1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXB; ++it) {
      if (it < cnt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) buf[ob[it] + q * Ns] = v[it][q];
      }
    }
    __syncthreads();
  }
  if (s < log2M) {
    // final radix-2 pass: Ns = M/2, in place (each thread owns its pair)
    const int H = M >> 1;
    const int total = NF * H;
    for (int g = tid; g < total; g += nthr) {
      const int f = g >> (log2M - 1);
      const int j = g & (H - 1);
      C *x = buf + f * M;
      C t = tw[j * tws];
      if (inverse) t = cconj(t);
      const C a0 = x[j], a1 = cmul(x[j + H], t);
      x[j] = cadd(a0, a1);
      x[j + H] = csub(a0, a1);
    }
    __syncthreads();
  }
}

// 4-point DFT in place (forward: X_q = sum_r a_r exp(-2 pi i r q / 4)).
template <class C>
__device__ __forceinline__ void dft4(C &a0, C &a1, C &a2, C &a3, bool inverse) {
  const C b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3);
  const C b3 = cmuli(csub(a1, a3), inverse);
  a0 = cadd(b0, b2);
  a1 = cadd(b1, b3);
  a2 = csub(b0, b2);
  a3 = csub(b1, b3);
}
// exp(-2 pi i m / 16) (conjugate for the inverse) of the 16-point DFT's
// inner twiddles, m = r2 q1 in {1, 2, 3, 4, 6, 9}
template <class C>
__device__ __forceinline__ C w16(int m, bool inverse) {
  using R = decltype(C().x);
  const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173);
  const R h = R(0.70710678118654752440);
  R x, y;
  switch (m) {
    case 1: x = c1; y = -s1; break;
    case 2: x = h; y = -h; break;
    case 3: x = s1; y = -c1; break;
    case 4: x = 0; y = -1; break;
    case 6: x = -h; y = -h; break;
    default: x = -c1; y = s1; break;  // 9
  }
  return cmk(x, inverse ? -y : y);
}
// 16-point DFT in registers as 4 x 4: a[r] -> y_q with q = q1 + 4 q2 stored
// at a[4 q1 + q2].
template <class C>
__device__ __forceinline__ void dft16(C a[16], bool inverse) {
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) dft4(a[r2], a[4 + r2], a[8 + r2], a[12 + r2], inverse);
#pragma unroll
  for (int q1 = 1; q1 < 4; ++q1)
#pragma unroll
    for (int r2 = 1; r2 < 4; ++r2) a[4 * q1 + r2] = cmul(a[4 * q1 + r2], w16<C>(r2 * q1, inverse));
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1) dft4(a[4 * q1], a[4 * q1 + 1], a[4 * q1 + 2], a[4 * q1 + 3], inverse);
}
// NF transforms of length M in LDS, radix-16 Stockham passes (one 16-point
// butterfly per thread, all of them held in registers across the barrier)
// while they fit the block, then the radix-4/2 passes of lds_fft.  Same
// result as lds_fft.
template <class C, int MAXB>
__device__ __forceinline__ void lds_fft16(C *buf, int M, int log2M, int NF, const C *__restrict__ tw, int tws,
                          bool inverse) {
  int s = 0;
  if (NF * (M >> 4) <= (int)blockDim.x) {
    const int Q = M >> 4, log2Q = log2M - 4, g = threadIdx.x;
    for (; s + 4 <= log2M; s += 4) {
      const int Ns = 1 << s;
      C v[16];
      int ob = 0;
      const bool act = g < NF * Q;
      if (act) {
        const int f = g >> log2Q, j = g & (Q - 1), k = j & (Ns - 1);
        const C *x = buf + f * M;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = x[j + r * Q];
        if (s > 0) {
          // twiddle w^(r k), w = exp(-+2 pi i / (16 Ns)): table index r k M / (16 Ns)
          const int e = k << (log2Q - s);
#pragma unroll
          for (int r = 1; r < 16; ++r) {
            C t = tw[(r * e) * tws];
            if (inverse) t = cconj(t);
            v[r] = cmul(v[r], t);
          }
        }
        dft16(v, inverse);
        ob = f * M + ((j >> s) << (s + 4)) + k;
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
          for (int q2 = 0; q2 < 4; ++q2) buf[ob + (q1 + 4 * q2) * Ns] = v[4 * q1 + q2];
      }
      __syncthreads();
    }
  }
  lds_fft<C, MAXB>(buf, M, log2M, NF, tw, tws, inverse, s);
}

// NF transforms of length M in LDS (as lds_fft), one transform at a time when
// the radix-4 passes of all NF at once would need more than MAXB butterflies
// per thread (n1 = 8192 rows: three components of M = 4096).  The choice is
// uniform over the block, so the barriers inside stay uniform.
template <class C, int MAXB>
__device__ __forceinline__ void lds_fft_rows(C *buf, int M, int log2M, int NF, const C *__restrict__ tw, int tws,
                             bool inverse) {
  if (NF * (M >> 2) <= MAXB * (int)blockDim.x) {
    lds_fft16<C, MAXB>(buf, M, log2M, NF, tw, tws, inverse);
    return;
  }
  for (int f = 0; f < NF; ++f) lds_fft16<C, MAXB>(buf + f * M, M, log2M, 1, tw, tws, inverse);
}

// ---------------------------------------------------------------- shapes
// Quadratic B-spline weights of the nodes m-1, m, m+1 for a particle at signed
// distance d in [-1/2, 1/2) from its nearest node m.
template <class R> __device__ __forceinline__ void spline3(R d, R w[3]) {
  const R a = R(0.5) - d, b = R(0.5) + d;
  w[0] = R(0.5) * a * a;
  w[1] = R(0.75) - d * d;
  w[2] = R(0.5) * b * b;
}
// Linear B-spline on the same three nodes (energy-conserving gather along a
// staggered direction): for d in [-1/2, 1/2) the weights of m-1, m, m+1.
template <class R> __device__ __forceinline__ void line3(R d, R w[3]) {
  w[0] = d < R(0) ? -d : R(0);
  w[1] = R(1) - (d < R(0) ? -d : d);
  w[2] = d > R(0) ? d : R(0);
}
// Weights of a half-node (staggered) stencil: quadratic, or linear for the
// energy-conserving gather.
template <class R> __device__ __forceinline__ void half3(R d, R w[3], bool ec) {
  if (ec)
    line3<R>(d, w);
  else
    spline3<R>(d, w);
}

// Quantised quadratic shape of one coordinate (cell + FP32 offset): integers
// s[0..2] of the nodes m-1, m, m+1 with exact sum 2^P; returns m.  The same
// definition as the FP32-precision reference deposit:
//   s[0] = floor(((2^(P-1) - D)^2 + 2^P) / 2^(P+1)), s[2] likewise with +D,
// D = rint(d 2^P).  SMALL (P <= 22): the square is a full-rate 24-bit
// multiply pair and floor((x^2 + 2^P) / 2^(P+1)) is evaluated as
// (floor(x^2 / 2^P) + 1) >> 1, which is the same integer.
template <bool SMALL>
__device__ __forceinline__ int fixed_shape(int cell, float f, int P, int s[3]) {
  const int up = (f >= 0.5f) ? 1 : 0;
  const float d = up ? (f - 1.0f) : f;             // exact
  const float scaled = d * (float)(1 << P);         // exact
  const int D = (int)rintf(scaled);                 // |D| <= 2^(P-1)
  const int h = 1 << (P - 1);
  const int lo = h - D, hi = h + D;                 // in [0, 2^P]
  if (SMALL) {
    const unsigned long long l2 = (unsigned long long)(unsigned)(lo & 0xffffff) * (unsigned)(lo & 0xffffff);
    const unsigned long long h2 = (unsigned long long)(unsigned)(hi & 0xffffff) * (unsigned)(hi & 0xffffff);
    const unsigned ql = __builtin_amdgcn_alignbit((unsigned)(l2 >> 32), (unsigned)l2, (unsigned)P);
    const unsigned qh = __builtin_amdgcn_alignbit((unsigned)(h2 >> 32), (unsigned)h2, (unsigned)P);
    s[0] = (int)((ql + 1u) >> 1);
    s[2] = (int)((qh + 1u) >> 1);
  } else {
    const long long bias = 1ll << P;
    s[0] = (int)(((long long)lo * lo + bias) >> (P + 1));
    s[2] = (int)(((long long)hi * hi + bias) >> (P + 1));
  }
  s[1] = (1 << P) - s[0] - s[2];
  return cell + up;
}

// Exact product of two integers in [-2^23, 2^23) as a 64-bit value.  The
// explicit sign extension from 24 bits lets the compiler select the full-rate
// v_mul_i32_i24 / v_mul_hi_i32_i24 pair.
__device__ __forceinline__ long long mul24_wide(int a, int b) {
  return (long long)((a << 8) >> 8) * (long long)((b << 8) >> 8);
}
// Product of two integers in [-2^23, 2^23) whose value fits 32 bits: one
// v_mul_i32_i24 (written out, as the compiler otherwise folds the sign
// extensions into a quarter-rate 32-bit multiply).
__device__ __forceinline__ int mul24_lo(int a, int b) {
  int r;
  asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Nearest integer (ties to even) of |v| < 2^51 as a 64-bit integer: adding
// 1.5 2^52 rounds v to an integer held in the low mantissa bits (one FP64 add
// and one 64-bit subtract instead of the multi-instruction FP64 -> int64
// conversion).
__device__ __forceinline__ long long rint_i64(double v) {
#pragma clang fp contract(off)
  const double t = v + 6755399441055744.0;
  return __double_as_longlong(t) - 0x4338000000000000LL;
}

// Global-memory view of a pointer held in a descriptor: lets the compiler use
// global (not flat) loads, stores and atomics.
template <class T> using gptr = T __attribute__((address_space(1))) *;
template <class T> __device__ __forceinline__ gptr<T> G(T *p) { return (gptr<T>)p; }

__device__ __forceinline__ int wrap_pow2(int i, int n) { return i & (n - 1); }
__device__ __forceinline__ int wrap_small(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

// Wave-aggregated atomic add of 1 per lane to cnt[key]: lanes with equal keys
// share one atomic; returns the lane's rank among the previous value and its
// peers (so the result equals a per-lane atomicAdd(cnt + key, 1) up to the
// order among peers).
__device__ __forceinline__ int wave_atomic_inc(int *cnt, int key, bool active) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(active);
  int result = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lk = __shfl(key, leader);
    const unsigned long long same = __ballot(active && key == lk) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt + lk, __popcll(same));
    base = __shfl(base, leader);
    if (active && key == lk) result = base + __popcll(same & ((1ull << lane) - 1));
    todo &= ~same;
  }
  return result;
}

// Error bits of the device error word.
enum : unsigned { ERR_RANGE = 1u, ERR_NUMERIC = 2u };

// Statistics words of the push kernel: [0] tiles that fell back to global
// memory (bounding box too large for LDS), [1] tiles processed.
enum { STAT_FALLBACK = 0, STAT_TILES = 1, NSTAT = 2 };

// LDS of one push+deposit workgroup: staged fields (24 B per node in FP32,
// 48 B in FP64) and current accumulators (3 x 8 B per node).  The budget is
// set per handle from the tile shape (push_lds_bytes), between the minimum
// and maximum here.
constexpr int KSTRIP = 8;  // rows per thread of the 2D k-space update
constexpr int PUSH_THREADS = 256;
constexpr int PUSH_BATCH = 4;  // particles loaded per thread before pushing
constexpr int PUSH_LDS_MIN = 16384;
constexpr int PUSH_LDS_MAX = 64512;  // with the static LDS, under 64 KiB
// The 3D push of the FP32 form runs 3 waves per SIMD (register budget 168,
// three workgroups per compute unit), so its LDS budget is a third of the
// compute unit's 160 KiB less the static LDS; the FP64 form runs 2 (budget
// 256 registers: left alone the compiler takes 259 and gets 1 wave).
constexpr int PUSH3_LDS_MAX_FP32 = 53248;
template <class R> struct Push3Occupancy { static constexpr int WAVES_PER_SIMD = 2; };
template <> struct Push3Occupancy<float> { static constexpr int WAVES_PER_SIMD = 3; };

// ---------------------------------------------------------------- launches
// Host-side launch wrappers (kernels.hip), one instantiation per precision.
template <class R>
struct Launch {
  // unit: every run's charges satisfy the 24-bit product bound (FP32 form);
  // ec: energy-conserving gather (all runs of a handle share it)
  static void push_deposit(const Run<R> *runs, const Item *items, int nitems, int parity,
                           int pp, int lds_bytes, bool unit, bool ec, unsigned *err,
                           unsigned *stats, hipStream_t s);
  // tile sort of the particles of all runs: items are (run, first particle,
  // count) chunks; per_run lists (run, 0, 0) once per run.  scramble = true
  // spreads the particles of one cell over a tile's slots (for input in cell
  // order); false keeps the arrival order, so the scatter writes are coalesced
  static void sort(const Run<R> *runs, const Item *chunks, int nchunks, const Item *per_run,
                   int nruns, int pp, bool scramble, hipStream_t s);
  // row transforms: ncomp = 3 components per block (item = run, row[, group])
  // or 1 (item = run, row, component) for long rows
  static void fft_j(const Run<R> *runs, const Item *items, int nitems, int parity, int maxM,
                    int ncomp, hipStream_t s);
  static void kupdate(const Run<R> *runs, const Item *items, int nitems, int parity,
                      hipStream_t s);
  // 3D: the same update as two passes (E and the half-step B, then B)
  static void kupdate3(const Run<R> *runs, const Item *items, int nitems, int parity,
                       hipStream_t s);
  static void push_deposit3(const Run<R> *runs, const Item *items, int nitems, int parity,
                            int pp, int lds_bytes, unsigned *err, unsigned *stats,
                            hipStream_t s);
  static void ifft_eb(const Run<R> *runs, const Item *items, int nitems, int parity, int maxM,
                      int ncomp, hipStream_t s);
  static void fields_to_k(const Run<R> *runs, const Item *items, int nitems, int parity,
                          int maxM, int ncomp, hipStream_t s);
};


// Diagnostics and helpers (FP64 unless noted).
// 3D: charge density in FP64 from the particle state (any form).
template <class R>
void launch_rho3(const Run<R> *run_dev, int pp, int np, double *rho, hipStream_t s);
// 3D Gauss residual per row (i2, i3) of the k-space master copy; rows_out [rows][3].
template <class R>
void launch_gauss3(const Run<R> *run_dev, int rows, int n1, int parity, const double *rho,
                   const double2 *tw64, const double *sym64, const double *filt, double idx2,
                   double idx3, double *rows_out, hipStream_t s);
// 3D continuity residual max |(rho_n - rho_o)/dt + div j| with j = fac[d] * J.
template <class A>
void launch_cont3(const double *rn, const double *ro, const A *J, int n1, int n2, int n3,
                  double dt, double f1, double f2, double f3, double idx1, double idx2,
                  double idx3, double *partial, int nblocks, hipStream_t s);
void launch_rho_fixed(const Run<float> *run_dev, int pp, int np, long long *rho, hipStream_t s);
// 2D with the cubic shape: push + deposit (items: run, tile; unit: every
// run's |charge| 2^P fits the 24-bit products), and the charge density in the
// deposit's units (FP32 form: integers, FP64 form: physical)
template <class R>
void launch_push_cubic(const Run<R> *runs, const Item *items, int nitems, int parity, int pp,
                       int lds_bytes, bool unit, bool ec, unsigned *err, hipStream_t s);
template <class R>
void launch_rho_cubic(const Run<R> *run_dev, int pp, int np, typename AccOf<R>::T *rho,
                      hipStream_t s);
void launch_rho_fp64(const Run<double> *run_dev, int pp, int np, double *rho, hipStream_t s);
// Moving antenna of a 2D run (see hp_set_antenna): device parameters.
struct AntennaDev {
  int run;             // run index in the handle
  int n1, n2;
  double dx1, dx2, dt;
  double x0, v, t0, T, K0, omega, phase, x2c, waist;
  double scale;        // physical j3 -> accumulator units
};
// Adds every antenna's current of the step (time (*step + 1/2) dt) to j3 of
// the run's accumulators of the given parity; then, in a separate launch,
// the step counter advances by one (both are captured in step graphs).
template <class R>
void launch_antenna(const Run<R> *runs, const AntennaDev *ants, int nant, int maxn2, int parity,
                    const long long *step, hipStream_t s);
void launch_step_tick(long long *step, hipStream_t s);
template <class R>
void launch_energy(const R *F, long long cells, double *partial, int nblocks, hipStream_t s);
template <class R>
void launch_kinetic(const Run<R> *run_dev, int pp, double *partial, int nblocks, hipStream_t s);
// Gauss residual per row: rho (physical, FP64, [n2][n1]) and the k-space E1,E2
// of a run; writes per-row [3]: sum |R|^2, max |R|, sum |f rho|^2.
template <class R>
void launch_gauss(const Run<R> *run_dev, int n2, int n1, int parity, const double *rho,
                  const double2 *tw64, const double *sym64, const double *filt, double idx2,
                  double *rows_out, hipStream_t s);
void launch_cont_fixed(const long long *rho_new, const long long *rho_old, const long long *J,
                       int n1, int n2, long long *partial_max, int nblocks, hipStream_t s);
void launch_cont_fp64(const double *rho_new, const double *rho_old, const double *J, int n1,
                      int n2, double dt, double idx1, double idx2, double *partial_max,
                      int nblocks, hipStream_t s);
void launch_debug_deposit(int n1, int n2, int P, float inv_wunit, float c3, int np,
                          const int *cell0, const float *off0, const int *cell1,
                          const float *off1, const float *v3, const float *qw, long long *J,
                          unsigned *err, hipStream_t s);
template <class R>
void launch_inverse_rows(const typename Cplx<R>::T *Xk, int nk, int n1, int nrows,
                         const typename Cplx<R>::T *tw, R scale, R *out, hipStream_t s);

// ---------------------------------------------------------------- device I/O
// (io.hip) Geometry of a Cartesian run for loading particles from FP64 device
// arrays: box lengths L = n dx, cell sizes, packing of the cell index.
struct LoadGeom {
  int dim, n1, n2, n3, log2n1, sh3;
  double L[3], dx[3];
};
// Validation pass over n particles (x[dim][n], u[3][n], w[n] in device memory):
// *bad |= 1 for a non-finite input, count[cells] += particles per cell,
// qbits[0] = max and qbits[1] = min of |(R)(q w)| as FP64 bit patterns.
template <class R>
void launch_scan_particles(const LoadGeom &g, long long n, const double *x, const double *u,
                           const double *w, double q, int *count, unsigned long long *qbits,
                           unsigned *bad, hipStream_t s);
void launch_max_int(const int *a, long long n, int *out, hipStream_t s);
template <class A>
void launch_current_out(const A *raw, long long n, double f, double bg, double *out, hipStream_t s);
template <class R>
void launch_real_to_double(const R *in, long long n, double *out, hipStream_t s);
void launch_zero_i64(long long *p, long long n, hipStream_t s);
// Conversion pass: the run's structure of arrays A in input order.
template <class R>
void launch_load_particles(const LoadGeom &g, long long n, const double *x, const double *u,
                           const double *w, double q, Parts<R> A, hipStream_t s);
// The run's particle state (buffer pp, current order) into device buffers.
template <class R>
void launch_unload_particles(const Run<R> *run_dev, int pp, int np, int *cell, R *off, R *u, R *qw,
                             int *id, hipStream_t s);

}  // namespace hp
