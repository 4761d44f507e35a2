// solve.hip -- field side of the hybrid Yee-FFT PIC step on gfx950.
//
// After the particle push and deposit (push.hip), a step runs: fft_j (FFT of j
// along x1, current correction of Eq. (11) and the low-pass filter of Sec. 4),
// kupdate (hybrid Maxwell update of Eqs. (12)-(17) in (k1, x2) space) and
// ifft_eb (inverse FFT of E and B for the next gather).  Every launch is
// batched over all runs of a handle through a work-item list.  FP64
// diagnostics (energies, Gauss and continuity residuals) live here too.
#include "hpic_internal.h"
#include "hpic_update3.h"

namespace hp {

// =====================================================================
// FFT of the current along x1, correction and filter
// =====================================================================

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

// One workgroup per (run, row): the three current components of the row
// (ncomp = 3), or per (run, row, component) for long rows (ncomp = 1, item.b
// the component), so that a block's LDS stays small enough for several
// blocks per CU.
template <class R, int MAXB>
__global__ void __launch_bounds__(256) k_fft_j(const Run<R> *__restrict__ runs,
                                               const Item *__restrict__ items, int parity,
                                               int ncomp) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int row = it.a;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, cells = r.cells;
  const auto *Jin = r.J[parity];
  auto *Jz = r.J[parity ^ 1];
  const int cb = ncomp == 3 ? 0 : it.b;
  for (int cc = 0; cc < ncomp; ++cc) {
    const long long base = (long long)(cb + cc) * cells + (long long)row * n1;
    // the uniform background is added per node in FP64 before the conversion:
    // for a drifting plasma it cancels the bulk current, so that the FP32
    // transform (FP32 form) rounds relative to the current's fluctuation
    const double bg = r.jbgu[cb + cc];
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
      const R x0 = (R)((double)Jin[base + 2 * n] + bg);
      const R x1 = (R)((double)Jin[base + 2 * n + 1] + bg);
      lds[cc * M + n] = cmk(x0, x1);
      Jz[base + 2 * n] = 0;
      Jz[base + 2 * n + 1] = 0;
    }
  }
  __syncthreads();
  lds_fft_rows<C, MAXB>(lds, M, log2M, ncomp, r.tw, 2, false);
  const int nk = r.nk;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    const C Wk = r.tw[k], Wmk = r.tw[mk];
    for (int cc = 0; cc < ncomp; ++cc) {
      const int c = cb + cc;
      const C Zk = lds[cc * M + k];
      const C Zmk = lds[cc * M + (mk & (M - 1))];
      C Xk = r2c_post(Zk, Zmk, Wk);
      const R fk = r.jfac[k * 3 + c];
      Xk = cscale(Xk, fk);
      C *out = r.Jk + (long long)c * r.rows * nk + (long long)row * nk;
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
// master (initialisation).  Item = (run, row, group): group g covers 3g..3g+2
// (ncomp = 3), or (run, row, component) (ncomp = 1).
template <class R, int MAXB>
__global__ void __launch_bounds__(256) k_fields_to_k(const Run<R> *__restrict__ runs,
                                                     const Item *__restrict__ items, int parity,
                                                     int ncomp) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int row = it.a, cb = ncomp == 3 ? 3 * it.b : it.b;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, cells = r.cells, nk = r.nk;
  for (int cc = 0; cc < ncomp; ++cc) {
    const R *src = r.F + (long long)(cb + cc) * cells + (long long)row * n1;
    for (int n = threadIdx.x; n < M; n += blockDim.x) lds[cc * M + n] = cmk(src[2 * n], src[2 * n + 1]);
  }
  __syncthreads();
  lds_fft_rows<C, MAXB>(lds, M, log2M, ncomp, r.tw, 2, false);
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int cc = 0; cc < ncomp; ++cc) {
      const C Zk = lds[cc * M + k];
      const C Zmk = lds[cc * M + (mk & (M - 1))];
      double2 *out = r.Fk[parity] + (long long)(cb + cc) * r.rows * nk + (long long)row * nk;
      out[k] = to_d2(r2c_post(Zk, Zmk, r.tw[k]));
      if (mk != k) out[mk] = to_d2(r2c_post(Zmk, Zk, r.tw[mk]));
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
// 2D update, one thread per (strip of KSTRIP rows, kappa1): the thread walks
// its rows in order, keeping the previous row's half-step B and new E in
// registers, so each input row is read once per strip (plus the rows just
// outside it) instead of up to four times.  Row j needs E^n on rows j-1 .. j+2,
// B^{n+1/2} on rows j-1 .. j+1 and E^{n+1} on rows j and j+1; every value is
// computed by the same expressions as for a single row.
template <class R>
__global__ void __launch_bounds__(256) k_kupdate(const Run<R> *__restrict__ runs,
                                                 const Item *__restrict__ items, int parity) {
  using C = double2;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int nk = r.nk, n2 = r.n2;
  const int nstrips = (n2 + KSTRIP - 1) / KSTRIP;
  const int e = it.a + threadIdx.x;
  if (e >= nstrips * nk) return;
  const int strip = e / nk, k = e - strip * nk;
  const int q0 = strip * KSTRIP, q1 = min(q0 + KSTRIP, n2);  // output rows q0 .. q1-1
  const long long plane = (long long)n2 * nk;
  const C *Fi = r.Fk[parity];
  C *Fo = r.Fk[parity ^ 1];
  auto at = [&](int comp, int row) {
    return Fi[comp * plane + (long long)wrap_small(row, n2) * nk + k];
  };
  const auto *Jk = r.Jk;
  auto jat = [&](int comp, int row) { return to_d2(Jk[comp * plane + (long long)row * nk + k]); };
  const C dp = cmk(r.sym[4 * k + 0], r.sym[4 * k + 1]);
  const C dm = cmk(r.sym[4 * k + 2], r.sym[4 * k + 3]);
  const double hdt = r.mhdt, dt = r.mdt, i2x = r.midx2;
  auto b1h = [&](C B, C Ea, C Eb) { return csub(B, cscale(csub(Eb, Ea), hdt * i2x)); };
  auto b2h = [&](C B, C E) { return cadd(B, cscale(cmul(dp, E), hdt)); };
  auto b3h = [&](C B, C E2x, C E1a, C E1b) {
    return csub(B, cscale(csub(cmul(dp, E2x), cscale(csub(E1b, E1a), i2x)), hdt));
  };
  auto e1n = [&](C E, C Ba, C Bb, C j) { return cadd(E, cscale(csub(cscale(csub(Bb, Ba), i2x), j), dt)); };
  auto e3n = [&](C E, C B2x, C B1a, C B1b, C j) {
    return cadd(E, cscale(csub(csub(cmul(dm, B2x), cscale(csub(B1b, B1a), i2x)), j), dt));
  };
  // row q0-1: the half-step B1 and B3 that row q0 needs
  C E1 = at(0, q0), E2 = at(1, q0), E3 = at(2, q0);  // E^n of the current row
  C B1h_m, B3h_m;
  {
    const C E1m = at(0, q0 - 1), E2m = at(1, q0 - 1), E3m = at(2, q0 - 1);
    B1h_m = b1h(at(3, q0 - 1), E3m, E3);
    B3h_m = b3h(at(5, q0 - 1), E2m, E1m, E1);
  }
  // previous row's values, for its output once the current row's E^{n+1} exists
  C pE1n, pE2n, pE3n, pB1h, pB2h, pB3h;
  // row j: its half-step B and new E1, E3; the output of row j-1; then, below
  // the strip's last row + 1, the shift to row j+1
  auto row = [&](int j, bool last) {
    const int jw = wrap_small(j, n2);
    const C E1p = at(0, j + 1), E3p = at(2, j + 1);
    const C B1h = b1h(at(3, j), E3, E3p);
    const C B2h = b2h(at(4, j), E3);
    const C B3h = b3h(at(5, j), E2, E1, E1p);
    const C E1n = e1n(E1, B3h_m, B3h, jat(0, jw));
    const C E3n = e3n(E3, B2h, B1h_m, B1h, jat(2, jw));
    if (j > q0) {
      // B^{n+1} on row j-1 and the stores of that row
      const long long o = (long long)(j - 1) * nk + k;
      Fo[o] = pE1n;
      Fo[plane + o] = pE2n;
      Fo[2 * plane + o] = pE3n;
      Fo[3 * plane + o] = b1h(pB1h, pE3n, E3n);
      Fo[4 * plane + o] = b2h(pB2h, pE3n);
      Fo[5 * plane + o] = b3h(pB3h, pE2n, pE1n, E1n);
    }
    if (last) return;
    pE2n = cadd(E2, cscale(csub(cscale(cmul(dm, B3h), -1.0), jat(1, jw)), dt));
    pE1n = E1n;
    pE3n = E3n;
    pB1h = B1h;
    pB2h = B2h;
    pB3h = B3h;
    B1h_m = B1h;
    B3h_m = B3h;
    E1 = E1p;
    E3 = E3p;
    E2 = at(1, j + 1);
  };
  if (q1 - q0 == KSTRIP) {
    // a whole strip: unrolled, so that the rows' loads can be issued early
#pragma unroll
    for (int t = 0; t <= KSTRIP; ++t) row(q0 + t, t == KSTRIP);
  } else {
    for (int j = q0; j <= q1; ++j) row(j, j == q1);
  }
}

// =====================================================================
// 3D hybrid Maxwell update: x1 spectral, x2 and x3 finite differences
// =====================================================================
// Two passes per step over (i3, i2, kappa1), FP64 master copy:
//   pass A: B^{n+1/2} = B^n - (dt/2) C_E E^n (on the thread's row and, by
//           recomputation, the parts of the rows i2-1 and i3-1 that the
//           backward differences need), E^{n+1} = E^n + dt (C_B B^{n+1/2} - j~);
//           writes E^{n+1} and B^{n+1/2} into the other master buffer;
//   pass B: B^{n+1} = B^{n+1/2} - (dt/2) C_E E^{n+1} in that buffer.
// C_E E = (D2+ E3 - D3+ E2, D3+ E1 - D1+ E3, D1+ E2 - D2+ E1) and
// C_B B = (D2- B3 - D3- B2, D3- B1 - D1- B3, D1- B2 - D2- B1) (the Yee curl of
// Sec. 2.2 with the x1 derivative replaced by i k1 xi+-).
// One thread per (strip of KSTRIP3 planes i3, i2, kappa1): the thread walks
// its planes in order and carries what the next plane shares with this one
// (E1 and E2 of plane i3 + 1, E2 of row i2 - 1 there, and the half-step B1,
// B2 of plane i3 that plane i3 + 1 needs as its i3 - 1 values), so a plane
// reads 13 complex values of the master copy instead of 21.  Every value is
// computed by the same expression as for a single plane.
template <class R>
__global__ void __launch_bounds__(256) k_kupdate3a(const Run<R> *__restrict__ runs,
                                                   const Item *__restrict__ items, int parity) {
  using C = double2;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int nk = r.nk, n2 = r.n2, n3 = r.n3;
  const int nstrips = (n3 + KSTRIP3 - 1) / KSTRIP3;
  const int e = it.a + threadIdx.x;
  if (e >= nstrips * n2 * nk) return;
  const int strip = e / (n2 * nk), rem = e - strip * (n2 * nk);
  const int i2 = rem / nk, k = rem - i2 * nk;
  const int q0 = strip * KSTRIP3, q1 = min(q0 + KSTRIP3, n3);  // planes q0 .. q1-1
  const long long vol = (long long)r.rows * nk;
  const C *Fi = r.Fk[parity];
  C *Fo = r.Fk[parity ^ 1];
  const int a2p = wrap_small(i2 + 1, n2), a2m = wrap_small(i2 - 1, n2);
  auto at = [&](int comp, int j2, int j3) {
    return Fi[comp * vol + ((long long)wrap_small(j3, n3) * n2 + j2) * nk + k];
  };
  const C dp = cmk(r.sym[4 * k + 0], r.sym[4 * k + 1]);
  const C dm = cmk(r.sym[4 * k + 2], r.sym[4 * k + 3]);
  const double hdt = r.mhdt, dt = r.mdt, i2x = r.midx2, i3x = r.midx3;
  // curl E components, forward differences
  auto cE1 = [&](C e3, C e3n2, C e2, C e2n3) {
    return csub(cscale(csub(e3n2, e3), i2x), cscale(csub(e2n3, e2), i3x));
  };
  auto cE2 = [&](C e1, C e1n3, C e3) { return csub(cscale(csub(e1n3, e1), i3x), cmul(dp, e3)); };
  auto cE3 = [&](C e2, C e1, C e1n2) { return csub(cmul(dp, e2), cscale(csub(e1n2, e1), i2x)); };
  const auto *Jk = r.Jk;
  // carried values: E1, E2 on (i2, i3), E2 on (i2-1, i3), and B1, B2 at the
  // half step on (i2, i3-1)
  C E1 = at(0, i2, q0), E2 = at(1, i2, q0), E2_2m = at(1, a2m, q0);
  C B1h_3m, B2h_3m;
  {
    const C E1_3m = at(0, i2, q0 - 1), E2_3m = at(1, i2, q0 - 1), E3_3m = at(2, i2, q0 - 1);
    const C E3_2p3m = at(2, a2p, q0 - 1);
    B1h_3m = csub(at(3, i2, q0 - 1), cscale(cE1(E3_3m, E3_2p3m, E2_3m, E2), hdt));
    B2h_3m = csub(at(4, i2, q0 - 1), cscale(cE2(E1_3m, E1, E3_3m), hdt));
  }
  auto plane = [&](int i3) {
    const C E3 = at(2, i2, i3);
    const C E1_2p = at(0, a2p, i3), E3_2p = at(2, a2p, i3);     // (i2+1, i3)
    const C E1_2m = at(0, a2m, i3), E3_2m = at(2, a2m, i3);     // (i2-1, i3)
    const C E1_3p = at(0, i2, i3 + 1), E2_3p = at(1, i2, i3 + 1);  // (i2, i3+1)
    const C E2_2m3p = at(1, a2m, i3 + 1);                       // (i2-1, i3+1)
    // B^{n+1/2} on (i2, i3)
    const C B1h = csub(at(3, i2, i3), cscale(cE1(E3, E3_2p, E2, E2_3p), hdt));
    const C B2h = csub(at(4, i2, i3), cscale(cE2(E1, E1_3p, E3), hdt));
    const C B3h = csub(at(5, i2, i3), cscale(cE3(E2, E1, E1_2p), hdt));
    // on (i2-1, i3): B1 and B3
    const C B1h_2m = csub(at(3, a2m, i3), cscale(cE1(E3_2m, E3, E2_2m, E2_2m3p), hdt));
    const C B3h_2m = csub(at(5, a2m, i3), cscale(cE3(E2_2m, E1_2m, E1), hdt));
    // curl B, backward differences
    const C cB1 = csub(cscale(csub(B3h, B3h_2m), i2x), cscale(csub(B2h, B2h_3m), i3x));
    const C cB2 = csub(cscale(csub(B1h, B1h_3m), i3x), cmul(dm, B3h));
    const C cB3 = csub(cmul(dm, B2h), cscale(csub(B1h, B1h_2m), i2x));
    const long long o = ((long long)i3 * n2 + i2) * nk + k;
    const C j1 = to_d2(Jk[o]), j2 = to_d2(Jk[vol + o]), j3 = to_d2(Jk[2 * vol + o]);
    Fo[o] = cadd(E1, cscale(csub(cB1, j1), dt));
    Fo[vol + o] = cadd(E2, cscale(csub(cB2, j2), dt));
    Fo[2 * vol + o] = cadd(E3, cscale(csub(cB3, j3), dt));
    Fo[3 * vol + o] = B1h;
    Fo[4 * vol + o] = B2h;
    Fo[5 * vol + o] = B3h;
    B1h_3m = B1h;
    B2h_3m = B2h;
    E1 = E1_3p;
    E2 = E2_3p;
    E2_2m = E2_2m3p;
  };
  if (q1 - q0 == KSTRIP3) {
#pragma unroll
    for (int t = 0; t < KSTRIP3; ++t) plane(q0 + t);
  } else {
    for (int i3 = q0; i3 < q1; ++i3) plane(i3);
  }
}

// Pass B over the same (strip, i2, kappa1) threads: E1, E2 of plane i3 + 1
// are carried to the next plane.
template <class R>
__global__ void __launch_bounds__(256) k_kupdate3b(const Run<R> *__restrict__ runs,
                                                   const Item *__restrict__ items, int parity) {
  using C = double2;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int nk = r.nk, n2 = r.n2, n3 = r.n3;
  const int nstrips = (n3 + KSTRIP3 - 1) / KSTRIP3;
  const int e = it.a + threadIdx.x;
  if (e >= nstrips * n2 * nk) return;
  const int strip = e / (n2 * nk), rem = e - strip * (n2 * nk);
  const int i2 = rem / nk, k = rem - i2 * nk;
  const int q0 = strip * KSTRIP3, q1 = min(q0 + KSTRIP3, n3);
  const long long vol = (long long)r.rows * nk;
  C *F = r.Fk[parity ^ 1];
  const int a2p = wrap_small(i2 + 1, n2);
  auto at = [&](int comp, int j2, int j3) {
    return F[comp * vol + ((long long)wrap_small(j3, n3) * n2 + j2) * nk + k];
  };
  const C dp = cmk(r.sym[4 * k + 0], r.sym[4 * k + 1]);
  const double hdt = r.mhdt, i2x = r.midx2, i3x = r.midx3;
  C E1 = at(0, i2, q0), E2 = at(1, i2, q0);
  auto plane = [&](int i3) {
    const C E3 = at(2, i2, i3);
    const C E1_2p = at(0, a2p, i3), E3_2p = at(2, a2p, i3);
    const C E1_3p = at(0, i2, i3 + 1), E2_3p = at(1, i2, i3 + 1);
    const C c1 = csub(cscale(csub(E3_2p, E3), i2x), cscale(csub(E2_3p, E2), i3x));
    const C c2 = csub(cscale(csub(E1_3p, E1), i3x), cmul(dp, E3));
    const C c3 = csub(cmul(dp, E2), cscale(csub(E1_2p, E1), i2x));
    const long long o = ((long long)i3 * n2 + i2) * nk + k;
    F[3 * vol + o] = csub(F[3 * vol + o], cscale(c1, hdt));
    F[4 * vol + o] = csub(F[4 * vol + o], cscale(c2, hdt));
    F[5 * vol + o] = csub(F[5 * vol + o], cscale(c3, hdt));
    E1 = E1_3p;
    E2 = E2_3p;
  };
  if (q1 - q0 == KSTRIP3) {
#pragma unroll
    for (int t = 0; t < KSTRIP3; ++t) plane(q0 + t);
  } else {
    for (int i3 = q0; i3 < q1; ++i3) plane(i3);
  }
}

// =====================================================================
// inverse FFT of E and B
// =====================================================================
// Item = (run, row, group): components 3g..3g+2 of the master buffer of the
// given parity, written to the real-space fields (ncomp = 3); or (run, row,
// component) (ncomp = 1).
template <class R, int MAXB>
__global__ void __launch_bounds__(256) k_ifft_eb(const Run<R> *__restrict__ runs,
                                                 const Item *__restrict__ items, int parity,
                                                 int ncomp) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C *lds = (C *)smem_raw;
  const Item it = items[blockIdx.x];
  const Run<R> &r = runs[it.run];
  const int row = it.a, cb = ncomp == 3 ? 3 * it.b : it.b;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, cells = r.cells, nk = r.nk;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int cc = 0; cc < ncomp; ++cc) {
      const double2 *X = r.Fk[parity] + (long long)(cb + cc) * r.rows * nk + (long long)row * nk;
      const C Xk = from_d2<C>(X[k]), Xmk = from_d2<C>(X[mk]);
      lds[cc * M + k] = c2r_pre(Xk, Xmk, r.tw[k]);
      if (k != 0 && mk != k) lds[cc * M + mk] = c2r_pre(Xmk, Xk, r.tw[mk]);
    }
  }
  __syncthreads();
  lds_fft_rows<C, MAXB>(lds, M, log2M, ncomp, r.tw, 2, true);
  const R s = r.inv_m;
  for (int cc = 0; cc < ncomp; ++cc) {
    R *dst = r.F + (long long)(cb + cc) * cells + (long long)row * n1;
    for (int n = threadIdx.x; n < M; n += blockDim.x) {
      const C z = lds[cc * M + n];
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

// Gauss residual (Eq. (27)) of one row in FP64: R = D1- E1 + D2- E2 - f rho.
template <class R>
__global__ void __launch_bounds__(256) k_gauss(const Run<R> *run, int parity, const double *rho,
                                               const double2 *tw64, const double *sym64,
                                               const double *filt, double idx2, double *rows_out) {
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
  const double2 *Fk = r.Fk[parity];
  const int rm = wrap_small(row - 1, n2);
  double s2 = 0, smax = 0, sref = 0;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int side = 0; side < 2; ++side) {
      const int kk = side ? mk : k;
      if (side && mk == k) break;
      const double2 Zk = lds[kk & (M - 1)], Zmk = lds[(M - kk) & (M - 1)];
      const double2 rh = r2c_post(Zk, Zmk, tw64[kk]);
      const double2 e1 = Fk[(long long)row * nk + kk];
      const double2 e2 = Fk[plane + (long long)row * nk + kk];
      const double2 e2m = Fk[plane + (long long)rm * nk + kk];
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

// Row transforms whose radix-4 passes need at most 3 butterflies per thread
// (256 threads): rows of up to 2048 points with three components per block,
// or one component per block (the radix-16 passes then cover up to 4096).
// Their kernels are built with the smaller register buffer.
static bool small_rows(int maxM, int ncomp) { return maxM <= 1024 || ncomp == 1; }

template <class R>
void Launch<R>::fft_j(const Run<R> *runs, const Item *items, int nitems, int parity, int maxM,
                      int ncomp, hipStream_t s) {
  if (nitems <= 0) return;
  const size_t lds = (size_t)ncomp * maxM * sizeof(typename Cplx<R>::T);
  if (small_rows(maxM, ncomp))
    hipLaunchKernelGGL((k_fft_j<R, 3>), dim3(nitems), dim3(256), lds, s, runs, items, parity, ncomp);
  else
    hipLaunchKernelGGL((k_fft_j<R, 6>), dim3(nitems), dim3(256), lds, s, runs, items, parity, ncomp);
}

// 3D Gauss residual on the row (i2, i3): R = D1- E1 + D2- E2 + D3- E3 - f rho
// in (kappa1, i2, i3) space, FP64.
template <class R>
__global__ void __launch_bounds__(256) k_gauss3(const Run<R> *run, int parity, const double *rho,
                                                const double2 *tw64, const double *sym64,
                                                const double *filt, double idx2, double idx3,
                                                double *rows_out) {
  extern __shared__ unsigned char smem_raw[];
  double2 *lds = (double2 *)smem_raw;
  __shared__ double red[256][3];
  const Run<R> &r = *run;
  const int row = blockIdx.x;
  const int n1 = r.n1, M = n1 >> 1, log2M = r.log2n1 - 1, nk = r.nk, n2 = r.n2, n3 = r.n3;
  const int i3 = row / n2, i2 = row - i3 * n2;
  for (int n = threadIdx.x; n < M; n += blockDim.x)
    lds[n] = make_double2(rho[(long long)row * n1 + 2 * n], rho[(long long)row * n1 + 2 * n + 1]);
  __syncthreads();
  lds_fft<double2, 6>(lds, M, log2M, 1, tw64, 2, false);
  const long long vol = (long long)r.rows * nk;
  const double2 *Fk = r.Fk[parity];
  const long long rm2 = ((long long)i3 * n2 + wrap_small(i2 - 1, n2)) * nk;
  const long long rm3 = ((long long)wrap_small(i3 - 1, n3) * n2 + i2) * nk;
  double s2 = 0, smax = 0, sref = 0;
  for (int k = threadIdx.x; k <= (M >> 1); k += blockDim.x) {
    const int mk = M - k;
    for (int side = 0; side < 2; ++side) {
      const int kk = side ? mk : k;
      if (side && mk == k) break;
      const double2 Zk = lds[kk & (M - 1)], Zmk = lds[(M - kk) & (M - 1)];
      const double2 rh = r2c_post(Zk, Zmk, tw64[kk]);
      const double2 e1 = Fk[(long long)row * nk + kk];
      const double2 e2 = Fk[vol + (long long)row * nk + kk], e2m = Fk[vol + rm2 + kk];
      const double2 e3 = Fk[2 * vol + (long long)row * nk + kk], e3m = Fk[2 * vol + rm3 + kk];
      const double2 dm = make_double2(sym64[4 * kk + 2], sym64[4 * kk + 3]);
      double2 div = cmul(dm, e1);
      div.x += (e2.x - e2m.x) * idx2 + (e3.x - e3m.x) * idx3;
      div.y += (e2.y - e2m.y) * idx2 + (e3.y - e3m.y) * idx3;
      const double fr_x = filt[kk] * rh.x, fr_y = filt[kk] * rh.y;
      const double rx = div.x - fr_x, ry = div.y - fr_y;
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

// 3D continuity residual (Eq. (23) with the x3 term) in FP64: the current of
// the last step is fac[d] * J (J the deposit accumulators of either form).
template <class A>
__global__ void k_cont3(const double *rn, const double *ro, const A *J, int n1, int n2, int n3,
                        double dt, double f1, double f2, double f3, double idx1, double idx2,
                        double idx3, double *partial) {
  __shared__ double red[256];
  const long long cells = (long long)n1 * n2 * n3;
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells;
       i += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(i % n1);
    const long long rr = i / n1;
    const int i2 = (int)(rr % n2), i3 = (int)(rr / n2);
    const long long w1 = (long long)(rr * n1) + wrap_small(i1 - 1, n1);
    const long long w2 = ((long long)i3 * n2 + wrap_small(i2 - 1, n2)) * n1 + i1;
    const long long w3 = ((long long)wrap_small(i3 - 1, n3) * n2 + i2) * n1 + i1;
    const double div = f1 * ((double)J[i] - (double)J[w1]) * idx1 +
                       f2 * ((double)J[cells + i] - (double)J[cells + w2]) * idx2 +
                       f3 * ((double)J[2 * cells + i] - (double)J[2 * cells + w3]) * idx3;
    m = fmax(m, fabs((rn[i] - ro[i]) / dt + div));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <class R>
void Launch<R>::kupdate(const Run<R> *runs, const Item *items, int nitems, int parity,
                        hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_kupdate<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity);
}

template <class R>
void Launch<R>::ifft_eb(const Run<R> *runs, const Item *items, int nitems, int parity, int maxM,
                        int ncomp, hipStream_t s) {
  if (nitems <= 0) return;
  const size_t lds = (size_t)ncomp * maxM * sizeof(typename Cplx<R>::T);
  if (small_rows(maxM, ncomp))
    hipLaunchKernelGGL((k_ifft_eb<R, 3>), dim3(nitems), dim3(256), lds, s, runs, items, parity, ncomp);
  else
    hipLaunchKernelGGL((k_ifft_eb<R, 6>), dim3(nitems), dim3(256), lds, s, runs, items, parity, ncomp);
}

template <class R>
void Launch<R>::fields_to_k(const Run<R> *runs, const Item *items, int nitems, int parity,
                            int maxM, int ncomp, hipStream_t s) {
  if (nitems <= 0) return;
  const size_t lds = (size_t)ncomp * maxM * sizeof(typename Cplx<R>::T);
  if (small_rows(maxM, ncomp))
    hipLaunchKernelGGL((k_fields_to_k<R, 3>), dim3(nitems), dim3(256), lds, s, runs, items, parity,
                       ncomp);
  else
    hipLaunchKernelGGL((k_fields_to_k<R, 6>), dim3(nitems), dim3(256), lds, s, runs, items, parity,
                       ncomp);
}

template <class R>
void Launch<R>::kupdate3(const Run<R> *runs, const Item *items, int nitems, int parity,
                         hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_kupdate3a<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity);
  hipLaunchKernelGGL(k_kupdate3b<R>, dim3(nitems), dim3(256), 0, s, runs, items, parity);
}

template struct Launch<float>;
template struct Launch<double>;

template <class R>
void launch_gauss3(const Run<R> *run_dev, int rows, int n1, int parity, const double *rho,
                   const double2 *tw64, const double *sym64, const double *filt, double idx2,
                   double idx3, double *rows_out, hipStream_t s) {
  const size_t lds = (size_t)(n1 / 2) * sizeof(double2);
  hipLaunchKernelGGL(k_gauss3<R>, dim3(rows), dim3(256), lds, s, run_dev, parity, rho, tw64,
                     sym64, filt, idx2, idx3, rows_out);
}
template void launch_gauss3<float>(const Run<float> *, int, int, int, const double *,
                                   const double2 *, const double *, const double *, double, double,
                                   double *, hipStream_t);
template void launch_gauss3<double>(const Run<double> *, int, int, int, const double *,
                                    const double2 *, const double *, const double *, double,
                                    double, double *, hipStream_t);

template <class A>
void launch_cont3(const double *rn, const double *ro, const A *J, int n1, int n2, int n3,
                  double dt, double f1, double f2, double f3, double idx1, double idx2,
                  double idx3, double *partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_cont3<A>, dim3(nblocks), dim3(256), 0, s, rn, ro, J, n1, n2, n3, dt, f1,
                     f2, f3, idx1, idx2, idx3, partial);
}
template void launch_cont3<long long>(const double *, const double *, const long long *, int, int,
                                      int, double, double, double, double, double, double, double,
                                      double *, int, hipStream_t);
template void launch_cont3<double>(const double *, const double *, const double *, int, int, int,
                                   double, double, double, double, double, double, double,
                                   double *, int, hipStream_t);

template <class R>
void launch_energy(const R *F, long long cells, double *partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_energy<R>, dim3(nblocks), dim3(256), 0, s, F, cells, partial);
}
template void launch_energy<float>(const float *, long long, double *, int, hipStream_t);
template void launch_energy<double>(const double *, long long, double *, int, hipStream_t);

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
