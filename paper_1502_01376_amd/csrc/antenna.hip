// antenna.hip -- moving current-sheet antenna of 2D runs on gfx950 (Sec. 6
// launches the boosted-frame laser with a moving antenna; the form is the one
// hp_set_antenna documents).  One thread per (antenna, row): the sheet's
// surface current K(t) g(x2) spread over the three x1 nodes around its
// position with the quadratic B-spline, added to j3 in the accumulator's units
// (FP32 form: one rounding per node to the 64-bit integers; FP64 form: the
// physical current).  The time comes from a device step counter, so that a
// captured step graph replays with the right time.
#include "hpic_internal.h"

namespace hp {

namespace {

template <class A> __device__ __forceinline__ A to_accum(double v);
template <> __device__ __forceinline__ long long to_accum<long long>(double v) {
  return rint_i64(v);
}
template <> __device__ __forceinline__ double to_accum<double>(double v) { return v; }

template <class R>
__global__ void __launch_bounds__(256) k_antenna(const Run<R> *__restrict__ runs,
                                                 const AntennaDev *__restrict__ ants, int parity,
                                                 const long long *__restrict__ step) {
  using A = typename AccOf<R>::T;
  const AntennaDev a = ants[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n2) return;
  const double t = ((double)*step + 0.5) * a.dt;
  const double s = t - a.t0;
  if (!(s >= 0.0 && s <= a.T)) return;
  const double env = sin(3.14159265358979323846 * s / a.T);
  const double K = a.K0 * env * env * sin(a.omega * s + a.phase);
  double gx = 1.0;
  if (a.waist > 0.0) {
    const double L2 = a.n2 * a.dx2;
    double d = fmod(j * a.dx2 - a.x2c, L2);
    if (d < -0.5 * L2) d += L2;
    if (d >= 0.5 * L2) d -= L2;
    gx = exp(-(d / a.waist) * (d / a.waist));
  }
  const double L1 = a.n1 * a.dx1;
  double xa = fmod(a.x0 + a.v * t, L1);
  if (xa < 0.0) xa += L1;
  const double sa = xa / a.dx1;
  const int m = (int)floor(sa + 0.5);  // nearest node
  const double d = sa - m;             // in [-1/2, 1/2]
  const double w[3] = {0.5 * (0.5 - d) * (0.5 - d), 0.75 - d * d, 0.5 * (0.5 + d) * (0.5 + d)};
  const double c = K * gx / a.dx1 * a.scale;
  A *J3 = runs[a.run].J[parity] + 2LL * runs[a.run].cells + (long long)j * a.n1;
  for (int k = 0; k < 3; ++k) {
    int i = m - 1 + k;
    i = ((i % a.n1) + a.n1) % a.n1;
    J3[i] += to_accum<A>(c * w[k]);
  }
}

__global__ void k_step_tick(long long *step) { *step += 1; }

}  // namespace

template <class R>
void launch_antenna(const Run<R> *runs, const AntennaDev *ants, int nant, int maxn2, int parity,
                    const long long *step, hipStream_t s) {
  if (nant <= 0 || maxn2 <= 0) return;
  hipLaunchKernelGGL(k_antenna<R>, dim3((maxn2 + 255) / 256, nant), dim3(256), 0, s, runs, ants,
                     parity, step);
}
void launch_step_tick(long long *step, hipStream_t s) {
  hipLaunchKernelGGL(k_step_tick, dim3(1), dim3(1), 0, s, step);
}
template void launch_antenna<float>(const Run<float> *, const AntennaDev *, int, int, int,
                                    const long long *, hipStream_t);
template void launch_antenna<double>(const Run<double> *, const AntennaDev *, int, int, int,
                                     const long long *, hipStream_t);

}  // namespace hp
