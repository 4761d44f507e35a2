// io.hip -- transfers between a Cartesian run's device state and caller-owned
// device buffers (the _device entry points of the C ABI): particles loaded from
// FP64 positions, momenta and weights in device memory, and the particle state
// and real-space fields copied out to device memory, all on the handle's stream.
#include "hpic_internal.h"

namespace hp {

// Cell index and offset in [0,1) of a physical position, wrapped periodically:
// the same FP64 operations, in the same order, as the host loader (fmod, the
// division by dx and floor are exact or correctly rounded in FP64), so a run
// loaded from device memory holds the same bits as one loaded from the host.
template <class R>
__device__ __forceinline__ void split_pos(double x, double L, double dx, int n, int &c, R &f) {
  double xw = fmod(x, L);
  if (xw < 0) xw += L;
  const double xi = xw / dx;
  const double cf = floor(xi);
  c = (int)cf;
  R g = (R)(xi - cf);
  if (g >= R(1)) {
    g = R(0);
    c += 1;
  }
  if (c >= n) c -= n;
  if (c < 0) c += n;
  f = g;
}

struct LoadArgs {
  int dim, n1, n2, n3, log2n1, sh3;
  double L1, L2, L3, dx1, dx2, dx3, q;
  long long n;
  const double *x, *u, *w;  // [dim][n], [3][n], [n]
};

__device__ __forceinline__ bool finite_all(const LoadArgs &a, long long p) {
  const long long n = a.n;
  bool ok = isfinite(a.x[p]) && isfinite(a.x[n + p]) && isfinite(a.u[p]) &&
            isfinite(a.u[n + p]) && isfinite(a.u[2 * n + p]) && isfinite(a.w[p]);
  if (a.dim == 3) ok = ok && isfinite(a.x[2 * n + p]);
  return ok;
}

template <class R>
__device__ __forceinline__ void cell_of(const LoadArgs &a, long long p, int &c1, int &c2, int &c3,
                                        R &g1, R &g2, R &g3) {
  const long long n = a.n;
  split_pos<R>(a.x[p], a.L1, a.dx1, a.n1, c1, g1);
  split_pos<R>(a.x[n + p], a.L2, a.dx2, a.n2, c2, g2);
  c3 = 0;
  g3 = R(0);
  if (a.dim == 3) split_pos<R>(a.x[2 * n + p], a.L3, a.dx3, a.n3, c3, g3);
}

// First pass (nothing of the run is changed): non-finite inputs (bad != 0),
// particles per cell (count[cells]), and the largest and smallest |q w| as
// the bits of non-negative doubles (ordered like the values).
template <class R>
__global__ void k_scan_particles(LoadArgs a, int *count, unsigned long long *qbits, unsigned *bad) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  if (!finite_all(a, p)) {
    atomicOr(bad, 1u);
    return;
  }
  int c1, c2, c3;
  R g1, g2, g3;
  cell_of<R>(a, p, c1, c2, c3, g1, g2, g3);
  atomicAdd(&count[((long long)c3 * a.n2 + c2) * a.n1 + c1], 1);
  const R qw = (R)(a.q * a.w[p]);
  const unsigned long long b = (unsigned long long)__double_as_longlong(fabs((double)qw));
  atomicMax(&qbits[0], b);
  atomicMin(&qbits[1], b);
}

// Largest entry of a[n] into *out (initially 0).
__global__ void k_max_int(const int *a, long long n, int *out) {
  int m = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = max(m, a[i]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// Second pass: the structure of arrays of the run in input order (id = index).
template <class R>
__global__ void k_load_particles(LoadArgs a, Parts<R> A) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const long long n = a.n;
  int c1, c2, c3;
  R g1, g2, g3;
  cell_of<R>(a, p, c1, c2, c3, g1, g2, g3);
  A.cell[p] = (c3 << a.sh3) | (c2 << a.log2n1) | c1;
  A.id[p] = (int)p;
  A.f1[p] = g1;
  A.f2[p] = g2;
  if (a.dim == 3) A.f3[p] = g3;
  A.u1[p] = (R)a.u[p];
  A.u2[p] = (R)a.u[n + p];
  A.u3[p] = (R)a.u[2 * n + p];
  A.qw[p] = (R)(a.q * a.w[p]);
}

// The run's particle state in its current order into caller buffers:
// cell[dim][n] (unpacked i1, i2, i3), off[dim][n], u[3][n], qw[n], id[n]; a
// null pointer skips that array.
template <class R>
__global__ void k_unload_particles(const Run<R> *run_dev, int pp, int *cell, R *off, R *u, R *qw,
                                   int *id) {
  const Run<R> &r = *run_dev;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = r.np;
  if (p >= n) return;
  const Parts<R> &A = r.pt[pp];
  const int c = A.cell[p];
  if (cell) {
    const int i1 = c & (r.n1 - 1);
    cell[p] = i1;
    if (r.dim == 3) {
      cell[n + p] = (c >> r.log2n1) & ((1 << (r.sh3 - r.log2n1)) - 1);
      cell[2 * n + p] = c >> r.sh3;
    } else {
      cell[n + p] = c >> r.log2n1;
    }
  }
  if (off) {
    off[p] = A.f1[p];
    off[n + p] = A.f2[p];
    if (r.dim == 3) off[2 * n + p] = A.f3[p];
  }
  if (u) {
    u[p] = A.u1[p];
    u[n + p] = A.u2[p];
    u[2 * n + p] = A.u3[p];
  }
  if (qw) qw[p] = A.qw[p];
  if (id) id[p] = A.id[p];
}

// out[i] = raw[i] f + bg in FP64, one rounding per operation as on the host
// (the deposited current in physical units from the accumulators).
template <class A>
__global__ void k_current_out(const A *raw, long long n, double f, double bg, double *out) {
#pragma clang fp contract(off)
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (double)raw[i] * f + bg;
}

template <class R>
__global__ void k_real_to_double(const R *in, long long n, double *out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

template <class A>
void launch_current_out(const A *raw, long long n, double f, double bg, double *out, hipStream_t s) {
  if (n <= 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_current_out<A>, dim3((unsigned)blocks), dim3(256), 0, s, raw, n, f, bg, out);
}
template <class R>
void launch_real_to_double(const R *in, long long n, double *out, hipStream_t s) {
  if (n <= 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_real_to_double<R>, dim3((unsigned)blocks), dim3(256), 0, s, in, n, out);
}
template void launch_current_out<long long>(const long long *, long long, double, double, double *,
                                            hipStream_t);
template void launch_current_out<double>(const double *, long long, double, double, double *,
                                         hipStream_t);
template void launch_real_to_double<float>(const float *, long long, double *, hipStream_t);
template void launch_real_to_double<double>(const double *, long long, double *, hipStream_t);

// p[0..n) = 0 (a kernel rather than a memset, so that a captured graph clears
// it on every replay).
__global__ void k_zero_i64(long long *p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0;
}

void launch_zero_i64(long long *p, long long n, hipStream_t s) {
  if (n <= 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

template <class R>
void launch_scan_particles(const LoadGeom &g, long long n, const double *x, const double *u,
                           const double *w, double q, int *count, unsigned long long *qbits,
                           unsigned *bad, hipStream_t s) {
  if (n <= 0) return;
  const LoadArgs a{g.dim, g.n1, g.n2, g.n3, g.log2n1, g.sh3, g.L[0], g.L[1], g.L[2],
                   g.dx[0], g.dx[1], g.dx[2], q, n, x, u, w};
  hipLaunchKernelGGL(k_scan_particles<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     count, qbits, bad);
}

void launch_max_int(const int *a, long long n, int *out, hipStream_t s) {
  if (n <= 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_max_int, dim3((unsigned)blocks), dim3(256), 0, s, a, n, out);
}

template <class R>
void launch_load_particles(const LoadGeom &g, long long n, const double *x, const double *u,
                           const double *w, double q, Parts<R> A, hipStream_t s) {
  if (n <= 0) return;
  const LoadArgs a{g.dim, g.n1, g.n2, g.n3, g.log2n1, g.sh3, g.L[0], g.L[1], g.L[2],
                   g.dx[0], g.dx[1], g.dx[2], q, n, x, u, w};
  hipLaunchKernelGGL(k_load_particles<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, A);
}

template <class R>
void launch_unload_particles(const Run<R> *run_dev, int pp, int np, int *cell, R *off, R *u, R *qw,
                             int *id, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_unload_particles<R>, dim3((np + 255) / 256), dim3(256), 0, s, run_dev, pp,
                     cell, off, u, qw, id);
}

template void launch_scan_particles<float>(const LoadGeom &, long long, const double *,
                                           const double *, const double *, double, int *,
                                           unsigned long long *, unsigned *, hipStream_t);
template void launch_scan_particles<double>(const LoadGeom &, long long, const double *,
                                            const double *, const double *, double, int *,
                                            unsigned long long *, unsigned *, hipStream_t);
template void launch_load_particles<float>(const LoadGeom &, long long, const double *,
                                           const double *, const double *, double, Parts<float>,
                                           hipStream_t);
template void launch_load_particles<double>(const LoadGeom &, long long, const double *,
                                            const double *, const double *, double, Parts<double>,
                                            hipStream_t);
template void launch_unload_particles<float>(const Run<float> *, int, int, int *, float *, float *,
                                             float *, int *, hipStream_t);
template void launch_unload_particles<double>(const Run<double> *, int, int, int *, double *,
                                              double *, double *, int *, hipStream_t);

}  // namespace hp
