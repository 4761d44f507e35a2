// runtime.cpp -- host runtime of the MI355X hybrid Yee-FFT PIC library: the C
// ABI of include/hpic.h.  Validation (Eq. (22) Courant limit, FFT sizes,
// fixed-point headroom), device allocation, FP64-computed symbol tables,
// batched work lists, step sequencing on the caller's stream, diagnostics and
// checkpointing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "hpic.h"
#include "hpic_q3d.h"
#include "hpic_update3.h"

using namespace hp;

// Staging memory of the entry point that allocates nothing
// (hp_debug_deposit_noalloc): the moves of at most NOALLOC_MAX_MOVES particles
// (40 bytes each: two cell pairs, two offset pairs, v3, qw) followed by the
// 64-bit accumulators of at most NOALLOC_MAX_CELLS cells (3 x 8 bytes each),
// 16 MiB per GPU, held by every GPU the library runs on until the process
// ends.  In host code `scratch` is a host-side stand-in for the symbol, not a
// device address: the address comes from hipGetSymbolAddress (once per device,
// with that device current) and only that address reaches kernels and copies.
constexpr size_t NOALLOC_MAX_MOVES = size_t(1) << 18;
constexpr size_t NOALLOC_MAX_CELLS = size_t(1) << 18;
constexpr size_t NOALLOC_J_OFFSET = 40 * NOALLOC_MAX_MOVES;
constexpr size_t NOALLOC_BYTES = NOALLOC_J_OFFSET + 24 * NOALLOC_MAX_CELLS;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(HP_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// Device address of this process's scratch region on device dev (the current
// device), looked up on the first call for that device.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[NOALLOC_MAX_DEVICES] = {nullptr};

int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(HP_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(HP_EDEVICE, "hipGetSymbolAddress of the scratch region: %s", hipGetErrorString(e));
    }
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return HP_OK;
}

const double PI = 3.14159265358979323846;

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Stability limit of the time step: Eq. (22) for the hybrid solver, the Yee
// limit when the finite-difference x1 symbol is used.
// In 3D the x3 difference adds 4/dx3^2 (1/dx3^2 for Yee) under the root.
double courant_limit(const hp_config &c) {
  const double a = c.dx[0], b = c.dx[1], e = c.dx[2];
  const bool three = c.geom == HP_GEOM_3D;
  if (c.deriv1)
    return 1.0 / std::sqrt(1.0 / (a * a) + 1.0 / (b * b) + (three ? 1.0 / (e * e) : 0.0));
  return 2.0 / std::sqrt(PI * PI / (a * a) + 4.0 / (b * b) + (three ? 4.0 / (e * e) : 0.0));
}

// Eq. (29): the bump added to the spectral x1 symbol with the coefficients
// Sec. 4 gives for the Table 1 set-up (k1l = 0.15 kg1, k1u = 0.26 kg1,
// dk_max = 0.01 kg1, kg1 = 2 pi / dx1); zero when kmod is off.
double dk_mod(const hp_config &c, double k1) {
  if (!c.kmod || c.deriv1) return 0.0;
  const double kg = 2.0 * PI / c.dx[0];
  const double kl = 0.15 * kg, ku = 0.26 * kg, dmax = 0.01 * kg, km = 0.5 * (kl + ku);
  if (k1 < kl || k1 > ku) return 0.0;
  const double t = std::cos((k1 - km) / (kl - km) * PI / 2.0);
  return dmax * t * t;
}

const int SORT_CHUNK = 256;   // particles per sort workgroup
const int UPD_BLOCK = 256;    // (row or row strip, kappa) elements per update workgroup
const int TILE1 = 32, TILE2 = 8;  // default particle tile (cells along x1, x2)
const int SLACK1 = 2, SLACK2 = 1;  // drift beyond the tile the LDS budget allows for
const int TILE1_3D = 8, TILE2_3D = 4;  // default 3D tile: 8 x 4 x 4 cells
const double CJ3 = 1099511627776.0;     // 2^40: integer scale of the 3D FP32 deposit
const int DEFAULT_SORT_INTERVAL = 16;

struct Event2 {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct SimBase {
  virtual ~SimBase() {}
  virtual int set_stream(hipStream_t s) = 0;
  virtual int set_particles(int run, int64_t n, const double *x, const double *u,
                            const double *w, double qm, double q) = 0;
  virtual int set_fields(int run, const double *E, const double *B) = 0;
  virtual int set_background(int run, int rho_from_particles, const double *jbg) = 0;
  virtual int step(int nsteps) = 0;
  virtual int sync() = 0;
  virtual int get_field(int run, int comp, double *out, size_t count) = 0;
  virtual int get_current(int run, int comp, int corrected, double *out, size_t count) = 0;
  virtual int get_current_fixed(int run, int comp, int64_t *out, size_t count) = 0;
  virtual int get_count(int run, int64_t *n) = 0;
  virtual int nruns() const = 0;
  virtual int get_particles(int run, int64_t n, double *x, double *u, double *w, int64_t *id) = 0;
  virtual int get_particles_raw(int run, int64_t n, int32_t *cell, float *off, float *u,
                                float *qw, int32_t *id) = 0;
  virtual int diagnostics(int run, hp_diag *out) = 0;
  virtual int get_state(void *blob, size_t *size) = 0;
  virtual int set_state(const void *blob, size_t size) = 0;
  virtual int debug_deposit(int run, int64_t n, const int32_t *c0, const float *o0,
                            const int32_t *c1, const float *o1, const float *v3, const float *qw,
                            int64_t *J) = 0;
  virtual int fixed_params(int run, double *out) = 0;
  virtual int profile(int enable) = 0;
  virtual int kernel_times(double *ms, int64_t *n) = 0;
  virtual int push_stats(int64_t *out) = 0;
  virtual int use_graphs(int enable) = 0;
  virtual int set_tiling(int t1, int t2, int K) = 0;
  virtual int get_tiling(hp_tune *out) = 0;
  virtual int autotune(int nsteps, hp_tune *out) = 0;
  // per-mode field access (quasi-3D); Cartesian handles accept mode 0 only
  virtual int set_fields_mode(int run, int mode, const double *E, const double *B) {
    if (mode != 0) return fail(HP_EINVAL, "mode must be 0 for Cartesian runs");
    return set_fields(run, E, B);
  }
  virtual int get_field_mode(int run, int comp, int mode, double *out, size_t count) {
    if (mode != 0) return fail(HP_EINVAL, "mode must be 0 for Cartesian runs");
    return get_field(run, comp, out, count);
  }
  // deposited current of one azimuthal mode (quasi-3D only)
  virtual int get_current_mode(int, int, int, double *, size_t) {
    return fail(HP_EINVAL, "per-mode currents exist for quasi-3D runs only");
  }
  // moving antenna (2D Cartesian runs only)
  virtual int set_antenna(int, const hp_antenna *) {
    return fail(HP_EINVAL, "the antenna is built for 2D runs only");
  }
  // transfers with caller-owned device buffers (Cartesian runs)
  virtual int set_particles_device(int, int64_t, const double *, const double *, const double *,
                                   double, double) {
    return fail(HP_EINVAL, "device-buffer particle loading exists for Cartesian runs only");
  }
  virtual int get_field_device(int, int, void *, size_t) {
    return fail(HP_EINVAL, "device-buffer field reads exist for Cartesian runs only");
  }
  virtual int get_particles_device(int, int64_t, int32_t *, void *, void *, void *, int32_t *) {
    return fail(HP_EINVAL, "device-buffer particle reads exist for Cartesian runs only");
  }
  virtual int get_current_device(int, int, int, double *, size_t) {
    return fail(HP_EINVAL, "device-buffer current reads exist for Cartesian runs only");
  }
  virtual int debug_deposit_noalloc(int, int64_t, const int32_t *, const float *, const int32_t *,
                                    const float *, const float *, const float *, int64_t *) {
    return fail(HP_EINVAL, "the deposit entry point is for 2D Cartesian runs only");
  }
};

// A pointer the device can dereference: device or managed memory of this
// process (a host pointer passed to a _device entry point is rejected instead
// of faulting in a kernel).
static bool device_pointer(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

struct hp_sim {
  SimBase *impl;
};

namespace {

template <class R>
class Sim : public SimBase {
  using C = typename Cplx<R>::T;
  using Acc = typename AccOf<R>::T;
  static constexpr bool FIXED = std::is_same<R, float>::value;

  struct RunHost {
    hp_config cfg;
    Run<R> d;              // descriptor uploaded to d_runs
    int64_t np = 0;
    double qm = -1.0, q = -1.0;
    int Qbits = 0;
    double jbg[3] = {0, 0, 0};
    // FP64 tables for diagnostics
    double2 *tw64 = nullptr;
    double *sym64 = nullptr, *filt64 = nullptr;
    // diagnostics state
    Acc *rho0 = nullptr;   // rho_e at hp_set_background (nullptr: none)
    Acc *rho_prev = nullptr;
    double *rho0_3 = nullptr, *rho_prev_3 = nullptr;  // 3D: FP64 charge density
    int64_t rho_prev_step = -2;
    int row0 = 0, grp0 = 0;  // first items of the run in the row/group lists
    bool has_ant = false;    // moving antenna (hp_set_antenna)
    hp_antenna ant{};
  };

 public:
  ~Sim() override {
    drop_graphs();
    if (capture_stream_) (void)hipStreamDestroy(capture_stream_);
    for (auto &e : events_) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (void *p : allocs_) (void)hipFree(p);
  }

  int init(const hp_config *cfgs, int nruns) {
    HIPCHK(hipGetDevice(&device_));
    {
      int rc;
      if ((rc = scratch_address(device_, &scratch_))) return rc;
    }
    {
      // LDS of the row transforms: ncomp components of n1/2 complex values
      // (three per block up to n1 = 4096, one beyond)
      int lim = 0, n1max = 0;
      HIPCHK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device_));
      long long nrows = 0;
      for (int i = 0; i < nruns; ++i) {
        n1max = std::max(n1max, cfgs[i].n[0]);
        nrows += (long long)cfgs[i].n[1] * (cfgs[i].geom == HP_GEOM_3D ? cfgs[i].n[2] : 1);
      }
      ncomp_ = n1max > 4096 ? 1 : 3;
      // the current's forward transform: one component per block when three
      // per block would leave fewer than about eight blocks per compute unit
      // (2048 x 512: 21.5 instead of 25.7 us; with 16384 rows of 512 one per
      // block is slower, 157 against 109 us)
      ncompj_ = (ncomp_ == 1 || nrows < 2048) ? 1 : 3;
      const size_t need = (size_t)ncomp_ * (n1max / 2) * sizeof(C);
      if (need > (size_t)lim)
        return fail(HP_EINVAL, "n1 = %d needs %zu bytes of LDS per row transform, the device allows %d",
                    n1max, need, lim);
    }
    HIPCHK(hipMalloc(&d_err_, sizeof(unsigned)));
    allocs_.push_back(d_err_);
    HIPCHK(hipMemset(d_err_, 0, sizeof(unsigned)));
    HIPCHK(hipMalloc(&d_step_, sizeof(long long)));
    allocs_.push_back(d_step_);
    HIPCHK(hipMemset(d_step_, 0, sizeof(long long)));
    HIPCHK(hipMalloc(&d_ant_, sizeof(AntennaDev) * std::max(nruns, 1)));
    allocs_.push_back(d_ant_);
    runs_.resize(nruns);
    std::vector<Item> rows, grps, upd, perrun;
    for (int i = 0; i < nruns; ++i) {
      RunHost &h = runs_[i];
      h.cfg = cfgs[i];
      const hp_config &c = cfgs[i];
      Run<R> &d = h.d;
      std::memset(&d, 0, sizeof d);
      d.n1 = c.n[0];
      d.n2 = c.n[1];
      d.dim = c.geom == HP_GEOM_3D ? 3 : 2;
      d.interp = c.interp;
      d.shape = c.shape_order;
      d.n3 = d.dim == 3 ? c.n[2] : 1;
      d.rows = d.n2 * d.n3;
      d.cells = d.n1 * d.rows;
      d.log2n1 = ilog2(d.n1);
      d.sh3 = d.log2n1 + ilog2(d.n2);
      d.nk = d.n1 / 2 + 1;
      d.dt = (R)c.dt;
      d.hdt = (R)(0.5 * c.dt);
      d.idx2 = (R)(1.0 / c.dx[1]);
      d.dtdx1 = (R)(c.dt / c.dx[0]);
      d.dtdx2 = (R)(c.dt / c.dx[1]);
      d.jfx1 = (R)(-c.dx[0] / c.dt);
      d.jfx2 = (R)(-c.dx[1] / c.dt);
      if (d.dim == 3) {
        d.idx3 = (R)(1.0 / c.dx[2]);
        d.dtdx3 = (R)(c.dt / c.dx[2]);
        d.jfx3 = (R)(-c.dx[2] / c.dt);
        d.cj = (float)CJ3;
      }
      d.inv_m = (R)(2.0 / d.n1);
      d.P = c.fixed_shape_bits > 0 ? c.fixed_shape_bits : 20;
      d.inv_wunit = 1.0f;
      d.c3 = (float)(std::ldexp(1.0, 30 - 2 * d.P) / 6.0);
      maxM_ = std::max(maxM_, d.n1 / 2);
      const size_t cells = (size_t)d.cells, kpl = (size_t)d.rows * d.nk;
      int rc;
      if ((rc = alloc(&d.F, 6 * cells))) return rc;
      if ((rc = alloc(&d.Fk[0], 6 * kpl))) return rc;  // FP64 master (both forms)
      if ((rc = alloc(&d.Fk[1], 6 * kpl))) return rc;
      if ((rc = alloc(&d.J[0], 3 * cells))) return rc;
      if ((rc = alloc(&d.J[1], 3 * cells))) return rc;
      if ((rc = alloc(&d.Jk, 3 * kpl))) return rc;
      // x1 tables, computed in FP64 and rounded once
      std::vector<C> tw(d.n1);
      std::vector<double2> tw64(d.n1);
      for (int m = 0; m < d.n1; ++m) {
        const double a = -2.0 * PI * m / d.n1;
        tw[m].x = (R)std::cos(a);
        tw[m].y = (R)std::sin(a);
        tw64[m] = make_double2(std::cos(a), std::sin(a));
      }
      std::vector<double> sym64(4 * d.nk), filt64(d.nk);
      for (int k = 0; k < d.nk; ++k) {
        const double k1 = 2.0 * PI * k / (d.n1 * c.dx[0]);
        const double hh = 0.5 * k1 * c.dx[0];
        const double kk = c.deriv1 ? std::sin(hh) / (0.5 * c.dx[0]) : k1 + dk_mod(c, k1);
        const double v[4] = {-kk * std::sin(hh), kk * std::cos(hh), kk * std::sin(hh),
                             kk * std::cos(hh)};  // i kk exp(+ih), i kk exp(-ih)
        for (int j = 0; j < 4; ++j) sym64[4 * k + j] = v[j];
        filt64[k] = (k <= c.filter_frac * 0.5 * d.n1) ? 1.0 : 0.0;
      }
      C *dtw;
      R *djfac;
      if ((rc = alloc(&dtw, d.n1)) || (rc = alloc(&djfac, 3 * d.nk)) || (rc = alloc(&h.tw64, d.n1)) ||
          (rc = alloc(&h.sym64, 4 * d.nk)) || (rc = alloc(&h.filt64, d.nk)))
        return rc;
      HIPCHK(hipMemcpy(dtw, tw.data(), sizeof(C) * d.n1, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(h.tw64, tw64.data(), sizeof(double2) * d.n1, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(h.sym64, sym64.data(), sizeof(double) * 4 * d.nk, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(h.filt64, filt64.data(), sizeof(double) * d.nk, hipMemcpyHostToDevice));
      d.tw = dtw;
      d.sym = h.sym64;
      d.mdt = c.dt;
      d.mhdt = 0.5 * c.dt;
      d.midx2 = 1.0 / c.dx[1];
      d.midx3 = d.dim == 3 ? 1.0 / c.dx[2] : 0.0;
      d.jfac = djfac;
      if ((rc = upload_jfac(i))) return rc;
      // row-transform items: (run, row, 0) for three components per block,
      // (run, row, component) for one
      h.row0 = (int)rows.size();
      for (int r = 0; r < d.rows; ++r)
        for (int c = 0; c < 3; c += ncompj_) rows.push_back(Item{i, r, ncompj_ == 3 ? 0 : c});
      h.grp0 = (int)grps.size();
      for (int r = 0; r < d.rows; ++r)
        for (int g = 0; g < 6; g += ncomp_) grps.push_back(Item{i, r, ncomp_ == 3 ? g / 3 : g});
      // 2D: one update thread per (strip of KSTRIP rows, kappa1); 3D: per
      // (strip of KSTRIP3 planes, i2, kappa1)
      const int nel =
          (d.dim == 3 ? ((d.n3 + KSTRIP3 - 1) / KSTRIP3) * d.n2 : (d.n2 + KSTRIP - 1) / KSTRIP) * d.nk;
      for (int e = 0; e < nel; e += UPD_BLOCK) upd.push_back(Item{i, e, 0});
      perrun.push_back(Item{i, 0, 0});
    }
    for (int i = 0; i < nruns; ++i)
      if (cfgs[i].sort_interval > 0) sort_interval_ = cfgs[i].sort_interval;
    int rc;
    if ((rc = alloc(&d_stats_, NSTAT))) return rc;
    dim_ = runs_[0].d.dim;
    if (dim_ == 3) {
      tile1_ = TILE1_3D;
      tile2_ = TILE2_3D;
    }
    if ((rc = make_tiles(tile1_, tile2_))) return rc;
    if ((rc = upload_items(perrun, &d_perrun_, &n_perrun_))) return rc;
    if ((rc = alloc(&d_runs_, nruns))) return rc;
    if ((rc = upload_items(rows, &d_rows_, &n_rows_))) return rc;
    if ((rc = upload_items(grps, &d_grps_, &n_grps_))) return rc;
    if ((rc = upload_items(upd, &d_upd_, &n_upd_))) return rc;
    return upload_runs();
  }

  int set_stream(hipStream_t s) override {
    stream_ = s;
    return HP_OK;
  }

  int set_particles(int run, int64_t n, const double *x, const double *u, const double *w,
                    double qm, double q) override {
    RunHost &h = runs_[run];
    Run<R> &d = h.d;
    if (n < 0 || n > 1000000000) return fail(HP_EINVAL, "particle count %lld out of range", (long long)n);
    if (n > 0 && (!x || !u || !w)) return fail(HP_EINVAL, "null particle array");
    if (!std::isfinite(qm) || !std::isfinite(q) || qm == 0.0) return fail(HP_EINVAL, "bad q/m or q");
    const double L1 = h.cfg.dx[0] * d.n1, L2 = h.cfg.dx[1] * d.n2, L3 = h.cfg.dx[2] * d.n3;
    const bool three = d.dim == 3;
    std::vector<int> cell(n), id(n);
    std::vector<R> f1(n), f2(n), f3(three ? n : 0), u1(n), u2(n), u3(n), qw(n);
    std::vector<int> count((size_t)d.cells, 0);
    double qmax = 0.0, qmin = INFINITY;
    for (int64_t p = 0; p < n; ++p) {
      const double x1 = x[p], x2 = x[n + p], x3 = three ? x[2 * n + p] : 0.0;
      if (!std::isfinite(x1) || !std::isfinite(x2) || !std::isfinite(x3) || !std::isfinite(u[p]) ||
          !std::isfinite(u[n + p]) || !std::isfinite(u[2 * n + p]) || !std::isfinite(w[p]))
        return fail(HP_EINVAL, "non-finite particle input at %lld", (long long)p);
      int c1, c2, c3 = 0;
      R g1, g2, g3 = 0;
      split(x1, L1, h.cfg.dx[0], d.n1, c1, g1);
      split(x2, L2, h.cfg.dx[1], d.n2, c2, g2);
      if (three) split(x3, L3, h.cfg.dx[2], d.n3, c3, g3);
      cell[p] = (c3 << d.sh3) | (c2 << d.log2n1) | c1;
      f1[p] = g1;
      f2[p] = g2;
      if (three) f3[p] = g3;
      u1[p] = (R)u[p];
      u2[p] = (R)u[n + p];
      u3[p] = (R)u[2 * n + p];
      const double qwd = q * w[p];
      qw[p] = (R)qwd;
      qmax = std::max(qmax, std::fabs((double)qw[p]));
      qmin = std::min(qmin, std::fabs((double)qw[p]));
      id[p] = (int)p;
      count[((size_t)c3 * d.n2 + c2) * d.n1 + c1]++;
    }
    {
      const int cmax = n > 0 ? *std::max_element(count.begin(), count.end()) : 0;
      int rc;
      if ((rc = fixed_params_for(h, n, qmax, qmin, cmax))) return rc;
    }
    h.qm = qm;
    h.q = q;
    d.qmhdt = (R)(0.5 * qm * h.cfg.dt);
    d.np = (int)n;
    h.np = n;
    int rc;
    if ((rc = alloc_particles(run, n))) return rc;
    Parts<R> &A = d.pt[pp_];
    if ((rc = h2d(A.cell, cell.data(), n)) || (rc = h2d(A.id, id.data(), n)) ||
        (rc = h2d(A.f1, f1.data(), n)) || (rc = h2d(A.f2, f2.data(), n)) ||
        (rc = h2d(A.u1, u1.data(), n)) || (rc = h2d(A.u2, u2.data(), n)) ||
        (rc = h2d(A.u3, u3.data(), n)) || (rc = h2d(A.qw, qw.data(), n)) ||
        (three && (rc = h2d(A.f3, f3.data(), n))))
      return rc;
    if ((rc = upload_jfac(run))) return rc;
    if ((rc = rebuild_sort_items())) return rc;
    if ((rc = upload_runs())) return rc;
    return sort_now(true);
  }

  // Particles from FP64 arrays in device memory: the conversion of
  // set_particles done on the device (same operations, same bits).  A first
  // pass only validates and measures (non-finite input, charges, particles per
  // cell for the headroom) and changes nothing; then the run's arrays are
  // replaced and sorted as by set_particles.
  int set_particles_device(int run, int64_t n, const double *x, const double *u, const double *w,
                           double qm, double q) override {
    RunHost &h = runs_[run];
    Run<R> &d = h.d;
    if (n < 0 || n > 1000000000) return fail(HP_EINVAL, "particle count %lld out of range", (long long)n);
    if (n > 0 && (!device_pointer(x) || !device_pointer(u) || !device_pointer(w)))
      return fail(HP_EINVAL, "particle arrays must be device memory");
    if (!std::isfinite(qm) || !std::isfinite(q) || qm == 0.0) return fail(HP_EINVAL, "bad q/m or q");
    const LoadGeom g{d.dim, d.n1, d.n2, d.n3, d.log2n1, d.sh3,
                     {h.cfg.dx[0] * d.n1, h.cfg.dx[1] * d.n2, h.cfg.dx[2] * d.n3},
                     {h.cfg.dx[0], h.cfg.dx[1], h.cfg.dx[2]}};
    double qmax = 0.0, qmin = INFINITY;
    int cmax = 0;
    if (n > 0) {
      int *count, *dmax;
      unsigned long long *qbits;
      unsigned *bad;
      int rc;
      if ((rc = alloc(&count, (size_t)d.cells)) || (rc = alloc(&dmax, 1)) ||
          (rc = alloc(&qbits, 2)) || (rc = alloc(&bad, 1)))
        return rc;
      const unsigned long long init[2] = {0ull, 0x7ff0000000000000ull};  // 0, +inf
      auto done = [&](int code) {
        release(count); release(dmax); release(qbits); release(bad);
        return code;
      };
      if ((rc = h2d(qbits, init, 2))) return done(rc);
      launch_scan_particles<R>(g, n, x, u, w, q, count, qbits, bad, stream_);
      launch_max_int(count, d.cells, dmax, stream_);
      if (hipGetLastError() != hipSuccess) return done(fail(HP_EDEVICE, "particle scan launch failed"));
      unsigned long long qb[2];
      unsigned flag = 0;
      if ((rc = d2h(qb, qbits, 2)) || (rc = d2h(&flag, bad, 1)) || (rc = d2h(&cmax, dmax, 1)))
        return done(rc);
      done(HP_OK);
      if (flag) return fail(HP_EINVAL, "non-finite particle input");
      std::memcpy(&qmax, &qb[0], sizeof qmax);
      std::memcpy(&qmin, &qb[1], sizeof qmin);
    }
    int rc;
    if ((rc = fixed_params_for(h, n, qmax, qmin, cmax))) return rc;
    h.qm = qm;
    h.q = q;
    d.qmhdt = (R)(0.5 * qm * h.cfg.dt);
    d.np = (int)n;
    h.np = n;
    if ((rc = alloc_particles(run, n))) return rc;
    launch_load_particles<R>(g, n, x, u, w, q, d.pt[pp_], stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    if ((rc = upload_jfac(run))) return rc;
    if ((rc = rebuild_sort_items())) return rc;
    if ((rc = upload_runs())) return rc;
    return sort_now(true);
  }

  // The real-space field of one component (the copy the next gather reads) into
  // a device buffer of the form's real type; asynchronous on the stream.
  int get_field_device(int run, int comp, void *out, size_t count) override {
    const Run<R> &d = runs_[run].d;
    const size_t cells = (size_t)d.cells;
    if (comp < 0 || comp > 5 || count != cells) return fail(HP_EINVAL, "bad field request");
    if (!device_pointer(out)) return fail(HP_EINVAL, "output must be device memory");
    HIPCHK(hipMemcpyAsync(out, d.F + comp * cells, cells * sizeof(R), hipMemcpyDeviceToDevice,
                          stream_));
    return HP_OK;
  }

  // The particle state in the library's current order into device buffers;
  // asynchronous on the stream.
  int get_particles_device(int run, int64_t n, int32_t *cell, void *off, void *u, void *qw,
                           int32_t *id) override {
    const RunHost &h = runs_[run];
    if (n != h.np) return fail(HP_EINVAL, "particle count mismatch");
    const void *ptrs[5] = {cell, off, u, qw, id};
    for (const void *p : ptrs)
      if (p && !device_pointer(p)) return fail(HP_EINVAL, "outputs must be device memory");
    launch_unload_particles<R>(d_runs_ + run, pp_, (int)n, cell, (R *)off, (R *)u, (R *)qw, id,
                               stream_);
    HIPCHK(hipGetLastError());
    return HP_OK;
  }

  // The current of the last step into a device buffer (FP64, as get_current);
  // asynchronous on the stream.
  int get_current_device(int run, int comp, int corrected, double *out, size_t count) override {
    const RunHost &h = runs_[run];
    const Run<R> &d = h.d;
    const size_t cells = (size_t)d.cells;
    if (comp < 0 || comp > 2 || count != cells) return fail(HP_EINVAL, "bad current request");
    if (!device_pointer(out)) return fail(HP_EINVAL, "output must be device memory");
    if (corrected) {
      if (cur_tmp_n_ < cells) {
        int rc;
        if (cur_tmp_) release(cur_tmp_);
        cur_tmp_ = nullptr;
        cur_tmp_n_ = 0;
        if ((rc = alloc(&cur_tmp_, cells))) return rc;
        cur_tmp_n_ = cells;
      }
      launch_inverse_rows<R>(d.Jk + (size_t)comp * d.rows * d.nk, d.nk, d.n1, d.rows, d.tw,
                             d.inv_m, cur_tmp_, stream_);
      launch_real_to_double<R>(cur_tmp_, (long long)cells, out, stream_);
    } else {
      launch_current_out<Acc>(d.J[parity_ ^ 1] + comp * cells, (long long)cells,
                              acc_factor(h, comp), h.jbg[comp], out, stream_);
    }
    HIPCHK(hipGetLastError());
    return HP_OK;
  }

  // Fixed-point parameters of a run (FP32 form) from its charges |q w| (largest
  // and smallest) and the largest number of particles in one cell: the
  // accumulators' headroom decides the shape and charge bits.
  int fixed_params_for(RunHost &h, int64_t n, double qmax, double qmin, int cmax) {
    Run<R> &d = h.d;
    if (FIXED && n > 0 && d.dim == 3) {
      // 3D: each node's contribution is at most 3.4 cj in integers, a node
      // collects from the particles of 4 x 4 x 4 cells
      if (!(qmax > 0.0)) return fail(HP_EINVAL, "all particle charges are zero");
      if (64.0 * std::max(cmax, 1) * 4.0 * CJ3 >= std::ldexp(1.0, 62))
        return fail(HP_ERANGE, "fixed-point headroom: %d particles in one cell", cmax);
      h.Qbits = 0;
      d.unit_charge = 0;
      d.inv_wunit = (float)(1.0 / qmax);
      d.cj = (float)CJ3;
    } else if (FIXED && n > 0) {
      if (!(qmax > 0.0)) return fail(HP_EINVAL, "all particle charges are zero");
      // per node |J| <= K * (particles per cell) * 2^(2P+Q): keep below 2^62.
      // Quadratic: 3 x 3 cells reach a node, |C| <= 2^P, A <= 1.5 2^P (K = 24);
      // cubic: 5 x 5 cells, A <= (4/3) 2^P (K = 34)
      const double K = d.shape == 3 ? 34.0 : 24.0;
      auto room_for = [&](int P) {
        return std::ldexp(1.0, 62 - 2 * P) / (K * std::max(cmax, 1));
      };
      // automatic shape bits: 22 when all charges are equal (no charge bits
      // needed, products still fit 24 bits), else 20
      if (h.cfg.fixed_shape_bits <= 0)
        d.P = (qmin == qmax && h.cfg.fixed_weight_bits <= 0 && room_for(22) >= 1.0) ? 22 : 20;
      const int P = d.P;
      const double room = room_for(P);
      int Q;
      if (h.cfg.fixed_weight_bits > 0) {
        Q = h.cfg.fixed_weight_bits;
      } else {
        Q = (qmin == qmax) ? 0 : std::min(15, (int)std::floor(std::log2(room)));
      }
      if (Q < 0 || std::ldexp(1.0, Q) > room)
        return fail(HP_ERANGE,
                    "fixed-point headroom: %d particles in one cell with %d charge bits and "
                    "%d shape bits would overflow the 64-bit accumulators",
                    cmax, Q, P);
      h.Qbits = Q;
      d.unit_charge = (Q + P <= 22) ? 1 : 0;  // |Q C| fits 24 signed bits
      d.inv_wunit = (float)(std::ldexp(1.0, Q) / qmax);
      d.c3 = (float)(std::ldexp(1.0, 30 - Q - 2 * P) / 6.0);
    }
    return HP_OK;
  }

  int set_fields(int run, const double *E, const double *B) override {
    RunHost &h = runs_[run];
    Run<R> &d = h.d;
    const size_t cells = (size_t)d.cells;
    std::vector<R> F(6 * cells);
    for (size_t i = 0; i < 3 * cells; ++i) {
      if (!std::isfinite(E[i]) || !std::isfinite(B[i])) return fail(HP_EINVAL, "non-finite field");
      F[i] = (R)E[i];
      F[3 * cells + i] = (R)B[i];
    }
    int rc;
    if ((rc = h2d(d.F, F.data(), 6 * cells))) return rc;
    Launch<R>::fields_to_k(d_runs_, d_grps_ + h.grp0, (6 / ncomp_) * d.rows, parity_, maxM_, ncomp_,
                           stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    return HP_OK;
  }

  int set_background(int run, int rho_from_particles, const double *jbg) override {
    RunHost &h = runs_[run];
    Run<R> &d = h.d;
    for (int c = 0; c < 3; ++c) h.jbg[c] = jbg ? jbg[c] : 0.0;
    if (rho_from_particles) {
      int rc;
      if (d.dim == 3) {
        if (!h.rho0_3 && (rc = alloc(&h.rho0_3, (size_t)d.cells))) return rc;
        if ((rc = deposit_rho3(run, h.rho0_3))) return rc;
      } else {
        if (!h.rho0 && (rc = alloc(&h.rho0, (size_t)d.cells))) return rc;
        if ((rc = deposit_rho(run, h.rho0))) return rc;
      }
    }
    return upload_runs();
  }

  // One eager step (with per-kernel events when profiling).
  void launch_step() {
    const int p = parity_;
    if (sort_interval_ > 0 && since_sort_ >= sort_interval_) {
      mark(HP_K_SORT, true);
      Launch<R>::sort(d_runs_, d_chunks_, n_chunks_, d_perrun_, (int)runs_.size(), pp_, false,
                      stream_);
      mark(HP_K_SORT, false);
      if (n_chunks_ > 0) pp_ ^= 1;
      since_sort_ = 0;
    }
    mark(HP_K_PUSH_DEPOSIT, true);
    if (dim_ == 3)
      Launch<R>::push_deposit3(d_runs_, d_tiles_, n_tiles_, p, pp_, push_lds_, d_err_, d_stats_,
                               stream_);
    else if (runs_[0].d.shape == 3)
      launch_push_cubic<R>(d_runs_, d_tiles_, n_tiles_, p, pp_, push_lds_, all_unit(),
                           runs_[0].cfg.interp == 1, d_err_, stream_);
    else
      Launch<R>::push_deposit(d_runs_, d_tiles_, n_tiles_, p, pp_, push_lds_, all_unit(),
                              runs_[0].cfg.interp == 1, d_err_,
                              d_stats_, stream_);
    mark(HP_K_PUSH_DEPOSIT, false);
    ++since_sort_;
    if (n_ant_ > 0) launch_antenna<R>(d_runs_, d_ant_, n_ant_, ant_maxn2_, p, d_step_, stream_);
    mark(HP_K_FFT_J, true);
    Launch<R>::fft_j(d_runs_, d_rows_, n_rows_, p, maxM_, ncompj_, stream_);
    mark(HP_K_FFT_J, false);
    mark(HP_K_KUPDATE, true);
    if (dim_ == 3)
      Launch<R>::kupdate3(d_runs_, d_upd_, n_upd_, p, stream_);
    else
      Launch<R>::kupdate(d_runs_, d_upd_, n_upd_, p, stream_);
    mark(HP_K_KUPDATE, false);
    mark(HP_K_IFFT_EB, true);
    Launch<R>::ifft_eb(d_runs_, d_grps_, n_grps_, p ^ 1, maxM_, ncomp_, stream_);
    mark(HP_K_IFFT_EB, false);
    if (n_ant_ > 0) launch_step_tick(d_step_, stream_);
    parity_ ^= 1;
    ++step_;
  }

  // ---- moving antenna
  int set_antenna(int run, const hp_antenna *a) override {
    RunHost &h = runs_[run];
    if (h.d.dim != 2) return fail(HP_EINVAL, "run %d: the antenna is built for 2D runs only", run);
    if (a) {
      const double f[9] = {a->x0, a->v, a->t0, a->T, a->K0, a->omega, a->phase, a->x2c, a->waist};
      for (double x : f)
        if (!std::isfinite(x)) return fail(HP_EINVAL, "run %d: non-finite antenna parameter", run);
      if (!(std::fabs(a->v) < 1.0)) return fail(HP_EINVAL, "run %d: antenna speed |v| >= 1", run);
      if (!(a->T > 0.0)) return fail(HP_EINVAL, "run %d: antenna duration T <= 0", run);
    }
    int rc;
    if ((rc = sync())) return rc;
    drop_graphs();
    h.has_ant = a != nullptr;
    if (a) h.ant = *a;
    const long long s = step_;
    HIPCHK(hipMemcpy(d_step_, &s, sizeof s, hipMemcpyHostToDevice));
    return upload_antennas();
  }
  // Device table of the runs' antennas (the accumulator scale follows the
  // run's fixed-point set-up, so it is rebuilt with every upload of the runs).
  int upload_antennas() {
    std::vector<AntennaDev> v;
    int maxn2 = 0;
    for (int i = 0; i < (int)runs_.size(); ++i) {
      const RunHost &h = runs_[i];
      if (!h.has_ant) continue;
      AntennaDev a{};
      a.run = i;
      a.n1 = h.d.n1;
      a.n2 = h.d.n2;
      a.dx1 = h.cfg.dx[0];
      a.dx2 = h.cfg.dx[1];
      a.dt = h.cfg.dt;
      a.x0 = h.ant.x0;
      a.v = h.ant.v;
      a.t0 = h.ant.t0;
      a.T = h.ant.T;
      a.K0 = h.ant.K0;
      a.omega = h.ant.omega;
      a.phase = h.ant.phase;
      a.x2c = h.ant.x2c;
      a.waist = h.ant.waist;
      a.scale = 1.0 / acc_factor(h, 2);
      // FP32 form: a node's contribution (at most 0.75 |K0| / dx1 scaled) must
      // stay well inside the 64-bit accumulators and the rounding helper
      if (FIXED && std::fabs(a.K0) / a.dx1 * a.scale >= std::ldexp(1.0, 50))
        return fail(HP_ERANGE, "run %d: antenna current too large for the fixed-point accumulators", i);
      v.push_back(a);
      maxn2 = std::max(maxn2, a.n2);
    }
    if (!v.empty()) HIPCHK(hipMemcpy(d_ant_, v.data(), sizeof(AntennaDev) * v.size(), hipMemcpyHostToDevice));
    if ((int)v.size() != n_ant_) drop_graphs();
    n_ant_ = (int)v.size();
    ant_maxn2_ = maxn2;
    return HP_OK;
  }

  // A block of one sort followed by K steps (K = sort interval, even), as a
  // HIP graph per (particle parity, step parity): the block starts with a due
  // sort and leaves the step parity unchanged.
  int block_graph(hipGraphExec_t *out) {
    hipGraphExec_t &g = graph_[pp_][parity_];
    if (!g) {
      if (!capture_stream_) HIPCHK(hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking));
      const hipStream_t keep = stream_;
      const int keep_pp = pp_, keep_par = parity_, keep_since = since_sort_;
      const int64_t keep_step = step_;
      const bool keep_prof = profiling_;
      profiling_ = false;
      stream_ = capture_stream_;
      HIPCHK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < sort_interval_; ++k) launch_step();
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(stream_, &graph);
      stream_ = keep;
      pp_ = keep_pp;
      parity_ = keep_par;
      since_sort_ = keep_since;
      step_ = keep_step;
      profiling_ = keep_prof;
      if (e != hipSuccess) return fail(HP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
      const hipError_t ei = hipGraphInstantiateWithFlags(&g, graph, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        g = nullptr;
        return fail(HP_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
      }
    }
    *out = g;
    return HP_OK;
  }

  void drop_graphs() {
    for (auto &row : graph_)
      for (auto &g : row)
        if (g) {
          (void)hipGraphExecDestroy(g);
          g = nullptr;
        }
  }

  int step(int nsteps) override {
    if (nsteps < 0) return fail(HP_EINVAL, "negative step count");
    int left = nsteps;
    while (left > 0) {
      const int K = sort_interval_;
      if (use_graphs_ && !profiling_ && K > 0 && (K & 1) == 0 && since_sort_ >= K && left >= K &&
          n_chunks_ > 0) {
        hipGraphExec_t g;
        int rc;
        if ((rc = block_graph(&g))) return rc;
        HIPCHK(hipGraphLaunch(g, stream_));
        pp_ ^= 1;
        since_sort_ = K;
        step_ += K;
        left -= K;
      } else {
        launch_step();
        --left;
      }
    }
    HIPCHK(hipGetLastError());
    return HP_OK;
  }

  int set_tiling(int t1, int t2, int K) override {
    if (t1 < 1 || t1 > 4096 || t2 < 1 || t2 > 4096 || K < 1 || K > 1024)
      return fail(HP_EINVAL, "tiling %d x %d, sort interval %d out of range", t1, t2, K);
    int rc;
    if ((rc = sync())) return rc;
    if ((rc = make_tiles(t1, t2)) || (rc = upload_runs())) return rc;
    sort_interval_ = K;
    return sort_now(false);
  }

  int get_tiling(hp_tune *out) override {
    out->tile[0] = tile1_;
    out->tile[1] = tile2_;
    out->sort_interval = sort_interval_;
    out->lds_bytes = push_lds_;
    out->ms_per_step = tuned_ms_;
    out->candidates = 0;
    out->steps = 0;
    return HP_OK;
  }

  // Advances every run by nsteps while timing tile shapes, then sort
  // intervals, on the live simulation; keeps the fastest.  The FP32 form's
  // results do not depend on either (integer deposit), so no step is wasted.
  int autotune(int nsteps, hp_tune *out) override {
    if (nsteps < 0) return fail(HP_EINVAL, "negative step count");
    int rc;
    if ((rc = sync())) return rc;
    hipEvent_t ea, eb;
    HIPCHK(hipEventCreate(&ea));
    HIPCHK(hipEventCreate(&eb));
    int left = nsteps, tried = 0;
    auto trial = [&](int t1, int t2, int K, double *ms) -> int {
      int rc2;
      if ((rc2 = set_tiling(t1, t2, K))) return rc2;
      since_sort_ = K;  // the timed block starts with a sort, as in steady state
      const int len = 2 * K;
      HIPCHK(hipEventRecord(ea, stream_));
      if ((rc2 = step(len))) return rc2;
      HIPCHK(hipEventRecord(eb, stream_));
      HIPCHK(hipEventSynchronize(eb));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, ea, eb));
      if ((rc2 = sync())) return rc2;
      *ms = t / len;
      left -= len;
      ++tried;
      return HP_OK;
    };
    int best1 = tile1_, best2 = tile2_, bestK = sort_interval_ > 0 ? sort_interval_ : 16;
    double best = INFINITY;
    // 2D tiles t1 x t2; 3D tiles t1 x t2 x t2
    const std::vector<std::array<int, 2>> shapes =
        dim_ == 3 ? std::vector<std::array<int, 2>>{{8, 4}, {16, 4}, {8, 8}, {16, 2}, {4, 4}, {32, 2}}
                  : std::vector<std::array<int, 2>>{{32, 8}, {64, 4}, {16, 16}, {64, 8}, {32, 16},
                                                    {128, 4}, {16, 8}, {128, 2}};
    std::vector<std::vector<int>> seen;
    const int K0 = bestK;
    // a shape whose current box, grown by one cell of particle spread per
    // axis, no longer fits the LDS budget would send its tiles to global
    // atomics later in a run (a short trial does not see that): skipped
    const int lds_max = (FIXED && dim_ == 3) ? PUSH3_LDS_MAX_FP32 : PUSH_LDS_MAX;
    auto fits = [&](int t1, int t2) {
      for (const RunHost &h : runs_) {
        const long long w = std::min(t1, h.d.n1) + 6, hh = std::min(t2, h.d.n2) + 6;
        const long long dd = h.d.dim == 3 ? std::min(t2, h.d.n3) + 6 : 1;
        if (w * hh * dd * 3 * (long long)sizeof(Acc) > lds_max) return false;
      }
      return true;
    };
    for (const auto &sh : shapes) {
      std::vector<int> key;
      for (const RunHost &h : runs_) {
        key.push_back(std::min(sh[0], h.d.n1));
        key.push_back(std::min(sh[1], h.d.n2));
        key.push_back(std::min(sh[1], h.d.n3));
      }
      if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
      seen.push_back(key);
      if (!fits(sh[0], sh[1])) continue;
      if (left < 2 * K0) break;
      double ms;
      if ((rc = trial(sh[0], sh[1], K0, &ms))) break;
      if (ms < best) { best = ms; best1 = sh[0]; best2 = sh[1]; }
    }
    for (int K : {8, 16, 32, 64, 128}) {
      if (rc || K == K0) continue;
      if (left < 2 * K) break;
      double ms;
      if ((rc = trial(best1, best2, K, &ms))) break;
      if (ms < best) { best = ms; bestK = K; }
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (rc) return rc;
    if ((rc = set_tiling(best1, best2, bestK))) return rc;
    tuned_ms_ = std::isfinite(best) ? best : 0.0;
    if (left > 0 && (rc = step(left))) return rc;
    if (out) {
      get_tiling(out);
      out->candidates = tried;
      out->steps = nsteps;
    }
    return HP_OK;
  }

  int use_graphs(int enable) override {
    use_graphs_ = enable != 0;
    return HP_OK;
  }

  int sync() override {
    HIPCHK(hipStreamSynchronize(stream_));
    unsigned e = 0;
    HIPCHK(hipMemcpy(&e, d_err_, sizeof e, hipMemcpyDeviceToHost));
    if (e) {
      HIPCHK(hipMemset(d_err_, 0, sizeof(unsigned)));
      if (e & ERR_NUMERIC) return fail(HP_ENUMERIC, "non-finite particle momentum or position");
      return fail(HP_ERANGE, "a particle moved a cell or more in one step");
    }
    return HP_OK;
  }

  int get_field(int run, int comp, double *out, size_t count) override {
    const Run<R> &d = runs_[run].d;
    const size_t cells = (size_t)d.cells;
    if (comp < 0 || comp > 5 || count != cells || !out) return fail(HP_EINVAL, "bad field request");
    int rc;
    if ((rc = sync())) return rc;
    std::vector<R> tmp(cells);
    if ((rc = d2h(tmp.data(), d.F + comp * cells, cells))) return rc;
    for (size_t i = 0; i < cells; ++i) out[i] = (double)tmp[i];
    return HP_OK;
  }

  int get_current(int run, int comp, int corrected, double *out, size_t count) override {
    const RunHost &h = runs_[run];
    const Run<R> &d = h.d;
    const size_t cells = (size_t)d.cells;
    if (comp < 0 || comp > 2 || count != cells || !out) return fail(HP_EINVAL, "bad current request");
    int rc;
    if ((rc = sync())) return rc;
    if (corrected) {
      R *tmp;
      if ((rc = alloc(&tmp, cells))) return rc;
      launch_inverse_rows<R>(d.Jk + (size_t)comp * d.rows * d.nk, d.nk, d.n1, d.rows, d.tw,
                             d.inv_m, tmp, stream_);
      std::vector<R> host(cells);
      rc = d2h(host.data(), tmp, cells);
      release(tmp);
      if (rc) return rc;
      for (size_t i = 0; i < cells; ++i) out[i] = (double)host[i];
      return HP_OK;
    }
    std::vector<Acc> raw(cells);
    if ((rc = d2h(raw.data(), d.J[parity_ ^ 1] + comp * cells, cells))) return rc;
    const double f = acc_factor(h, comp);
    for (size_t i = 0; i < cells; ++i) out[i] = (double)raw[i] * f + h.jbg[comp];
    return HP_OK;
  }

  int get_current_fixed(int run, int comp, int64_t *out, size_t count) override {
    if (!FIXED) return fail(HP_EINVAL, "fixed-point current exists only in the FP32 form");
    const Run<R> &d = runs_[run].d;
    const size_t cells = (size_t)d.cells;
    if (comp < 0 || comp > 2 || count != cells || !out) return fail(HP_EINVAL, "bad current request");
    int rc;
    if ((rc = sync())) return rc;
    return d2h((Acc *)out, d.J[parity_ ^ 1] + comp * cells, cells);
  }

  int get_count(int run, int64_t *n) override {
    *n = runs_[run].np;
    return HP_OK;
  }
  int nruns() const override { return (int)runs_.size(); }

  int get_particles(int run, int64_t n, double *x, double *u, double *w, int64_t *id) override {
    const RunHost &h = runs_[run];
    const Run<R> &d = h.d;
    if (n != h.np) return fail(HP_EINVAL, "particle count mismatch");
    int rc;
    if ((rc = sync())) return rc;
    const bool three = d.dim == 3;
    std::vector<int> cell(n), pid(n);
    std::vector<R> f1(n), f2(n), f3(three ? n : 0), a(n), b(n), c(n), qw(n);
    const Parts<R> &A = d.pt[pp_];
    if ((rc = d2h(cell.data(), A.cell, n)) || (rc = d2h(pid.data(), A.id, n)) ||
        (rc = d2h(f1.data(), A.f1, n)) || (rc = d2h(f2.data(), A.f2, n)) ||
        (rc = d2h(a.data(), A.u1, n)) || (rc = d2h(b.data(), A.u2, n)) ||
        (rc = d2h(c.data(), A.u3, n)) || (rc = d2h(qw.data(), A.qw, n)) ||
        (three && (rc = d2h(f3.data(), A.f3, n))))
      return rc;
    for (int64_t p = 0; p < n; ++p) {
      int i1, i2, i3;
      unpack_cell(d, cell[p], i1, i2, i3);
      if (x) {
        x[p] = ((double)i1 + (double)f1[p]) * h.cfg.dx[0];
        x[n + p] = ((double)i2 + (double)f2[p]) * h.cfg.dx[1];
        if (three) x[2 * n + p] = ((double)i3 + (double)f3[p]) * h.cfg.dx[2];
      }
      if (u) {
        u[p] = a[p];
        u[n + p] = b[p];
        u[2 * n + p] = c[p];
      }
      if (w) w[p] = (double)qw[p] / h.q;
      if (id) id[p] = pid[p];
    }
    return HP_OK;
  }

  int get_particles_raw(int run, int64_t n, int32_t *cellout, float *off, float *u, float *qwo,
                        int32_t *id) override {
    if (!FIXED) return fail(HP_EINVAL, "raw particle state exists only in the FP32 form");
    const RunHost &h = runs_[run];
    const Run<R> &d = h.d;
    if (n != h.np) return fail(HP_EINVAL, "particle count mismatch");
    int rc;
    if ((rc = sync())) return rc;
    const Parts<R> &A = d.pt[pp_];
    std::vector<int> cell(n);
    if ((rc = d2h(cell.data(), A.cell, n))) return rc;
    const bool three = d.dim == 3;
    if (cellout)
      for (int64_t p = 0; p < n; ++p) {
        int i1, i2, i3;
        unpack_cell(d, cell[p], i1, i2, i3);
        cellout[p] = i1;
        cellout[n + p] = i2;
        if (three) cellout[2 * n + p] = i3;
      }
    if (off && ((rc = d2h((R *)off, A.f1, n)) || (rc = d2h((R *)off + n, A.f2, n)) ||
                (three && (rc = d2h((R *)off + 2 * n, A.f3, n)))))
      return rc;
    if (u && ((rc = d2h((R *)u, A.u1, n)) || (rc = d2h((R *)u + n, A.u2, n)) ||
              (rc = d2h((R *)u + 2 * n, A.u3, n))))
      return rc;
    if (qwo && (rc = d2h((R *)qwo, A.qw, n))) return rc;
    if (id && (rc = d2h(id, A.id, n))) return rc;
    return HP_OK;
  }

  // 3D diagnostics: energies, kinetic energy, FP64 charge density, Gauss
  // residual over the rows (i2, i3) and the FP64 continuity residual of the
  // last step (the 3D deposit is exact to FP32 rounding, so cont_int is -1).
  int diagnostics3(int run, hp_diag *out) {
    RunHost &h = runs_[run];
    Run<R> &d = h.d;
    const size_t cells = (size_t)d.cells;
    const double dV = h.cfg.dx[0] * h.cfg.dx[1] * h.cfg.dx[2];
    int rc;
    if ((rc = sync())) return rc;
    std::memset(out, 0, sizeof *out);
    out->step = step_;
    const int nb = 256;
    double *part;
    if ((rc = alloc(&part, 6 * nb))) return rc;
    launch_energy<R>(d.F, (long long)cells, part, nb, stream_);
    std::vector<double> hp(6 * nb);
    rc = d2h(hp.data(), part, 6 * nb);
    if (rc) { release(part); return rc; }
    for (int b = 0; b < nb; ++b)
      for (int c = 0; c < 3; ++c) {
        out->W_E[c] += 0.5 * dV * hp[6 * b + c];
        out->W_B[c] += 0.5 * dV * hp[6 * b + 3 + c];
      }
    if (h.np > 0) {
      launch_kinetic<R>(d_runs_ + run, pp_, part, nb, stream_);
      rc = d2h(hp.data(), part, nb);
      if (rc) { release(part); return rc; }
      double sk = 0;
      for (int b = 0; b < nb; ++b) sk += hp[b];
      out->kinetic = sk * dV / h.qm;
    }
    release(part);
    double *rho;
    if ((rc = alloc(&rho, cells))) return rc;
    if ((rc = deposit_rho3(run, rho))) { release(rho); return rc; }
    std::vector<double> rn(cells), r0;
    if ((rc = d2h(rn.data(), rho, cells))) { release(rho); return rc; }
    if (h.rho0_3) {
      r0.resize(cells);
      if ((rc = d2h(r0.data(), h.rho0_3, cells))) { release(rho); return rc; }
    }
    std::vector<double> tot(cells);
    double qsum = 0;
    for (size_t i = 0; i < cells; ++i) {
      tot[i] = h.rho0_3 ? rn[i] - r0[i] : rn[i];
      qsum += rn[i];
    }
    out->charge_total = qsum * dV;
    double *dtot, *rows;
    if ((rc = alloc(&dtot, cells)) || (rc = alloc(&rows, 3 * (size_t)d.rows))) { release(rho); return rc; }
    if ((rc = h2d(dtot, tot.data(), cells))) { release(rho); release(dtot); release(rows); return rc; }
    launch_gauss3<R>(d_runs_ + run, d.rows, d.n1, parity_, dtot, h.tw64, h.sym64, h.filt64,
                     1.0 / h.cfg.dx[1], 1.0 / h.cfg.dx[2], rows, stream_);
    std::vector<double> hr(3 * (size_t)d.rows);
    rc = d2h(hr.data(), rows, 3 * (size_t)d.rows);
    release(dtot);
    release(rows);
    if (rc) { release(rho); return rc; }
    double s2 = 0, smax = 0, sref = 0;
    for (int r = 0; r < d.rows; ++r) {
      s2 += hr[3 * r];
      smax = std::max(smax, hr[3 * r + 1]);
      sref += hr[3 * r + 2];
    }
    out->gauss_l2 = std::sqrt(s2);
    out->gauss_linf = smax;
    out->gauss_ref_l2 = std::sqrt(sref);
    out->cont_linf = -1.0;
    out->cont_int = -1;
    if (h.rho_prev_3 && h.rho_prev_step == step_ - 1 && step_ > 0) {
      const int nbc = 256;
      double *pm;
      if ((rc = alloc(&pm, nbc))) { release(rho); return rc; }
      launch_cont3<Acc>(rho, h.rho_prev_3, d.J[parity_ ^ 1], d.n1, d.n2, d.n3, h.cfg.dt,
                        acc_factor(h, 0), acc_factor(h, 1), acc_factor(h, 2), 1.0 / h.cfg.dx[0],
                        1.0 / h.cfg.dx[1], 1.0 / h.cfg.dx[2], pm, nbc, stream_);
      std::vector<double> hm(nbc);
      rc = d2h(hm.data(), pm, nbc);
      release(pm);
      if (rc) { release(rho); return rc; }
      out->cont_linf = *std::max_element(hm.begin(), hm.end());
    }
    if (h.rho_prev_3) release(h.rho_prev_3);
    h.rho_prev_3 = rho;
    h.rho_prev_step = step_;
    return HP_OK;
  }

  int diagnostics(int run, hp_diag *out) override {
    if (runs_[run].d.dim == 3) return diagnostics3(run, out);
    RunHost &h = runs_[run];
    Run<R> &d = h.d;
    const size_t cells = (size_t)d.n1 * d.n2;
    const double dV = h.cfg.dx[0] * h.cfg.dx[1];
    int rc;
    if ((rc = sync())) return rc;
    std::memset(out, 0, sizeof *out);
    out->step = step_;
    // field energies
    const int nb = 256;
    double *part;
    if ((rc = alloc(&part, 6 * nb))) return rc;
    launch_energy<R>(d.F, (long long)cells, part, nb, stream_);
    std::vector<double> hp(6 * nb);
    rc = d2h(hp.data(), part, 6 * nb);
    if (rc) { release(part); return rc; }
    for (int b = 0; b < nb; ++b)
      for (int c = 0; c < 3; ++c) {
        out->W_E[c] += 0.5 * dV * hp[6 * b + c];
        out->W_B[c] += 0.5 * dV * hp[6 * b + 3 + c];
      }
    if (h.np > 0) {
      launch_kinetic<R>(d_runs_ + run, pp_, part, nb, stream_);
      rc = d2h(hp.data(), part, nb);
      if (rc) { release(part); return rc; }
      double s = 0;
      for (int b = 0; b < nb; ++b) s += hp[b];
      out->kinetic = s * dV / h.qm;
    }
    release(part);
    // charge density now, and Gauss residual
    Acc *rho;
    if ((rc = alloc(&rho, cells))) return rc;
    if ((rc = deposit_rho(run, rho))) { release(rho); return rc; }
    std::vector<Acc> rn(cells), r0;
    if ((rc = d2h(rn.data(), rho, cells))) { release(rho); return rc; }
    if (h.rho0) {
      r0.resize(cells);
      if ((rc = d2h(r0.data(), h.rho0, cells))) { release(rho); return rc; }
    }
    const double rf = rho_factor(h);
    std::vector<double> tot(cells);
    double qsum = 0;
    for (size_t i = 0; i < cells; ++i) {
      const Acc v = h.rho0 ? (Acc)(rn[i] - r0[i]) : rn[i];
      tot[i] = (double)v * rf;
      qsum += (double)rn[i] * rf;
    }
    out->charge_total = qsum * dV;
    double *dtot, *rows;
    if ((rc = alloc(&dtot, cells)) || (rc = alloc(&rows, 3 * (size_t)d.n2))) { release(rho); return rc; }
    if ((rc = h2d(dtot, tot.data(), cells))) { release(rho); release(dtot); release(rows); return rc; }
    launch_gauss<R>(d_runs_ + run, d.n2, d.n1, parity_, dtot, h.tw64, h.sym64, h.filt64,
                    1.0 / h.cfg.dx[1], rows, stream_);
    std::vector<double> hr(3 * d.n2);
    rc = d2h(hr.data(), rows, 3 * d.n2);
    release(dtot);
    release(rows);
    if (rc) { release(rho); return rc; }
    double s2 = 0, smax = 0, sref = 0;
    for (int r = 0; r < d.n2; ++r) {
      s2 += hr[3 * r];
      smax = std::max(smax, hr[3 * r + 1]);
      sref += hr[3 * r + 2];
    }
    out->gauss_l2 = std::sqrt(s2);
    out->gauss_linf = smax;
    out->gauss_ref_l2 = std::sqrt(sref);
    // continuity residual of the last step
    out->cont_linf = -1.0;
    out->cont_int = -1;
    if (h.rho_prev && h.rho_prev_step == step_ - 1 && step_ > 0) {
      const int nbc = 256;
      if (FIXED) {
        long long *pm;
        if ((rc = alloc(&pm, nbc))) { release(rho); return rc; }
        launch_cont_fixed((const long long *)rho, (const long long *)h.rho_prev,
                          (const long long *)d.J[parity_ ^ 1], d.n1, d.n2, pm, nbc, stream_);
        std::vector<long long> hm(nbc);
        rc = d2h(hm.data(), pm, nbc);
        release(pm);
        if (rc) { release(rho); return rc; }
        out->cont_int = *std::max_element(hm.begin(), hm.end());
        // in physical units: integers of rho times rho_factor / dt
        out->cont_linf = 0.5 * (double)out->cont_int * rf / h.cfg.dt;
      } else {
        double *pm;
        if ((rc = alloc(&pm, nbc))) { release(rho); return rc; }
        launch_cont_fp64((const double *)rho, (const double *)h.rho_prev,
                         (const double *)d.J[parity_ ^ 1], d.n1, d.n2, h.cfg.dt,
                         1.0 / h.cfg.dx[0], 1.0 / h.cfg.dx[1], pm, nbc, stream_);
        std::vector<double> hm(nbc);
        rc = d2h(hm.data(), pm, nbc);
        release(pm);
        if (rc) { release(rho); return rc; }
        out->cont_linf = *std::max_element(hm.begin(), hm.end());
      }
    }
    if (h.rho_prev) release(h.rho_prev);
    h.rho_prev = rho;
    h.rho_prev_step = step_;
    return HP_OK;
  }

  // ---- checkpoint: header + per run raw arrays (bit-exact resume)
  int get_state(void *blob, size_t *size) override {
    int rc;
    if ((rc = sync())) return rc;
    size_t need = state_size();
    if (!blob) {
      *size = need;
      return HP_OK;
    }
    if (*size < need) return fail(HP_EINVAL, "state buffer too small (%zu < %zu)", *size, need);
    char *o = (char *)blob;
    auto put = [&](const void *src, size_t bytes) {
      std::memcpy(o, src, bytes);
      o += bytes;
    };
    const int64_t hdr[6] = {0x48504943, 3, (int64_t)runs_.size(), FIXED ? 0 : 1, step_, parity_};
    put(hdr, sizeof hdr);
    for (RunHost &h : runs_) {
      Run<R> &d = h.d;
      const size_t cells = (size_t)d.cells, kpl = (size_t)d.rows * d.nk;
      const bool has_rho0 = d.dim == 3 ? h.rho0_3 != nullptr : h.rho0 != nullptr;
      const double meta[12] = {(double)h.np, h.qm, h.q, (double)h.Qbits, (double)d.inv_wunit,
                               (double)d.c3, h.jbg[0], h.jbg[1], h.jbg[2], has_rho0 ? 1.0 : 0.0,
                               (double)d.P, 0};
      put(meta, sizeof meta);
      const int64_t n = h.np;
      const Parts<R> &A = d.pt[pp_];
      if ((rc = d2h((int *)o, A.cell, n))) return rc; o += sizeof(int) * n;
      if ((rc = d2h((int *)o, A.id, n))) return rc; o += sizeof(int) * n;
      R *arrs[7] = {A.f1, A.f2, A.u1, A.u2, A.u3, A.qw, A.f3};
      for (int k = 0; k < (d.dim == 3 ? 7 : 6); ++k) {
        if ((rc = d2h((R *)o, arrs[k], n))) return rc;
        o += sizeof(R) * n;
      }
      if ((rc = d2h((R *)o, d.F, 6 * cells))) return rc; o += sizeof(R) * 6 * cells;
      if ((rc = d2h((double2 *)o, d.Fk[parity_], 6 * kpl))) return rc; o += sizeof(double2) * 6 * kpl;
      if ((rc = d2h((Acc *)o, d.J[parity_ ^ 1], 3 * cells))) return rc; o += sizeof(Acc) * 3 * cells;
      if ((rc = d2h((C *)o, d.Jk, 3 * kpl))) return rc; o += sizeof(C) * 3 * kpl;
      if (d.dim == 3 && h.rho0_3) {
        if ((rc = d2h((double *)o, h.rho0_3, cells))) return rc;
        o += sizeof(double) * cells;
      } else if (d.dim == 2 && h.rho0) {
        if ((rc = d2h((Acc *)o, h.rho0, cells))) return rc;
        o += sizeof(Acc) * cells;
      }
    }
    *size = need;
    return HP_OK;
  }

  int set_state(const void *blob, size_t size) override {
    const char *o = (const char *)blob;
    const char *end = o + size;
    auto take = [&](void *dst, size_t bytes) {
      if (o + bytes > end) return false;
      std::memcpy(dst, o, bytes);
      o += bytes;
      return true;
    };
    int64_t hdr[6];
    if (!take(hdr, sizeof hdr) || hdr[0] != 0x48504943 || hdr[1] != 3 ||
        hdr[2] != (int64_t)runs_.size() || hdr[3] != (FIXED ? 0 : 1))
      return fail(HP_EINVAL, "state blob does not match this handle");
    int rc;
    if ((rc = sync())) return rc;
    step_ = hdr[4];
    parity_ = (int)hdr[5];
    {
      const long long s = step_;
      HIPCHK(hipMemcpy(d_step_, &s, sizeof s, hipMemcpyHostToDevice));
    }
    for (int i = 0; i < (int)runs_.size(); ++i) {
      RunHost &h = runs_[i];
      Run<R> &d = h.d;
      const size_t cells = (size_t)d.cells, kpl = (size_t)d.rows * d.nk;
      double meta[12];
      if (!take(meta, sizeof meta)) return fail(HP_EINVAL, "truncated state");
      const int64_t n = (int64_t)meta[0];
      const int nR = d.dim == 3 ? 7 : 6;
      const size_t rho_bytes = d.dim == 3 ? sizeof(double) : sizeof(Acc);
      const size_t pbytes = n * (2 * sizeof(int) + nR * sizeof(R));
      const size_t fbytes = sizeof(R) * 6 * cells + sizeof(double2) * 6 * kpl +
                            sizeof(C) * 3 * kpl + sizeof(Acc) * 3 * cells +
                            (meta[9] != 0 ? rho_bytes * cells : 0);
      if (o + pbytes + fbytes > end) return fail(HP_EINVAL, "truncated state");
      h.qm = meta[1];
      h.q = meta[2];
      h.Qbits = (int)meta[3];
      d.inv_wunit = (float)meta[4];
      d.c3 = (float)meta[5];
      d.P = (int)meta[10];
      d.unit_charge = (d.dim == 2 && h.Qbits + d.P <= 22) ? 1 : 0;
      for (int c = 0; c < 3; ++c) h.jbg[c] = meta[6 + c];
      d.qmhdt = (R)(0.5 * h.qm * h.cfg.dt);
      h.np = n;
      d.np = (int)n;
      if ((rc = alloc_particles(i, n))) return rc;
      const Parts<R> &A = d.pt[pp_];
      if ((rc = h2d(A.cell, (const int *)o, n))) return rc; o += sizeof(int) * n;
      if ((rc = h2d(A.id, (const int *)o, n))) return rc; o += sizeof(int) * n;
      R *arrs[7] = {A.f1, A.f2, A.u1, A.u2, A.u3, A.qw, A.f3};
      for (int k = 0; k < nR; ++k) {
        if ((rc = h2d(arrs[k], (const R *)o, n))) return rc;
        o += sizeof(R) * n;
      }
      if ((rc = h2d(d.F, (const R *)o, 6 * cells))) return rc; o += sizeof(R) * 6 * cells;
      if ((rc = h2d(d.Fk[parity_], (const double2 *)o, 6 * kpl))) return rc; o += sizeof(double2) * 6 * kpl;
      if ((rc = h2d(d.J[parity_ ^ 1], (const Acc *)o, 3 * cells))) return rc; o += sizeof(Acc) * 3 * cells;
      HIPCHK(hipMemsetAsync(d.J[parity_], 0, sizeof(Acc) * 3 * cells, stream_));
      if ((rc = h2d(d.Jk, (const C *)o, 3 * kpl))) return rc; o += sizeof(C) * 3 * kpl;
      if (meta[9] != 0 && d.dim == 3) {
        if (!h.rho0_3 && (rc = alloc(&h.rho0_3, cells))) return rc;
        if ((rc = h2d(h.rho0_3, (const double *)o, cells))) return rc;
        o += sizeof(double) * cells;
      } else if (meta[9] != 0) {
        if (!h.rho0 && (rc = alloc(&h.rho0, cells))) return rc;
        if ((rc = h2d(h.rho0, (const Acc *)o, cells))) return rc;
        o += sizeof(Acc) * cells;
      }
      h.rho_prev_step = -2;
      if (h.rho_prev_3) {
        release(h.rho_prev_3);
        h.rho_prev_3 = nullptr;
      }
      if ((rc = upload_jfac(i))) return rc;
    }
    if ((rc = rebuild_sort_items())) return rc;
    if ((rc = upload_runs())) return rc;
    return sort_now(false);
  }

  // Arguments of the deposit entry points: the 2D quadratic integer deposit of
  // a run, n moves with cells inside the grid and offsets in [0,1).
  int check_moves(int run, int64_t n, const int32_t *c0, const float *o0, const int32_t *c1,
                  const float *o1, const float *v3, const float *qw) {
    if (!FIXED) return fail(HP_EINVAL, "the fixed-point deposit exists only in the FP32 form");
    const Run<R> &d = runs_[run].d;
    if (d.dim != 2 || d.shape != 2)
      return fail(HP_EINVAL, "the deposit test hook is for the 2D quadratic integer deposit");
    if (n < 0 || n > 0x7fffffff) return fail(HP_EINVAL, "bad count");
    for (int64_t p = 0; p < n; ++p) {
      if (!(o0[p] >= 0.0f && o0[p] < 1.0f && o0[n + p] >= 0.0f && o0[n + p] < 1.0f &&
            o1[p] >= 0.0f && o1[p] < 1.0f && o1[n + p] >= 0.0f && o1[n + p] < 1.0f))
        return fail(HP_EINVAL, "offset out of [0,1) at %lld", (long long)p);
      if (c0[p] < 0 || c0[p] >= d.n1 || c0[n + p] < 0 || c0[n + p] >= d.n2 || c1[p] < 0 ||
          c1[p] >= d.n1 || c1[n + p] < 0 || c1[n + p] >= d.n2)
        return fail(HP_EINVAL, "cell out of range at %lld", (long long)p);
      if (!std::isfinite(v3[p]) || !std::isfinite(qw[p])) return fail(HP_EINVAL, "non-finite input");
    }
    return HP_OK;
  }

  // The deposit of debug_deposit staged in the process's scratch region
  // instead of fresh allocations: no hipMalloc, no hipFree.  The region is
  // shared by every call on this GPU (calls that overlap race); the
  // accumulators are cleared by a kernel before the deposit.
  int debug_deposit_noalloc(int run, int64_t n, const int32_t *c0, const float *o0,
                            const int32_t *c1, const float *o1, const float *v3, const float *qw,
                            int64_t *J) override {
    int rc;
    if ((rc = check_moves(run, n, c0, o0, c1, o1, v3, qw))) return rc;
    const Run<R> &d = runs_[run].d;
    const size_t cells = (size_t)d.n1 * d.n2;
    if ((size_t)n > NOALLOC_MAX_MOVES)
      return fail(HP_EINVAL, "%lld moves exceed the %zu of the no-allocation deposit", (long long)n,
                  NOALLOC_MAX_MOVES);
    if (cells > NOALLOC_MAX_CELLS)
      return fail(HP_EINVAL, "%zu cells exceed the %zu of the no-allocation deposit", cells,
                  NOALLOC_MAX_CELLS);
    if (!scratch_) return fail(HP_EDEVICE, "no scratch region on this device");
    char *base = (char *)scratch_;
    const size_t M = NOALLOC_MAX_MOVES;
    int *dc0 = (int *)base, *dc1 = (int *)(base + 8 * M);
    float *do0 = (float *)(base + 16 * M), *do1 = (float *)(base + 24 * M);
    float *dv3 = (float *)(base + 32 * M), *dqw = (float *)(base + 36 * M);
    long long *dJ = (long long *)(base + NOALLOC_J_OFFSET);
    if (n > 0 && ((rc = h2d(dc0, c0, 2 * n)) || (rc = h2d(dc1, c1, 2 * n)) ||
                  (rc = h2d(do0, o0, 2 * n)) || (rc = h2d(do1, o1, 2 * n)) ||
                  (rc = h2d(dv3, v3, n)) || (rc = h2d(dqw, qw, n))))
      return rc;
    launch_zero_i64(dJ, (long long)(3 * cells), stream_);
    launch_debug_deposit(d.n1, d.n2, d.P, d.inv_wunit, d.c3, (int)n, dc0, do0, dc1, do1, dv3, dqw,
                         dJ, d_err_, stream_);
    HIPCHK(hipGetLastError());
    if ((rc = d2h((long long *)J, dJ, 3 * cells))) return rc;
    return sync();
  }

  int debug_deposit(int run, int64_t n, const int32_t *c0, const float *o0, const int32_t *c1,
                    const float *o1, const float *v3, const float *qw, int64_t *J) override {
    int rcv;
    if ((rcv = check_moves(run, n, c0, o0, c1, o1, v3, qw))) return rcv;
    const Run<R> &d = runs_[run].d;
    const size_t cells = (size_t)d.n1 * d.n2;
    int *dc0, *dc1;
    float *do0, *do1, *dv3, *dqw;
    long long *dJ;
    int rc;
    const size_t m = n > 0 ? n : 1;
    if ((rc = alloc(&dc0, 2 * m)) || (rc = alloc(&dc1, 2 * m)) || (rc = alloc(&do0, 2 * m)) ||
        (rc = alloc(&do1, 2 * m)) || (rc = alloc(&dv3, m)) || (rc = alloc(&dqw, m)) ||
        (rc = alloc(&dJ, 3 * cells)))
      return rc;
    if (!(n > 0 && ((rc = h2d(dc0, c0, 2 * n)) || (rc = h2d(dc1, c1, 2 * n)) ||
                    (rc = h2d(do0, o0, 2 * n)) || (rc = h2d(do1, o1, 2 * n)) ||
                    (rc = h2d(dv3, v3, n)) || (rc = h2d(dqw, qw, n))))) {
      if (hipMemsetAsync(dJ, 0, sizeof(long long) * 3 * cells, stream_) != hipSuccess) {
        rc = fail(HP_EDEVICE, "clearing the accumulators failed");
      } else {
        launch_debug_deposit(d.n1, d.n2, d.P, d.inv_wunit, d.c3, (int)n, dc0, do0, dc1, do1, dv3,
                             dqw, dJ, d_err_, stream_);
        rc = d2h((long long *)J, dJ, 3 * cells);
      }
    }
    release(dc0); release(dc1); release(do0); release(do1); release(dv3); release(dqw); release(dJ);
    if (rc) return rc;
    return sync();
  }

  int fixed_params(int run, double *out) override {
    if (!FIXED) return fail(HP_EINVAL, "fixed-point parameters exist only in the FP32 form");
    const RunHost &h = runs_[run];
    const bool fw = h.d.dim == 3;  // FP32 weights, integer contributions
    out[0] = fw ? 0 : h.d.P;
    out[1] = h.d.inv_wunit;
    out[2] = fw ? h.d.cj : h.d.c3;
    out[3] = h.Qbits;
    return HP_OK;
  }

  int push_stats(int64_t *out) override {
    int rc;
    if ((rc = sync())) return rc;
    unsigned h[NSTAT];
    if ((rc = d2h(h, d_stats_, NSTAT))) return rc;
    out[0] = h[STAT_FALLBACK];
    out[1] = h[STAT_TILES];
    return HP_OK;
  }

  int profile(int enable) override {
    int rc;
    if ((rc = sync())) return rc;
    HIPCHK(hipMemsetAsync(d_stats_, 0, sizeof(unsigned) * NSTAT, stream_));
    for (auto &e : events_) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    events_.clear();
    for (int k = 0; k < HP_NK; ++k) {
      kms_[k] = 0;
      kn_[k] = 0;
    }
    profiling_ = enable != 0;
    return HP_OK;
  }

  int kernel_times(double *ms, int64_t *n) override {
    int rc;
    if ((rc = sync())) return rc;
    for (auto &e : events_) {
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
      kms_[e.kind] += t;
      kn_[e.kind] += 1;
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    events_.clear();
    for (int k = 0; k < HP_NK; ++k) {
      if (ms) ms[k] = kms_[k];
      if (n) n[k] = kn_[k];
    }
    return HP_OK;
  }

 private:
  template <class T>
  int alloc(T **p, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    if (hipMemsetAsync(q, 0, bytes, stream_) != hipSuccess ||
        hipStreamSynchronize(stream_) != hipSuccess) {
      (void)hipFree(q);
      return fail(HP_EDEVICE, "clearing a new allocation failed");
    }
    allocs_.push_back(q);
    *p = (T *)q;
    return HP_OK;
  }
  void release(void *p) {
    auto it = std::find(allocs_.begin(), allocs_.end(), p);
    if (it != allocs_.end()) {
      (void)hipFree(p);
      allocs_.erase(it);
    }
  }
  template <class T>
  int h2d(T *dst, const T *src, size_t count) {
    if (count == 0) return HP_OK;
    HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    return HP_OK;
  }
  template <class T>
  int d2h(T *dst, const T *src, size_t count) {
    if (count == 0) return HP_OK;
    HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    return HP_OK;
  }
  int upload_items(const std::vector<Item> &v, Item **d, int *n) {
    int rc;
    if ((rc = alloc(d, v.size()))) return rc;
    *n = (int)v.size();
    return h2d(*d, v.data(), v.size());
  }
  int upload_runs() {
    std::vector<Run<R>> v(runs_.size());
    for (size_t i = 0; i < runs_.size(); ++i) {
      v[i] = runs_[i].d;
      // the background in the units of the accumulators, which change with
      // the particles' fixed-point scale
      for (int c = 0; c < 3; ++c) v[i].jbgu[c] = runs_[i].jbg[c] / acc_factor(runs_[i], c);
    }
    const int rc = h2d(d_runs_, v.data(), v.size());
    return rc ? rc : upload_antennas();
  }
  // Sort chunks: (run, first particle, count <= SORT_CHUNK) over all particles.
  // Particle tiles of every run (t1 x t2 cells, clipped to the grid), the
  // push work list and the push LDS budget; the caller uploads the runs and
  // re-sorts.
  int make_tiles(int t1, int t2) {
    drop_graphs();
    std::vector<Item> tiles;
    int maxbox = 0;
    for (int i = 0; i < (int)runs_.size(); ++i) {
      Run<R> &d = runs_[i].d;
      int **arrs[3] = {&d.tile_start, &d.tile_cnt, &d.tile_box};
      for (int **a : arrs)
        if (*a) {
          release(*a);
          *a = nullptr;
        }
      d.T1 = std::min(t1, d.n1);
      d.T2 = std::min(t2, d.n2);
      d.T3 = d.dim == 3 ? std::min(t2, d.n3) : 1;
      d.nt1 = (d.n1 + d.T1 - 1) / d.T1;
      d.nt2 = (d.n2 + d.T2 - 1) / d.T2;
      d.nt3 = (d.n3 + d.T3 - 1) / d.T3;
      d.ntiles = d.nt1 * d.nt2 * d.nt3;
      int rc;
      if ((rc = alloc(&d.tile_start, d.ntiles + 1)) || (rc = alloc(&d.tile_cnt, d.ntiles)) ||
          (rc = alloc(&d.tile_box, 6 * d.ntiles)))
        return rc;
      for (int t = 0; t < d.ntiles; ++t) tiles.push_back(Item{i, t, 0});
      // staged box of a tile whose particles spread SLACK cells beyond it
      const int b1 = std::min(d.T1 + 2 * SLACK1, d.n1) + 6;
      const int b2 = std::min(d.T2 + 2 * SLACK2, d.n2) + 6;
      const int b3 = d.dim == 3 ? std::min(d.T3 + 2 * SLACK2, d.n3) + 6 : 1;
      maxbox = std::max(maxbox, b1 * b2 * b3);
    }
    tile1_ = t1;
    tile2_ = t2;
    // per node: 3 accumulators + 6 staged field values (a 3D tile whose two
    // boxes do not fit gathers its fields through the cache; the 3D FP64 form
    // always does, it was measured faster so)
    const int node_bytes = FIXED ? 48 : (dim_ == 3 ? 24 : 72);
    const int lds_max = (FIXED && dim_ == 3) ? PUSH3_LDS_MAX_FP32 : PUSH_LDS_MAX;
    push_lds_ = std::min(lds_max, std::max(PUSH_LDS_MIN, ((maxbox * node_bytes + 1023) / 1024) * 1024));
    if (d_tiles_) release(d_tiles_);
    d_tiles_ = nullptr;
    n_tiles_ = 0;
    return tiles.empty() ? HP_OK : upload_items(tiles, &d_tiles_, &n_tiles_);
  }

  // every run with particles has the 24-bit product bound (FP32 form)
  bool all_unit() const {
    if (!FIXED) return false;
    for (const RunHost &h : runs_)
      if (h.np > 0 && !h.d.unit_charge) return false;
    return true;
  }

  int rebuild_sort_items() {
    drop_graphs();  // captured launches hold the old item lists and counts
    std::vector<Item> items;
    for (int i = 0; i < (int)runs_.size(); ++i)
      for (int64_t p = 0; p < runs_[i].np; p += SORT_CHUNK)
        items.push_back(Item{i, (int)p, (int)std::min<int64_t>(SORT_CHUNK, runs_[i].np - p)});
    if (d_chunks_) release(d_chunks_);
    d_chunks_ = nullptr;
    n_chunks_ = 0;
    if (items.empty()) return HP_OK;
    return upload_items(items, &d_chunks_, &n_chunks_);
  }
  // Particle buffers of a run: both sort buffers, released and re-made.
  int alloc_particles(int run, int64_t n) {
    Run<R> &d = runs_[run].d;
    for (int b = 0; b < 2; ++b) {
      Parts<R> &A = d.pt[b];
      void *old[9] = {A.cell, A.id, A.f1, A.f2, A.f3, A.u1, A.u2, A.u3, A.qw};
      for (void *o : old)
        if (o) release(o);
      A.f3 = nullptr;
      int rc;
      if ((rc = alloc(&A.cell, n)) || (rc = alloc(&A.id, n)) || (rc = alloc(&A.f1, n)) ||
          (rc = alloc(&A.f2, n)) || (rc = alloc(&A.u1, n)) || (rc = alloc(&A.u2, n)) ||
          (rc = alloc(&A.u3, n)) || (rc = alloc(&A.qw, n)) ||
          (d.dim == 3 && (rc = alloc(&A.f3, n))))
        return rc;
    }
    return HP_OK;
  }
  // Sort the particles of every run by tile now (into the other buffer).
  // scramble: the particles arrive in cell order (just loaded), so spread each
  // tile's slots over its cells (see k_sort_scatter); otherwise keep the
  // arrival order, already spread.
  int sort_now(bool scramble) {
    Launch<R>::sort(d_runs_, d_chunks_, n_chunks_, d_perrun_, (int)runs_.size(), pp_, scramble,
                    stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    if (n_chunks_ > 0) pp_ ^= 1;
    since_sort_ = 0;
    return HP_OK;
  }
  static void unpack_cell(const Run<R> &d, int cell, int &i1, int &i2, int &i3) {
    i1 = cell & (d.n1 - 1);
    if (d.dim == 3) {
      i2 = (cell >> d.log2n1) & ((1 << (d.sh3 - d.log2n1)) - 1);
      i3 = cell >> d.sh3;
    } else {
      i2 = cell >> d.log2n1;
      i3 = 0;
    }
  }
  int deposit_rho3(int run, double *rho) {
    RunHost &h = runs_[run];
    HIPCHK(hipMemsetAsync(rho, 0, sizeof(double) * (size_t)h.d.cells, stream_));
    launch_rho3<R>(d_runs_ + run, pp_, (int)h.np, rho, stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    return HP_OK;
  }
  // Factor from the deposit accumulator to physical current (before filtering).
  double acc_factor(const RunHost &h, int comp) const {
    if (!FIXED) return 1.0;
    if (h.d.dim == 3)
      return -(h.cfg.dx[comp] / h.cfg.dt) / (6.0 * (double)h.d.inv_wunit * (double)h.d.cj);
    const int P = h.d.P;
    const double iw = (double)h.d.inv_wunit;
    if (comp == 0) return -(h.cfg.dx[0] / h.cfg.dt) / (iw * std::ldexp(1.0, 2 * P + 1));
    if (comp == 1) return -(h.cfg.dx[1] / h.cfg.dt) / (iw * std::ldexp(1.0, 2 * P + 1));
    return 1.0 / (iw * (double)h.d.c3 * 6.0 * std::ldexp(1.0, 2 * P));
  }
  double rho_factor(const RunHost &h) const {
    if (!FIXED) return 1.0;
    return 1.0 / ((double)h.d.inv_wunit * std::ldexp(1.0, 2 * h.d.P));
  }
  int upload_jfac(int run) {
    RunHost &h = runs_[run];
    const Run<R> &d = h.d;
    std::vector<R> jf(3 * d.nk);
    for (int k = 0; k < d.nk; ++k) {
      const double hh = PI * k / d.n1;  // k1 dx1 / 2
      const bool corr = !h.cfg.deriv1 && h.cfg.correct && k > 0;
      // Eq. (11): [k]1,FD / [k]1 (sin(h)/h without the Eq. (29) bump)
      const double k1 = 2.0 * hh / h.cfg.dx[0];
      const double sinc = corr ? (std::sin(hh) / (0.5 * h.cfg.dx[0])) / (k1 + dk_mod(h.cfg, k1)) : 1.0;
      const double filt = (k <= h.cfg.filter_frac * 0.5 * d.n1) ? 1.0 : 0.0;
      jf[3 * k + 0] = (R)(acc_factor(h, 0) * sinc * filt);
      jf[3 * k + 1] = (R)(acc_factor(h, 1) * filt);
      jf[3 * k + 2] = (R)(acc_factor(h, 2) * filt);
    }
    return h2d((R *)d.jfac, jf.data(), 3 * d.nk);
  }
  int deposit_rho(int run, Acc *rho) {
    RunHost &h = runs_[run];
    const Run<R> &d = h.d;
    const size_t cells = (size_t)d.n1 * d.n2;
    HIPCHK(hipMemsetAsync(rho, 0, sizeof(Acc) * cells, stream_));
    if (d.shape == 3)
      launch_rho_cubic<R>(d_runs_ + run, pp_, (int)h.np, rho, stream_);
    else if constexpr (FIXED)
      launch_rho_fixed(d_runs_ + run, pp_, (int)h.np, rho, stream_);
    else
      launch_rho_fp64(d_runs_ + run, pp_, (int)h.np, rho, stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    return HP_OK;
  }
  size_t state_size() const {
    size_t s = 6 * sizeof(int64_t);
    for (const RunHost &h : runs_) {
      const size_t cells = (size_t)h.d.cells, kpl = (size_t)h.d.rows * h.d.nk;
      const int nR = h.d.dim == 3 ? 7 : 6;
      const size_t rho = h.d.dim == 3 ? (h.rho0_3 ? sizeof(double) * cells : 0)
                                      : (h.rho0 ? sizeof(Acc) * cells : 0);
      s += 12 * sizeof(double) + h.np * (2 * sizeof(int) + nR * sizeof(R)) + sizeof(R) * 6 * cells +
           sizeof(double2) * 6 * kpl + sizeof(C) * 3 * kpl + sizeof(Acc) * 3 * cells + rho;
    }
    return s;
  }
  // Cell index and offset in [0,1) of a physical position, wrapped periodically.
  static void split(double x, double L, double dx, int n, int &c, R &f) {
    double xw = std::fmod(x, L);
    if (xw < 0) xw += L;
    double xi = xw / dx;
    double cf = std::floor(xi);
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
  void mark(int kind, bool start) {
    if (!profiling_) return;
    if (start) {
      Event2 e;
      e.kind = kind;
      (void)hipEventCreate(&e.a);
      (void)hipEventCreate(&e.b);
      (void)hipEventRecord(e.a, stream_);
      events_.push_back(e);
    } else {
      (void)hipEventRecord(events_.back().b, stream_);
    }
  }

  int device_ = 0;
  hipStream_t stream_ = nullptr;
  std::vector<RunHost> runs_;
  std::vector<void *> allocs_;
  Run<R> *d_runs_ = nullptr;
  Item *d_chunks_ = nullptr, *d_tiles_ = nullptr, *d_perrun_ = nullptr;
  Item *d_rows_ = nullptr, *d_grps_ = nullptr, *d_upd_ = nullptr;
  int n_chunks_ = 0, n_tiles_ = 0, n_rows_ = 0, n_grps_ = 0, n_upd_ = 0;
  void *scratch_ = nullptr;  // device address of the process's scratch region (this device)
  int pp_ = 0;             // particle buffer parity
  int n_perrun_ = 0;
  int sort_interval_ = DEFAULT_SORT_INTERVAL, since_sort_ = 0;
  unsigned *d_stats_ = nullptr;
  int tile1_ = TILE1, tile2_ = TILE2, push_lds_ = PUSH_LDS_MIN;
  R *cur_tmp_ = nullptr;  // staging of hp_get_current_device (corrected current)
  size_t cur_tmp_n_ = 0;
  int dim_ = 2;
  double tuned_ms_ = 0.0;
  bool use_graphs_ = true;
  hipGraphExec_t graph_[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipStream_t capture_stream_ = nullptr;
  int maxM_ = 0;
  int ncomp_ = 3;                  // components per row-transform block (1 for n1 > 4096)
  int ncompj_ = 3;                 // the same for the current's forward transform
  int parity_ = 0;
  int64_t step_ = 0;
  unsigned *d_err_ = nullptr;
  long long *d_step_ = nullptr;    // step counter on the device (antenna time)
  AntennaDev *d_ant_ = nullptr;    // antennas of the runs that have one
  int n_ant_ = 0, ant_maxn2_ = 0;
  bool profiling_ = false;
  std::vector<Event2> events_;
  double kms_[HP_NK] = {0};
  int64_t kn_[HP_NK] = {0};
};

// ===================================================================== quasi-3D
// Handle of quasi-3D runs: the hybrid field solver per azimuthal mode (Sec. 5),
// every mode of every run advanced in one launch per stage.  Particles are not
// built for this geometry: the particle calls return HP_EINVAL.
template <class R>
class SimQ : public SimBase {
  using C = typename Cplx<R>::T;

  using A = typename AccQ<R>::T;
  struct RunHostQ {
    hp_config cfg;
    RunQ<R> d;
    int item0 = 0;   // first (6 m + c, row) item of the run
    int jitem0 = 0;  // first (3 m + c, row) item of the run
    double qm = -1.0, q = -1.0;
    double2 *rho_bg = nullptr;  // [M][nr][n1] background charge density, or NULL
    void *pbuf[24] = {nullptr};  // particle arrays (both buffers) and sort keys, ranks
  };

 public:
  ~SimQ() override {
    for (auto &e : events_) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (void *p : allocs_) (void)hipFree(p);
  }

  int init(const hp_config *cfgs, int nruns) {
    HIPCHK(hipGetDevice(&device_));
    runs_.resize(nruns);
    std::vector<Item> rows, upd, gitems, jitems;
    for (int i = 0; i < nruns; ++i) {
      RunHostQ &h = runs_[i];
      h.cfg = cfgs[i];
      const hp_config &c = cfgs[i];
      RunQ<R> &d = h.d;
      std::memset(&d, 0, sizeof d);
      d.n1 = c.n[0];
      d.n2 = c.n[1];
      d.nr = d.n2 + 1;
      d.M = c.n_modes;
      d.interp = c.interp;
      d.log2n1 = ilog2(d.n1);
      d.plane = (long long)d.nr * d.n1;
      d.dz = c.dx[0];
      d.dr = c.dx[1];
      d.dt = c.dt;
      d.hdt = 0.5 * c.dt;
      maxn1_ = std::max(maxn1_, d.n1);
      const size_t total = (size_t)d.M * 6 * d.plane;
      int rc;
      if ((rc = alloc(&d.Fk[0], total)) || (rc = alloc(&d.Fk[1], total)) || (rc = alloc(&d.F, total)))
        return rc;
      std::vector<C> tw(d.n1);
      std::vector<double> sym(4 * d.n1);
      for (int m = 0; m < d.n1; ++m) {
        const double a = -2.0 * PI * m / d.n1;
        tw[m].x = (R)std::cos(a);
        tw[m].y = (R)std::sin(a);
        const int ks = m <= d.n1 / 2 ? m : m - d.n1;  // signed wavenumber index
        const double k1 = 2.0 * PI * ks / (d.n1 * c.dx[0]);
        const double hh = 0.5 * k1 * c.dx[0];
        const double ka = std::fabs(k1);
        const double kk = c.deriv1 ? std::sin(hh) / (0.5 * c.dx[0])
                                   : k1 + (k1 < 0 ? -dk_mod(c, ka) : dk_mod(c, ka));
        // i [k]1 exp(+i h) and i [k]1 exp(-i h)
        sym[4 * m + 0] = -kk * std::sin(hh);
        sym[4 * m + 1] = kk * std::cos(hh);
        sym[4 * m + 2] = kk * std::sin(hh);
        sym[4 * m + 3] = kk * std::cos(hh);
      }
      C *dtw;
      double *dsym;
      if ((rc = alloc(&dtw, d.n1)) || (rc = alloc(&dsym, 4 * d.n1))) return rc;
      HIPCHK(hipMemcpy(dtw, tw.data(), sizeof(C) * d.n1, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(dsym, sym.data(), sizeof(double) * 4 * d.n1, hipMemcpyHostToDevice));
      d.tw = dtw;
      d.sym = dsym;
      // particle-side tables and buffers
      std::vector<double2> tw64(d.n1);
      std::vector<double> filt(d.n1);
      std::vector<R> kfac(2 * d.n1);
      for (int m = 0; m < d.n1; ++m) {
        const double a = -2.0 * PI * m / d.n1;
        tw64[m] = make_double2(std::cos(a), std::sin(a));
        const int ka = std::abs(m <= d.n1 / 2 ? m : m - d.n1);
        const double k1 = 2.0 * PI * ka / (d.n1 * c.dx[0]);
        const double hh = 0.5 * k1 * c.dx[0];
        const bool corr = !c.deriv1 && c.correct && ka > 0;
        const double sinc = corr ? (std::sin(hh) / (0.5 * c.dx[0])) / (k1 + dk_mod(c, k1)) : 1.0;
        filt[m] = (ka <= c.filter_frac * 0.5 * d.n1) ? 1.0 : 0.0;
        kfac[2 * m] = (R)(sinc * filt[m]);
        kfac[2 * m + 1] = (R)filt[m];
      }
      double2 *dtw64;
      double *dfilt, *djconv, *djbg;
      R *dkfac;
      const size_t jn = (size_t)d.M * 3 * d.plane;
      if ((rc = alloc(&dtw64, d.n1)) || (rc = alloc(&dfilt, d.n1)) || (rc = alloc(&dkfac, 2 * d.n1)) ||
          (rc = alloc(&djconv, (size_t)d.M * 3 * d.nr)) || (rc = alloc(&djbg, d.nr)) ||
          (rc = alloc(&d.J[0], 2 * jn)) || (rc = alloc(&d.J[1], 2 * jn)) || (rc = alloc(&d.Jk, jn)))
        return rc;
      HIPCHK(hipMemcpy(dtw64, tw64.data(), sizeof(double2) * d.n1, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(dfilt, filt.data(), sizeof(double) * d.n1, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(dkfac, kfac.data(), sizeof(R) * 2 * d.n1, hipMemcpyHostToDevice));
      d.tw64 = dtw64;
      d.filt64 = dfilt;
      d.kfac = dkfac;
      d.jconv = djconv;
      d.jbgk = djbg;
      d.dtdz = (R)(c.dt / c.dx[0]);
      d.dtdr = (R)(c.dt / c.dx[1]);
      d.rmax = (R)(d.n2 - 3);
      d.wscale = 1;
      h.jitem0 = (int)jitems.size();
      for (int mc = 0; mc < 3 * d.M; ++mc)
        for (int j = 0; j < d.nr; ++j) jitems.push_back(Item{i, mc, j});
      h.item0 = (int)rows.size();
      for (int mc = 0; mc < 6 * d.M; ++mc)
        for (int j = 0; j < d.nr; ++j) rows.push_back(Item{i, mc, j});
      const long long nel = (long long)d.M * d.nr * d.n1;
      for (long long e = 0; e < nel; e += 256) upd.push_back(Item{i, (int)e, 0});
      for (int m = 0; m < d.M; ++m)
        for (int j = 0; j < d.nr; ++j) gitems.push_back(Item{i, m, j});
    }
    int rc;
    if ((rc = upload(rows, &d_rows_, &n_rows_)) || (rc = upload(upd, &d_upd_, &n_upd_)) ||
        (rc = upload(gitems, &d_gauss_, &n_gauss_)) || (rc = upload(jitems, &d_jitems_, &n_jitems_)))
      return rc;
    if ((rc = alloc(&d_runs_, nruns)) || (rc = alloc(&d_err_, 1)) || (rc = set_bins(sbz_, sbr_)))
      return rc;
    for (int i = 0; i < nruns; ++i) set_jconv(i);
    return upload_runs();
  }

  int set_stream(hipStream_t st) override {
    stream_ = st;
    return HP_OK;
  }

  // E, B: complex (re, im interleaved) [3][n2+1][n1] of one mode
  int set_fields_mode(int run, int mode, const double *E, const double *B) override {
    RunHostQ &h = runs_[run];
    RunQ<R> &d = h.d;
    if (mode < 0 || mode >= d.M) return fail(HP_EINVAL, "mode %d out of range", mode);
    int rc;
    if ((rc = sync())) return rc;
    const size_t n = 3 * (size_t)d.plane;
    std::vector<C> tmp(2 * n);
    for (size_t i = 0; i < n; ++i) {
      if (!std::isfinite(E[2 * i]) || !std::isfinite(E[2 * i + 1]) || !std::isfinite(B[2 * i]) ||
          !std::isfinite(B[2 * i + 1]))
        return fail(HP_EINVAL, "non-finite field");
      tmp[i].x = (R)E[2 * i];
      tmp[i].y = (R)E[2 * i + 1];
      tmp[n + i].x = (R)B[2 * i];
      tmp[n + i].y = (R)B[2 * i + 1];
    }
    HIPCHK(hipMemcpy(d.F + (size_t)mode * 6 * d.plane, tmp.data(), sizeof(C) * 2 * n,
                     hipMemcpyHostToDevice));
    LaunchQ<R>::fields_to_k(d_runs_, d_rows_ + h.item0 + mode * 6 * d.nr, 6 * d.nr, parity_, maxn1_,
                            stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    return HP_OK;
  }

  // the mode count shared by every run (the push kernel then has its mode
  // loops unrolled), or 0 when runs differ
  int common_modes() const {
    int m = runs_.empty() ? 0 : runs_[0].d.M;
    for (const auto &h : runs_)
      if (h.d.M != m) return 0;
    return m;
  }

  int step(int nsteps) override {
    if (nsteps < 0) return fail(HP_EINVAL, "negative step count");
    for (int k = 0; k < nsteps; ++k) {
      if (n_push_ > 0 && sort_interval_ > 0 && since_sort_ >= sort_interval_) {
        mark(HP_K_SORT, true);
        for (size_t i = 0; i < runs_.size(); ++i) {
          RunQ<R> &d = runs_[i].d;
          if (d.np <= 0) continue;
          LaunchQ<R>::sort(d_runs_ + i, d.np, d.nbins, stream_);
          std::swap(d.pt, d.pt2);  // the host copy follows the device's swap
        }
        mark(HP_K_SORT, false);
        since_sort_ = 0;
      }
      if (n_push_ > 0) {
        ++since_sort_;
        mark(HP_K_PUSH_DEPOSIT, true);
        LaunchQ<R>::push_deposit(d_runs_, d_push_, n_push_, parity_, common_modes(), d_err_,
                                 stream_);
        mark(HP_K_PUSH_DEPOSIT, false);
        mark(HP_K_FFT_J, true);
        LaunchQ<R>::fft_j(d_runs_, d_jitems_, n_jitems_, parity_, maxn1_, stream_);
        mark(HP_K_FFT_J, false);
        deposited_ = true;
      }
      mark(HP_K_KUPDATE, true);
      LaunchQ<R>::kupdate(d_runs_, d_upd_, n_upd_, parity_, stream_);
      mark(HP_K_KUPDATE, false);
      mark(HP_K_IFFT_EB, true);
      LaunchQ<R>::ifft(d_runs_, d_rows_, n_rows_, parity_ ^ 1, maxn1_, stream_);
      mark(HP_K_IFFT_EB, false);
      parity_ ^= 1;
      ++step_;
    }
    HIPCHK(hipGetLastError());
    return HP_OK;
  }

  int sync() override {
    HIPCHK(hipStreamSynchronize(stream_));
    unsigned e = 0;
    HIPCHK(hipMemcpy(&e, d_err_, sizeof e, hipMemcpyDeviceToHost));
    if (e) {
      HIPCHK(hipMemset(d_err_, 0, sizeof e));
      if (e & ERR_NUMERIC) return fail(HP_ENUMERIC, "non-finite particle momentum or position");
      return fail(HP_ERANGE, "a particle reached r >= (n2 - 3) dr or moved a cell or more");
    }
    return HP_OK;
  }

  // Particles of a run: x[3][n] = (z, x, y) in physical units (r = hypot(x, y)
  // must be below (n2 - 3) dr), u[3][n] = (uz, ux, uy), w[n]; charge q w.
  int set_particles(int run, int64_t n, const double *x, const double *u, const double *w,
                    double qm, double q) override {
    RunHostQ &h = runs_[run];
    RunQ<R> &d = h.d;
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(HP_EINVAL, "particle count out of range");
    if (n > 0 && (!x || !u || !w)) return fail(HP_EINVAL, "null particle arrays");
    if (!std::isfinite(qm) || !std::isfinite(q) || qm == 0 || q == 0)
      return fail(HP_EINVAL, "q/m and q must be finite and non-zero");
    int rc;
    if ((rc = sync())) return rc;
    const double L = d.n1 * d.dz, rlim = (d.n2 - 3) * d.dr;
    std::vector<int> cell(n), cx(n), cy(n), id(n);
    std::vector<R> fz(n), fx(n), fy(n), uz(n), ux(n), uy(n), qw(n);
    // coordinate in cells -> cell index + offset in [0, 1)
    auto split = [](double v, int &c, R &f) {
      c = (int)std::floor(v);
      f = (R)(v - c);
      if (f >= R(1)) {
        f = 0;
        c += 1;
      }
    };
    double wmax = 0;
    for (int64_t p = 0; p < n; ++p) {
      const double z = x[p], xx = x[n + p], yy = x[2 * n + p];
      if (!std::isfinite(z) || !std::isfinite(xx) || !std::isfinite(yy) || !std::isfinite(u[p]) ||
          !std::isfinite(u[n + p]) || !std::isfinite(u[2 * n + p]) || !std::isfinite(w[p]))
        return fail(HP_EINVAL, "non-finite particle data");
      if (!(std::hypot(xx, yy) < rlim))
        return fail(HP_EINVAL, "particle %lld at r >= (n2 - 3) dr", (long long)p);
      double zc = std::fmod(z, L);
      if (zc < 0) zc += L;
      int c;
      split(zc / d.dz, c, fz[p]);
      cell[p] = c & (d.n1 - 1);
      split(xx / d.dr, cx[p], fx[p]);
      split(yy / d.dr, cy[p], fy[p]);
      uz[p] = (R)u[p];
      ux[p] = (R)u[n + p];
      uy[p] = (R)u[2 * n + p];
      qw[p] = (R)(q * w[p]);
      wmax = std::max(wmax, std::fabs(q * w[p]));
      id[p] = (int)p;
    }
    if ((rc = alloc_parts(h, n))) return rc;
    PartsQ<R> &P = d.pt;
    if (n > 0) {
      HIPCHK(hipMemcpy(P.cell, cell.data(), sizeof(int) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.fz, fz.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.ix, cx.data(), sizeof(int) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.fx, fx.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.iy, cy.data(), sizeof(int) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.fy, fy.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.uz, uz.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.ux, ux.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.uy, uy.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.qw, qw.data(), sizeof(R) * n, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(P.id, id.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    }
    d.np = (int)n;
    h.qm = qm;
    h.q = q;
    d.qmhdt = (R)(qm * 0.5 * d.dt);
    // FP32 form: contributions in units of 2^-40 of the largest charge.  One
    // contribution is at most 2^42 max(1, dr) in magnitude and a node collects
    // from the particles of 5 x 5 (z, r) cells: keep the sums below 2^62.
    d.wscale = sizeof(R) == 4 ? (R)(std::ldexp(1.0, 40) / (wmax > 0 ? wmax : 1.0)) : R(1);
    if (sizeof(R) == 4 && n > 0) {
      std::vector<int> count((size_t)d.n1 * d.nr, 0);
      int cmax = 0;
      for (int64_t p = 0; p < n; ++p) {
        const double rr = std::hypot((double)cx[p] + (double)fx[p], (double)cy[p] + (double)fy[p]);
        const int ir = std::min((int)rr, d.nr - 1);
        cmax = std::max(cmax, ++count[(size_t)ir * d.n1 + cell[p]]);
      }
      if (25.0 * cmax * std::ldexp(1.0, 42) * std::max(1.0, d.dr) >= std::ldexp(1.0, 62))
        return fail(HP_ERANGE, "fixed-point headroom: %d particles in one (z, r) cell", cmax);
    }
    set_jconv(run);
    if ((rc = rebuild_push_items())) return rc;
    return upload_runs();
  }

  int get_count(int run, int64_t *n) override {
    *n = runs_[run].d.np;
    return HP_OK;
  }

  int get_particles(int run, int64_t n, double *x, double *u, double *w, int64_t *id) override {
    const RunHostQ &h = runs_[run];
    const RunQ<R> &d = h.d;
    if (n != d.np) return fail(HP_EINVAL, "n must equal the particle count");
    int rc;
    if ((rc = sync())) return rc;
    if (n == 0) return HP_OK;
    const PartsQ<R> &P = d.pt;
    std::vector<int> cell(n), pid(n);
    std::vector<R> a(n);
    HIPCHK(hipMemcpy(cell.data(), P.cell, sizeof(int) * n, hipMemcpyDeviceToHost));
    if (x) {
      HIPCHK(hipMemcpy(a.data(), P.fz, sizeof(R) * n, hipMemcpyDeviceToHost));
      for (int64_t p = 0; p < n; ++p) x[p] = (cell[p] + (double)a[p]) * d.dz;
      HIPCHK(hipMemcpy(cell.data(), P.ix, sizeof(int) * n, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(a.data(), P.fx, sizeof(R) * n, hipMemcpyDeviceToHost));
      for (int64_t p = 0; p < n; ++p) x[n + p] = (cell[p] + (double)a[p]) * d.dr;
      HIPCHK(hipMemcpy(cell.data(), P.iy, sizeof(int) * n, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(a.data(), P.fy, sizeof(R) * n, hipMemcpyDeviceToHost));
      for (int64_t p = 0; p < n; ++p) x[2 * n + p] = (cell[p] + (double)a[p]) * d.dr;
    }
    if (u) {
      R *src[3] = {P.uz, P.ux, P.uy};
      for (int c = 0; c < 3; ++c) {
        HIPCHK(hipMemcpy(a.data(), src[c], sizeof(R) * n, hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < n; ++p) u[c * n + p] = a[p];
      }
    }
    if (w) {
      HIPCHK(hipMemcpy(a.data(), P.qw, sizeof(R) * n, hipMemcpyDeviceToHost));
      for (int64_t p = 0; p < n; ++p) w[p] = a[p] / h.q;
    }
    if (id) {
      HIPCHK(hipMemcpy(pid.data(), P.id, sizeof(int) * n, hipMemcpyDeviceToHost));
      for (int64_t p = 0; p < n; ++p) id[p] = pid[p];
    }
    return HP_OK;
  }

  // rho_from_particles: 0 none, 1 rho_bg = -rho_e(now) (every mode), 2 also the
  // co-drifting current of mode 0 along z from the particles' momenta.  j_bg
  // must be NULL or zero (a uniform current has no place in a bounded column).
  int set_background(int run, int mode, const double *jbg) override {
    RunHostQ &h = runs_[run];
    RunQ<R> &d = h.d;
    if (jbg && (jbg[0] != 0 || jbg[1] != 0 || jbg[2] != 0))
      return fail(HP_EINVAL, "quasi-3D: use rho_from_particles = 2 for a background current");
    if (mode < 0 || mode > 2) return fail(HP_EINVAL, "rho_from_particles must be 0, 1 or 2");
    int rc;
    if ((rc = sync())) return rc;
    const size_t n = (size_t)d.M * d.plane;
    if (mode == 0) {
      if (h.rho_bg) release(h.rho_bg);
      h.rho_bg = nullptr;
      HIPCHK(hipMemset((void *)d.jbgk, 0, sizeof(double) * d.nr));
      return HP_OK;
    }
    if (!h.rho_bg && (rc = alloc(&h.rho_bg, n))) return rc;
    HIPCHK(hipMemset(h.rho_bg, 0, sizeof(double2) * n));
    LaunchQ<R>::rho(d_runs_ + run, d.np, d.M, h.rho_bg, stream_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream_));
    std::vector<double2> t(n);
    HIPCHK(hipMemcpy(t.data(), h.rho_bg, sizeof(double2) * n, hipMemcpyDeviceToHost));
    for (auto &v : t) v = make_double2(-v.x, -v.y);
    HIPCHK(hipMemcpy(h.rho_bg, t.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
    std::vector<double> jb(d.nr, 0.0);
    if (mode == 2) {
      double *tmp;
      if ((rc = alloc(&tmp, d.nr))) return rc;
      LaunchQ<R>::jbg(d_runs_ + run, d.np, tmp, stream_);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(stream_));
      HIPCHK(hipMemcpy(jb.data(), tmp, sizeof(double) * d.nr, hipMemcpyDeviceToHost));
      release(tmp);
      for (auto &v : jb) v *= d.n1;  // the unnormalised transform's kappa = 0 term
    }
    HIPCHK(hipMemcpy((void *)d.jbgk, jb.data(), sizeof(double) * d.nr, hipMemcpyHostToDevice));
    return HP_OK;
  }

  // Deposited current density of the last step, one mode, before correction
  // and filter, without the background: complex [n2+1][n1] interleaved.
  int get_current_mode(int run, int comp, int mode, double *out, size_t count) override {
    const RunQ<R> &d = runs_[run].d;
    if (comp < 0 || comp > 2 || mode < 0 || mode >= d.M || count != 2 * (size_t)d.plane || !out)
      return fail(HP_EINVAL, "bad current request (quasi-3D: complex, count = 2 (n2+1) n1)");
    int rc;
    if ((rc = sync())) return rc;
    std::vector<A> acc(2 * (size_t)d.plane);
    const int par = deposited_ ? (parity_ ^ 1) : parity_;
    HIPCHK(hipMemcpy(acc.data(), d.J[par] + 2 * ((size_t)mode * 3 + comp) * d.plane,
                     sizeof(A) * acc.size(), hipMemcpyDeviceToHost));
    std::vector<double> conv((size_t)d.M * 3 * d.nr);
    HIPCHK(hipMemcpy(conv.data(), d.jconv, sizeof(double) * conv.size(), hipMemcpyDeviceToHost));
    for (int j = 0; j < d.nr; ++j) {
      const double f = conv[((size_t)mode * 3 + comp) * d.nr + j];
      for (int i = 0; i < d.n1; ++i) {
        const size_t o = (size_t)j * d.n1 + i;
        out[2 * o] = (double)acc[2 * o] * f;
        out[2 * o + 1] = (double)acc[2 * o + 1] * f;
      }
    }
    return HP_OK;
  }

  // out: complex (re, im interleaved), count = 2 (n2+1) n1 doubles
  int get_field_mode(int run, int comp, int mode, double *out, size_t count) override {
    const RunQ<R> &d = runs_[run].d;
    if (comp < 0 || comp > 5 || mode < 0 || mode >= d.M || count != 2 * (size_t)d.plane || !out)
      return fail(HP_EINVAL, "bad field request (quasi-3D: complex, count = 2 (n2+1) n1)");
    int rc;
    if ((rc = sync())) return rc;
    std::vector<C> tmp(d.plane);
    HIPCHK(hipMemcpy(tmp.data(), d.F + ((size_t)mode * 6 + comp) * d.plane, sizeof(C) * d.plane,
                     hipMemcpyDeviceToHost));
    for (long long i = 0; i < d.plane; ++i) {
      out[2 * i] = (double)tmp[i].x;
      out[2 * i + 1] = (double)tmp[i].y;
    }
    return HP_OK;
  }
  int get_field(int run, int comp, double *out, size_t count) override {
    return get_field_mode(run, comp, 0, out, count);
  }

  // field energies summed over modes (theta average: |F_0|^2 and |F_m|^2 / 2),
  // volume 2 pi r dr dz per node (pi dr^2/4 dz on the axis, half at the wall),
  // and the vacuum Gauss residual of the master
  int diagnostics(int run, hp_diag *out) override {
    const RunHostQ &h = runs_[run];
    const RunQ<R> &d = h.d;
    int rc;
    if ((rc = sync())) return rc;
    std::memset(out, 0, sizeof *out);
    out->step = step_;
    out->cont_linf = -1.0;
    out->cont_int = -1;
    std::vector<C> F((size_t)d.M * 6 * d.plane);
    HIPCHK(hipMemcpy(F.data(), d.F, sizeof(C) * F.size(), hipMemcpyDeviceToHost));
    for (int m = 0; m < d.M; ++m) {
      const double fm = m == 0 ? 1.0 : 0.5;
      for (int c = 0; c < 6; ++c) {
        const bool half_r = (c == 1 || c == 3 || c == 5);
        double acc = 0;
        for (int j = 0; j < d.nr; ++j) {
          double vol;
          if (half_r) {
            if (j == d.n2) continue;
            vol = 2.0 * PI * (j + 0.5) * d.dr * d.dr * d.dz;
          } else if (j == 0) {
            vol = PI * 0.25 * d.dr * d.dr * d.dz;
          } else {
            vol = 2.0 * PI * j * d.dr * d.dr * d.dz * (j == d.n2 ? 0.5 : 1.0);
          }
          const C *row = F.data() + ((size_t)m * 6 + c) * d.plane + (size_t)j * d.n1;
          double s2 = 0;
          for (int i = 0; i < d.n1; ++i) s2 += (double)row[i].x * row[i].x + (double)row[i].y * row[i].y;
          acc += vol * s2;
        }
        (c < 3 ? out->W_E[c] : out->W_B[c - 3]) += 0.5 * fm * acc;
      }
    }
    // kinetic energy sum (q w / (q/m)) (gamma - 1) of the particles
    if (d.np > 0) {
      std::vector<R> uz(d.np), ux(d.np), uy(d.np), qw(d.np);
      HIPCHK(hipMemcpy(uz.data(), d.pt.uz, sizeof(R) * d.np, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(ux.data(), d.pt.ux, sizeof(R) * d.np, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(uy.data(), d.pt.uy, sizeof(R) * d.np, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(qw.data(), d.pt.qw, sizeof(R) * d.np, hipMemcpyDeviceToHost));
      double ke = 0;
      for (int p = 0; p < d.np; ++p) {
        const double a = uz[p], b = ux[p], c = uy[p];
        ke += (qw[p] / h.qm) * (std::sqrt(1.0 + a * a + b * b + c * c) - 1.0);
      }
      out->kinetic = ke;
    }
    // charge density of the particles plus the background, FP64
    double2 *rho = nullptr;
    const size_t nrho = (size_t)d.M * d.plane;
    if (d.np > 0 || h.rho_bg) {
      if ((rc = alloc(&rho, nrho))) return rc;
      LaunchQ<R>::rho(d_runs_ + run, d.np, d.M, rho, stream_);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(stream_));
      std::vector<double2> t(d.plane);
      HIPCHK(hipMemcpy(t.data(), rho, sizeof(double2) * d.plane, hipMemcpyDeviceToHost));
      double qt = 0;
      for (int j = 0; j < d.nr; ++j) {
        const double V = j == 0 ? PI * 0.25 * d.dr * d.dr * d.dz : 2.0 * PI * j * d.dr * d.dr * d.dz;
        for (int i = 0; i < d.n1; ++i) qt += t[(size_t)j * d.n1 + i].x * V;
      }
      out->charge_total = qt;
      if (h.rho_bg) {
        std::vector<double2> a(nrho), b(nrho);
        HIPCHK(hipMemcpy(a.data(), rho, sizeof(double2) * nrho, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(b.data(), h.rho_bg, sizeof(double2) * nrho, hipMemcpyDeviceToHost));
        for (size_t e = 0; e < nrho; ++e) a[e] = make_double2(a[e].x + b[e].x, a[e].y + b[e].y);
        HIPCHK(hipMemcpy(rho, a.data(), sizeof(double2) * nrho, hipMemcpyHostToDevice));
      }
    }
    const int nit = d.M * d.nr;
    double *rows;
    if ((rc = alloc(&rows, 3 * (size_t)nit))) return rc;
    int first = 0;
    for (int i = 0; i < run; ++i) first += runs_[i].d.M * runs_[i].d.nr;
    LaunchQ<R>::gauss(d_runs_, d_gauss_ + first, nit, parity_, rho, rows, maxn1_, stream_);
    HIPCHK(hipGetLastError());
    std::vector<double> hr(3 * (size_t)nit);
    HIPCHK(hipMemcpy(hr.data(), rows, sizeof(double) * hr.size(), hipMemcpyDeviceToHost));
    release(rows);
    if (rho) release(rho);
    double s2 = 0, smax = 0, sref = 0;
    for (int i = 0; i < nit; ++i) {
      s2 += hr[3 * i];
      smax = std::max(smax, hr[3 * i + 1]);
      sref += hr[3 * i + 2];
    }
    out->gauss_l2 = std::sqrt(s2);
    out->gauss_linf = smax;
    out->gauss_ref_l2 = std::sqrt(sref);
    return HP_OK;
  }

  int profile(int enable) override {
    int rc;
    if ((rc = sync())) return rc;
    for (auto &e : events_) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    events_.clear();
    for (int k = 0; k < HP_NK; ++k) kms_[k] = 0, kn_[k] = 0;
    profiling_ = enable != 0;
    return HP_OK;
  }
  int kernel_times(double *ms, int64_t *n) override {
    int rc;
    if ((rc = sync())) return rc;
    for (auto &e : events_) {
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
      kms_[e.kind] += t;
      kn_[e.kind] += 1;
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    events_.clear();
    for (int k = 0; k < HP_NK; ++k) {
      if (ms) ms[k] = kms_[k];
      if (n) n[k] = kn_[k];
    }
    return HP_OK;
  }
  int nruns() const override { return (int)runs_.size(); }
  int use_graphs(int) override { return HP_OK; }

  // not available for quasi-3D handles
  int na() const { return fail(HP_EINVAL, "not available for quasi-3D runs"); }
  int set_fields(int, const double *, const double *) override { return na(); }
  int get_current(int, int, int, double *, size_t) override { return na(); }
  int get_current_fixed(int, int, int64_t *, size_t) override { return na(); }
  int get_particles_raw(int, int64_t, int32_t *, float *, float *, float *, int32_t *) override {
    return na();
  }
  // Checkpoint of every run: step and parity, per run its particles (11
  // arrays), the real-space fields, the FP64 k-space master of the current
  // parity, the last deposit (for the current reads), the background charge
  // and current.  Resuming from it repeats the same steps bit for bit.
  size_t state_size() const {
    size_t s = 7 * sizeof(int64_t);
    for (const RunHostQ &h : runs_) {
      const RunQ<R> &d = h.d;
      const size_t fn = (size_t)d.M * 6 * d.plane, jn = (size_t)d.M * 3 * d.plane;
      s += 8 * sizeof(double) + (size_t)d.np * (4 * sizeof(int) + 7 * sizeof(R)) +
           fn * (sizeof(C) + sizeof(double2)) + 2 * jn * sizeof(A) + d.nr * sizeof(double) +
           (h.rho_bg ? (size_t)d.M * d.plane * sizeof(double2) : 0);
    }
    return s;
  }

  int get_state(void *blob, size_t *size) override {
    int rc;
    if ((rc = sync())) return rc;
    const size_t need = state_size();
    if (!blob) {
      *size = need;
      return HP_OK;
    }
    if (*size < need) return fail(HP_EINVAL, "state buffer too small (%zu < %zu)", *size, need);
    char *o = (char *)blob;
    auto get = [&](const void *src, size_t bytes) {
      if (bytes) HIPCHK(hipMemcpy(o, src, bytes, hipMemcpyDeviceToHost));
      o += bytes;
      return HP_OK;
    };
    const int64_t hdr[7] = {0x48504951, 1, (int64_t)runs_.size(), sizeof(R) == 4 ? 0 : 1, step_,
                            parity_, deposited_ ? 1 : 0};
    std::memcpy(o, hdr, sizeof hdr);
    o += sizeof hdr;
    for (const RunHostQ &h : runs_) {
      const RunQ<R> &d = h.d;
      const size_t n = (size_t)d.np, fn = (size_t)d.M * 6 * d.plane, jn = (size_t)d.M * 3 * d.plane;
      const double meta[8] = {(double)d.np, h.qm, h.q, (double)d.wscale, h.rho_bg ? 1.0 : 0.0,
                              0, 0, 0};
      std::memcpy(o, meta, sizeof meta);
      o += sizeof meta;
      const PartsQ<R> &P = d.pt;
      const int *ia[4] = {P.cell, P.ix, P.iy, P.id};
      const R *ra[7] = {P.fz, P.fx, P.fy, P.uz, P.ux, P.uy, P.qw};
      for (const int *a : ia)
        if ((rc = get(a, sizeof(int) * n))) return rc;
      for (const R *a : ra)
        if ((rc = get(a, sizeof(R) * n))) return rc;
      if ((rc = get(d.F, sizeof(C) * fn)) || (rc = get(d.Fk[parity_], sizeof(double2) * fn)) ||
          (rc = get(d.J[parity_ ^ 1], 2 * sizeof(A) * jn)) ||
          (rc = get(d.jbgk, sizeof(double) * d.nr)))
        return rc;
      if (h.rho_bg && (rc = get(h.rho_bg, sizeof(double2) * (size_t)d.M * d.plane))) return rc;
    }
    *size = need;
    return HP_OK;
  }

  int set_state(const void *blob, size_t size) override {
    const char *o = (const char *)blob;
    const char *end = o + size;
    int64_t hdr[7];
    if (size < sizeof hdr) return fail(HP_EINVAL, "truncated state");
    std::memcpy(hdr, o, sizeof hdr);
    o += sizeof hdr;
    if (hdr[0] != 0x48504951 || hdr[1] != 1 || hdr[2] != (int64_t)runs_.size() ||
        hdr[3] != (sizeof(R) == 4 ? 0 : 1) || (hdr[5] != 0 && hdr[5] != 1))
      return fail(HP_EINVAL, "state blob does not match this handle");
    int rc;
    if ((rc = sync())) return rc;
    // check the whole blob before changing anything
    {
      const char *q = o;
      for (const RunHostQ &h : runs_) {
        const RunQ<R> &d = h.d;
        double meta[8];
        if (q + sizeof meta > end) return fail(HP_EINVAL, "truncated state");
        std::memcpy(meta, q, sizeof meta);
        q += sizeof meta;
        const double np = meta[0];
        if (!(np >= 0 && np <= (double)((int64_t)1 << 30) && np == std::floor(np)))
          return fail(HP_EINVAL, "bad particle count in state");
        const size_t n = (size_t)np, fn = (size_t)d.M * 6 * d.plane, jn = (size_t)d.M * 3 * d.plane;
        const size_t bytes = n * (4 * sizeof(int) + 7 * sizeof(R)) + fn * (sizeof(C) + sizeof(double2)) +
                             2 * jn * sizeof(A) + d.nr * sizeof(double) +
                             (meta[4] != 0 ? (size_t)d.M * d.plane * sizeof(double2) : 0);
        if ((size_t)(end - q) < bytes) return fail(HP_EINVAL, "truncated state");
        q += bytes;
      }
    }
    step_ = hdr[4];
    parity_ = (int)hdr[5];
    deposited_ = hdr[6] != 0;
    auto put = [&](void *dst, size_t bytes) {
      if (bytes) HIPCHK(hipMemcpy(dst, o, bytes, hipMemcpyHostToDevice));
      o += bytes;
      return HP_OK;
    };
    for (int i = 0; i < (int)runs_.size(); ++i) {
      RunHostQ &h = runs_[i];
      RunQ<R> &d = h.d;
      double meta[8];
      std::memcpy(meta, o, sizeof meta);
      o += sizeof meta;
      const int64_t n = (int64_t)meta[0];
      const size_t fn = (size_t)d.M * 6 * d.plane, jn = (size_t)d.M * 3 * d.plane;
      if ((rc = alloc_parts(h, n))) return rc;
      PartsQ<R> &P = d.pt;
      int *ia[4] = {P.cell, P.ix, P.iy, P.id};
      R *ra[7] = {P.fz, P.fx, P.fy, P.uz, P.ux, P.uy, P.qw};
      for (int *a : ia)
        if ((rc = put(a, sizeof(int) * n))) return rc;
      for (R *a : ra)
        if ((rc = put(a, sizeof(R) * n))) return rc;
      d.np = (int)n;
      h.qm = meta[1];
      h.q = meta[2];
      d.wscale = (R)meta[3];
      d.qmhdt = (R)(h.qm * 0.5 * d.dt);
      if ((rc = put(d.F, sizeof(C) * fn)) || (rc = put(d.Fk[parity_], sizeof(double2) * fn)) ||
          (rc = put(d.J[parity_ ^ 1], 2 * sizeof(A) * jn)) ||
          (rc = put((void *)d.jbgk, sizeof(double) * d.nr)))
        return rc;
      HIPCHK(hipMemset(d.J[parity_], 0, 2 * sizeof(A) * jn));
      if (meta[4] != 0) {
        if (!h.rho_bg && (rc = alloc(&h.rho_bg, (size_t)d.M * d.plane))) return rc;
        if ((rc = put(h.rho_bg, sizeof(double2) * (size_t)d.M * d.plane))) return rc;
      } else if (h.rho_bg) {
        release(h.rho_bg);
        h.rho_bg = nullptr;
      }
      set_jconv(i);
    }
    if ((rc = rebuild_push_items())) return rc;
    return upload_runs();
  }

  int debug_deposit(int, int64_t, const int32_t *, const float *, const int32_t *, const float *,
                    const float *, const float *, int64_t *) override { return na(); }
  int fixed_params(int, double *) override { return na(); }
  int push_stats(int64_t *) override { return na(); }
  // Quasi-3D: sort bins of tile1 z columns x tile2 radial rows, particles
  // re-sorted every sort_interval steps.
  int set_tiling(int t1, int t2, int k) override {
    if (t1 < 1 || t1 > 4096 || t2 < 1 || t2 > 4096 || k < 1 || k > 1024)
      return fail(HP_EINVAL, "tile sizes must be 1..4096 and the sort interval 1..1024");
    int rc;
    if ((rc = sync()) || (rc = set_bins(t1, t2))) return rc;
    sort_interval_ = k;
    return upload_runs();
  }
  int get_tiling(hp_tune *out) override {
    if (!out) return fail(HP_EINVAL, "null output");
    std::memset(out, 0, sizeof *out);
    out->tile[0] = sbz_;
    out->tile[1] = sbr_;
    out->sort_interval = sort_interval_;
    return HP_OK;
  }
  int autotune(int, hp_tune *) override { return na(); }

 private:
  template <class T>
  int alloc(T **p, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    if (hipMemset(q, 0, bytes) != hipSuccess) {
      (void)hipFree(q);
      return fail(HP_EDEVICE, "clearing a new allocation failed");
    }
    allocs_.push_back(q);
    *p = (T *)q;
    return HP_OK;
  }
  // Both particle buffers and the sort's per-particle arrays of a run, for n
  // particles (the previous ones released).
  int alloc_parts(RunHostQ &h, int64_t n) {
    for (void *&b : h.pbuf) {
      if (b) release(b);
      b = nullptr;
    }
    int k = 0, rc;
    for (PartsQ<R> *P : {&h.d.pt, &h.d.pt2}) {
      if ((rc = alloc(&P->cell, n)) || (rc = alloc(&P->fz, n)) || (rc = alloc(&P->ix, n)) ||
          (rc = alloc(&P->fx, n)) || (rc = alloc(&P->iy, n)) || (rc = alloc(&P->fy, n)) ||
          (rc = alloc(&P->uz, n)) || (rc = alloc(&P->ux, n)) || (rc = alloc(&P->uy, n)) ||
          (rc = alloc(&P->qw, n)) || (rc = alloc(&P->id, n)))
        return rc;
      void *bufs[11] = {P->cell, P->fz, P->ix, P->fx, P->iy, P->fy, P->uz, P->ux, P->uy, P->qw, P->id};
      for (void *b : bufs) h.pbuf[k++] = b;
    }
    if ((rc = alloc(&h.d.skey, n)) || (rc = alloc(&h.d.srank, n))) return rc;
    h.pbuf[k++] = h.d.skey;
    h.pbuf[k++] = h.d.srank;
    since_sort_ = sort_interval_;  // sort before the first step
    return HP_OK;
  }
  // Sort bins of sbz z columns x sbr radial rows for every run.
  int set_bins(int sbz, int sbr) {
    for (RunHostQ &h : runs_) {
      RunQ<R> &d = h.d;
      d.sbz = std::min(sbz, d.n1);
      d.sbr = std::min(sbr, d.n2);
      d.nbr = (d.n2 + d.sbr - 1) / d.sbr;
      d.nbins = ((d.n1 + d.sbz - 1) / d.sbz) * d.nbr;
      if (d.sbin) release(d.sbin);
      if (d.ssum) release(d.ssum);
      d.sbin = d.ssum = nullptr;
      int rc;
      if ((rc = alloc(&d.sbin, (size_t)d.nbins + 1)) ||
          (rc = alloc(&d.ssum, (size_t)(d.nbins + 1023) / 1024 + 1)))
        return rc;
    }
    sbz_ = sbz;
    sbr_ = sbr;
    return HP_OK;
  }
  void release(void *p) {
    for (auto it = allocs_.begin(); it != allocs_.end(); ++it)
      if (*it == p) {
        (void)hipFree(p);
        allocs_.erase(it);
        return;
      }
  }
  int upload(const std::vector<Item> &v, Item **d, int *n) {
    int rc;
    if ((rc = alloc(d, v.size()))) return rc;
    *n = (int)v.size();
    if (!v.empty()) HIPCHK(hipMemcpy(*d, v.data(), sizeof(Item) * v.size(), hipMemcpyHostToDevice));
    return HP_OK;
  }
  int upload_runs() {
    std::vector<RunQ<R>> v(runs_.size());
    for (size_t i = 0; i < runs_.size(); ++i) v[i] = runs_[i].d;
    HIPCHK(hipMemcpy(d_runs_, v.data(), sizeof(RunQ<R>) * v.size(), hipMemcpyHostToDevice));
    return HP_OK;
  }
  void mark(int kind, bool start) {
    if (!profiling_) return;
    if (start) {
      Event2 e;
      e.kind = kind;
      (void)hipEventCreate(&e.a);
      (void)hipEventCreate(&e.b);
      (void)hipEventRecord(e.a, stream_);
      events_.push_back(e);
    } else {
      (void)hipEventRecord(events_.back().b, stream_);
    }
  }

  // accumulator -> current density per (m, c, row): charge per step over
  // dt, the fixed-point scale and the face area (z), the r face (r), or the
  // node volume (direct azimuthal current: m = 0, m = 1 on the axis) or
  // 2 pi dr dz (azimuthal flux, m >= 1)
  void set_jconv(int run) {
    RunQ<R> &d = runs_[run].d;
    std::vector<double> cv((size_t)d.M * 3 * d.nr, 0.0);
    const double s = (double)d.wscale * d.dt, dr = d.dr, dz = d.dz;
    for (int m = 0; m < d.M; ++m)
      for (int j = 0; j < d.nr; ++j) {
        const double A = j == 0 ? 0.25 * PI * dr * dr : 2.0 * PI * j * dr * dr;
        double *c = cv.data() + (size_t)m * 3 * d.nr;
        c[j] = 1.0 / (s * A);
        c[d.nr + j] = 1.0 / (s * 2.0 * PI * (j + 0.5) * dr * dz);
        if (m == 0 || (m == 1 && j == 0))
          c[2 * d.nr + j] = 1.0 / (s * A * dz);
        else
          c[2 * d.nr + j] = j == 0 ? 0.0 : 1.0 / (s * 2.0 * PI * dr * dz);
      }
    (void)hipMemcpy((void *)d.jconv, cv.data(), sizeof(double) * cv.size(), hipMemcpyHostToDevice);
  }
  int rebuild_push_items() {
    std::vector<Item> v;
    for (int i = 0; i < (int)runs_.size(); ++i)
      for (int p = 0; p < runs_[i].d.np; p += 256) v.push_back(Item{i, p, 0});
    if (d_push_) release(d_push_);
    d_push_ = nullptr;
    n_push_ = 0;
    if (v.empty()) return HP_OK;
    return upload(v, &d_push_, &n_push_);
  }

  int device_ = 0;
  hipStream_t stream_ = nullptr;
  std::vector<RunHostQ> runs_;
  std::vector<void *> allocs_;
  RunQ<R> *d_runs_ = nullptr;
  Item *d_rows_ = nullptr, *d_upd_ = nullptr, *d_gauss_ = nullptr, *d_jitems_ = nullptr,
       *d_push_ = nullptr;
  int n_rows_ = 0, n_upd_ = 0, n_gauss_ = 0, n_jitems_ = 0, n_push_ = 0, maxn1_ = 0;
  unsigned *d_err_ = nullptr;
  bool deposited_ = false;
  int parity_ = 0;
  int64_t step_ = 0;
  bool profiling_ = false;
  std::vector<Event2> events_;
  double kms_[HP_NK] = {0};
  int64_t kn_[HP_NK] = {0};
  // particle sort: bins of sbz_ z columns x sbr_ radial rows, every
  // sort_interval_ steps, and before the first step after a load (4 x 2
  // cells: a wave's 64 particles of an 8-per-cell column then span few rows;
  // on the 4096 x 256 drift 1.27 ms per push against 1.47 ms for 2 x 4 and
  // 1.93 ms unsorted)
  int sbz_ = 4, sbr_ = 2, sort_interval_ = 64, since_sort_ = 0;
};

int check_sim(hp_sim *s) {
  if (!s || !s->impl) return fail(HP_EINVAL, "null handle");
  return HP_OK;
}

}  // namespace

// ============================================================== C ABI
extern "C" {

const char *hp_last_error(void) { return g_err.c_str(); }

int hp_create(const hp_config *cfgs, int32_t nruns, hp_sim **out) {
  if (!cfgs || !out || nruns < 1 || nruns > 4096) return fail(HP_EINVAL, "bad arguments");
  *out = nullptr;
  const int prec = cfgs[0].precision;
  for (int i = 0; i < nruns; ++i) {
    const hp_config &c = cfgs[i];
    if (c.geom != HP_GEOM_2D && c.geom != HP_GEOM_3D && c.geom != HP_GEOM_Q3D)
      return fail(HP_EINVAL, "run %d: geometry must be 2D or 3D Cartesian or quasi-3D", i);
    if (c.geom == HP_GEOM_Q3D && (c.n_modes < 1 || c.n_modes > 8))
      return fail(HP_EINVAL, "run %d: quasi-3D needs 1..8 azimuthal modes", i);
    if (c.geom != cfgs[0].geom) return fail(HP_EINVAL, "run %d: all runs of a handle share the geometry", i);
    if (c.interp != cfgs[0].interp)
      return fail(HP_EINVAL, "run %d: all runs of a handle share the gather variant", i);
    if (c.geom == HP_GEOM_3D) {
      if (c.n[2] < 4 || !(c.dx[2] > 0))
        return fail(HP_EINVAL, "run %d: n3 >= 4 and dx3 > 0 in 3D", i);
      int b2 = 0;
      while ((1 << b2) < c.n[1]) ++b2;
      if ((int64_t)c.n[0] * ((int64_t)1 << b2) * c.n[2] > ((int64_t)1 << 31) - 1)
        return fail(HP_EINVAL, "run %d: grid too large for the packed cell index", i);
    }
    if (c.precision != prec || (prec != HP_PREC_FP32_FIXED && prec != HP_PREC_FP64))
      return fail(HP_EINVAL, "run %d: precision must be one of the two forms and equal for all runs", i);
    // the row transforms hold n1/2 complex values per component in LDS (one
    // component per block beyond 4096): up to n1 = 8192 for Cartesian runs,
    // 4096 for quasi-3D ones
    const int n1max = c.geom != HP_GEOM_Q3D ? 8192 : 4096;
    if (!is_pow2(c.n[0]) || c.n[0] < 8 || c.n[0] > n1max)
      return fail(HP_EINVAL, "run %d: n1 = %d must be a power of two in [8, %d] for this form", i,
                  c.n[0], n1max);
    if (c.n[1] < 4 || (int64_t)c.n[0] * c.n[1] * (c.geom == HP_GEOM_3D ? c.n[2] : 1) > (int64_t)1 << 30)
      return fail(HP_EINVAL, "run %d: n2 = %d out of range", i, c.n[1]);
    if (!(c.dx[0] > 0) || !(c.dx[1] > 0) || !(c.dt > 0) || !std::isfinite(c.dt))
      return fail(HP_EINVAL, "run %d: non-positive cell size or time step", i);
    if ((c.shape_order != 2 && c.shape_order != 3) || (c.interp != 0 && c.interp != 1))
      return fail(HP_EINVAL, "run %d: shape order 2 or 3; interp 0 (momentum-) or 1 (energy-conserving)", i);
    if (c.shape_order == 3 && c.geom != HP_GEOM_2D)
      return fail(HP_EINVAL, "run %d: the cubic shape is built for 2D runs only", i);
    if (c.shape_order != cfgs[0].shape_order)
      return fail(HP_EINVAL, "run %d: all runs of a handle share the shape order", i);
    if (!(c.filter_frac > 0)) return fail(HP_EINVAL, "run %d: filter_frac must be > 0", i);
    if (c.deriv1 != 0 && c.deriv1 != 1) return fail(HP_EINVAL, "run %d: bad deriv1", i);
    if (c.kmod != 0 && c.kmod != 1) return fail(HP_EINVAL, "run %d: bad kmod", i);
    if (c.fixed_shape_bits != 0 && (c.fixed_shape_bits < 8 || c.fixed_shape_bits > 24))
      return fail(HP_EINVAL, "run %d: fixed_shape_bits in [8, 24]", i);
    if (c.fixed_weight_bits < 0 || c.fixed_weight_bits > 24)
      return fail(HP_EINVAL, "run %d: fixed_weight_bits in [0, 24]", i);
    const double lim = courant_limit(c);
    if (c.dt > lim * (1 + 1e-12))
      return fail(HP_ECOURANT, "run %d: dt = %g exceeds the stability limit %g", i, c.dt, lim);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(HP_EDEVICE, "no HIP device");
  }
  hp_sim *s = new hp_sim;
  int rc;
  if (cfgs[0].geom == HP_GEOM_Q3D) {
    if (prec == HP_PREC_FP32_FIXED) {
      auto *impl = new SimQ<float>();
      s->impl = impl;
      rc = impl->init(cfgs, nruns);
    } else {
      auto *impl = new SimQ<double>();
      s->impl = impl;
      rc = impl->init(cfgs, nruns);
    }
  } else if (prec == HP_PREC_FP32_FIXED) {
    auto *impl = new Sim<float>();
    s->impl = impl;
    rc = impl->init(cfgs, nruns);
  } else {
    auto *impl = new Sim<double>();
    s->impl = impl;
    rc = impl->init(cfgs, nruns);
  }
  if (rc != HP_OK) {
    std::string msg = g_err;
    delete s->impl;
    delete s;
    g_err = msg;
    return rc;
  }
  *out = s;
  return HP_OK;
}

void hp_destroy(hp_sim *sim) {
  if (!sim) return;
  delete sim->impl;
  delete sim;
}

int hp_set_stream(hp_sim *sim, void *stream) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->set_stream((hipStream_t)stream);
}

}  // extern "C"

namespace {
// Validates the handle and the run index, then runs f.
template <class F>
int with_run(hp_sim *sim, int run, F f) {
  int rc = check_sim(sim);
  if (rc) return rc;
  if (run < 0 || run >= sim->impl->nruns()) return fail(HP_EINVAL, "bad run index %d", run);
  return f();
}
}  // namespace

extern "C" {

int hp_set_particles(hp_sim *sim, int32_t run, int32_t species, int64_t n, const double *x,
                     const double *u, const double *w, double q_over_m, double q) {
  return with_run(sim, run, [&] {
    if (species != 0) return fail(HP_EINVAL, "only species 0 is supported");
    return sim->impl->set_particles(run, n, x, u, w, q_over_m, q);
  });
}

int hp_set_particles_device(hp_sim *sim, int32_t run, int32_t species, int64_t n,
                            const double *x, const double *u, const double *w, double q_over_m,
                            double q) {
  return with_run(sim, run, [&] {
    if (species != 0) return fail(HP_EINVAL, "only species 0 is supported");
    return sim->impl->set_particles_device(run, n, x, u, w, q_over_m, q);
  });
}

int hp_get_field_device(hp_sim *sim, int32_t run, int32_t comp, void *out, size_t count) {
  return with_run(sim, run, [&] { return sim->impl->get_field_device(run, comp, out, count); });
}

int hp_get_particles_device(hp_sim *sim, int32_t run, int64_t n, int32_t *cell, void *off,
                            void *u, void *qw, int32_t *id) {
  return with_run(sim, run,
                  [&] { return sim->impl->get_particles_device(run, n, cell, off, u, qw, id); });
}

int hp_get_current_device(hp_sim *sim, int32_t run, int32_t comp, int32_t corrected, double *out,
                          size_t count) {
  return with_run(sim, run,
                  [&] { return sim->impl->get_current_device(run, comp, corrected, out, count); });
}

int hp_set_fields(hp_sim *sim, int32_t run, int32_t mode, const double *E, const double *B) {
  return with_run(sim, run, [&] {
    if (!E || !B) return fail(HP_EINVAL, "null field arrays");
    return sim->impl->set_fields_mode(run, mode, E, B);
  });
}

int hp_set_background(hp_sim *sim, int32_t run, int32_t rho_from_particles, const double *j_bg) {
  return with_run(sim, run, [&] { return sim->impl->set_background(run, rho_from_particles, j_bg); });
}

int hp_set_antenna(hp_sim *sim, int32_t run, const hp_antenna *a) {
  return with_run(sim, run, [&] { return sim->impl->set_antenna(run, a); });
}

int hp_step(hp_sim *sim, int32_t nsteps) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->step(nsteps);
}

int hp_synchronize(hp_sim *sim) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->sync();
}

int hp_get_field(hp_sim *sim, int32_t run, int32_t comp, int32_t mode, double *out, size_t count) {
  return with_run(sim, run, [&] {
    return sim->impl->get_field_mode(run, comp, mode, out, count);
  });
}

int hp_get_current(hp_sim *sim, int32_t run, int32_t comp, int32_t corrected, double *out,
                   size_t count) {
  return with_run(sim, run, [&] { return sim->impl->get_current(run, comp, corrected, out, count); });
}

int hp_get_current_mode(hp_sim *sim, int32_t run, int32_t comp, int32_t mode, double *out,
                        size_t count) {
  return with_run(sim, run, [&] { return sim->impl->get_current_mode(run, comp, mode, out, count); });
}

int hp_get_current_fixed(hp_sim *sim, int32_t run, int32_t comp, int64_t *out, size_t count) {
  return with_run(sim, run, [&] { return sim->impl->get_current_fixed(run, comp, out, count); });
}

int hp_get_particle_count(hp_sim *sim, int32_t run, int64_t *n) {
  return with_run(sim, run, [&] { return sim->impl->get_count(run, n); });
}

int hp_get_particles(hp_sim *sim, int32_t run, int64_t n, double *x, double *u, double *w,
                     int64_t *id) {
  return with_run(sim, run, [&] { return sim->impl->get_particles(run, n, x, u, w, id); });
}

int hp_get_particles_raw(hp_sim *sim, int32_t run, int64_t n, int32_t *cell, float *off, float *u,
                         float *qw, int32_t *id) {
  return with_run(sim, run, [&] { return sim->impl->get_particles_raw(run, n, cell, off, u, qw, id); });
}

int hp_diagnostics(hp_sim *sim, int32_t run, hp_diag *out) {
  return with_run(sim, run, [&] {
    if (!out) return fail(HP_EINVAL, "null output");
    return sim->impl->diagnostics(run, out);
  });
}

int hp_get_state(hp_sim *sim, void *blob, size_t *size) {
  int rc = check_sim(sim);
  if (rc) return rc;
  if (!size) return fail(HP_EINVAL, "null size");
  return sim->impl->get_state(blob, size);
}

int hp_set_state(hp_sim *sim, const void *blob, size_t size) {
  int rc = check_sim(sim);
  if (rc) return rc;
  if (!blob) return fail(HP_EINVAL, "null blob");
  return sim->impl->set_state(blob, size);
}

int hp_debug_deposit(hp_sim *sim, int32_t run, int64_t n, const int32_t *cell0, const float *off0,
                     const int32_t *cell1, const float *off1, const float *v3, const float *qw,
                     int64_t *j_out) {
  return with_run(sim, run, [&] {
    if (n > 0 && (!cell0 || !off0 || !cell1 || !off1 || !v3 || !qw)) return fail(HP_EINVAL, "null input");
    if (!j_out) return fail(HP_EINVAL, "null output");
    return sim->impl->debug_deposit(run, n, cell0, off0, cell1, off1, v3, qw, j_out);
  });
}

int hp_debug_deposit_noalloc(hp_sim *sim, int32_t run, int64_t n, const int32_t *cell0,
                             const float *off0, const int32_t *cell1, const float *off1,
                             const float *v3, const float *qw, int64_t *j_out) {
  return with_run(sim, run, [&] {
    if (n > 0 && (!cell0 || !off0 || !cell1 || !off1 || !v3 || !qw)) return fail(HP_EINVAL, "null input");
    if (!j_out) return fail(HP_EINVAL, "null output");
    return sim->impl->debug_deposit_noalloc(run, n, cell0, off0, cell1, off1, v3, qw, j_out);
  });
}

int hp_get_fixed_params(hp_sim *sim, int32_t run, double *out) {
  return with_run(sim, run, [&] {
    if (!out) return fail(HP_EINVAL, "null output");
    return sim->impl->fixed_params(run, out);
  });
}

int hp_profile(hp_sim *sim, int32_t enable) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->profile(enable);
}

int hp_get_kernel_times(hp_sim *sim, double *ms, int64_t *n) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->kernel_times(ms, n);
}

int hp_set_tiling(hp_sim *sim, int32_t tile1, int32_t tile2, int32_t sort_interval) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->set_tiling(tile1, tile2, sort_interval);
}

int hp_get_tiling(hp_sim *sim, hp_tune *out) {
  int rc = check_sim(sim);
  if (rc) return rc;
  if (!out) return fail(HP_EINVAL, "null output");
  return sim->impl->get_tiling(out);
}

int hp_autotune(hp_sim *sim, int32_t nsteps, hp_tune *out) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->autotune(nsteps, out);
}

int hp_use_graphs(hp_sim *sim, int32_t enable) {
  int rc = check_sim(sim);
  return rc ? rc : sim->impl->use_graphs(enable);
}

int hp_get_push_stats(hp_sim *sim, int64_t *out) {
  int rc = check_sim(sim);
  if (rc) return rc;
  if (!out) return fail(HP_EINVAL, "null output");
  return sim->impl->push_stats(out);
}

}  // extern "C"
