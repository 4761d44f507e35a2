"""ctypes binding of libhpic.so (include/hpic.h): argument marshalling only.

Every step of the PIC path runs in the library's HIP kernels.  If the library
is missing this module raises; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "_lib", "libhpic.so")

HP_OK, HP_EINVAL, HP_ECOURANT, HP_ENOMEM, HP_EDEVICE, HP_ERANGE, HP_ENUMERIC, HP_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
HP_GEOM_2D = 2
HP_GEOM_3D = 3
HP_GEOM_Q3D = 4
HP_PREC_FP32_FIXED, HP_PREC_FP64 = 0, 1
KERNELS = ("push_deposit", "fft_j", "kupdate", "ifft_eb", "sort")
HP_NK = len(KERNELS)

# every function of the C ABI (checked against the header by the tests)
ABI = (
    "hp_create", "hp_destroy", "hp_last_error", "hp_set_stream", "hp_set_particles",
    "hp_set_fields", "hp_set_background", "hp_set_antenna", "hp_step", "hp_synchronize", "hp_get_field",
    "hp_get_current", "hp_get_current_fixed", "hp_get_particle_count", "hp_get_particles",
    "hp_get_particles_raw", "hp_diagnostics", "hp_get_state", "hp_set_state",
    "hp_debug_deposit", "hp_get_fixed_params", "hp_profile", "hp_get_kernel_times",
    "hp_get_push_stats", "hp_use_graphs", "hp_set_tiling", "hp_get_tiling", "hp_autotune",
    "hp_get_current_mode", "hp_set_particles_device", "hp_get_field_device",
    "hp_get_particles_device", "hp_get_current_device", "hp_debug_deposit_noalloc",
)


class HpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hpic error %d: %s" % (code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("geom", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double * 3),
        ("dt", ctypes.c_double), ("shape_order", ctypes.c_int32), ("interp", ctypes.c_int32),
        ("filter_frac", ctypes.c_double), ("deriv1", ctypes.c_int32), ("correct", ctypes.c_int32),
        ("n_modes", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("fixed_shape_bits", ctypes.c_int32), ("fixed_weight_bits", ctypes.c_int32),
        ("sort_interval", ctypes.c_int32), ("kmod", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 7),
    ]


class Tune(ctypes.Structure):
    _fields_ = [
        ("tile", ctypes.c_int32 * 2), ("sort_interval", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32), ("ms_per_step", ctypes.c_double),
        ("candidates", ctypes.c_int32), ("steps", ctypes.c_int32),
    ]

    def as_dict(self):
        return dict(tile=(self.tile[0], self.tile[1]), sort_interval=self.sort_interval,
                    lds_bytes=self.lds_bytes, ms_per_step=self.ms_per_step,
                    candidates=self.candidates, steps=self.steps)


class Antenna(ctypes.Structure):
    """hp_antenna: moving current-sheet antenna of a 2D run."""
    _fields_ = [(k, ctypes.c_double) for k in
                ("x0", "v", "t0", "T", "K0", "omega", "phase", "x2c", "waist")]


class Diag(ctypes.Structure):
    _fields_ = [
        ("W_E", ctypes.c_double * 3), ("W_B", ctypes.c_double * 3), ("kinetic", ctypes.c_double),
        ("gauss_l2", ctypes.c_double), ("gauss_linf", ctypes.c_double),
        ("gauss_ref_l2", ctypes.c_double), ("cont_linf", ctypes.c_double),
        ("cont_int", ctypes.c_int64), ("charge_total", ctypes.c_double), ("step", ctypes.c_int64),
    ]


_lib = None
_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError("libhpic.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIBPATH)
        i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sigs = {
            "hp_create": [ctypes.POINTER(Config), i32, ctypes.POINTER(_P)],
            "hp_destroy": [_P],
            "hp_last_error": [],
            "hp_set_stream": [_P, _P],
            "hp_set_particles": [_P, i32, i32, i64, _P, _P, _P, ctypes.c_double, ctypes.c_double],
            "hp_set_fields": [_P, i32, i32, _P, _P],
            "hp_set_background": [_P, i32, i32, _P],
            "hp_set_antenna": [_P, i32, _P],
            "hp_step": [_P, i32],
            "hp_synchronize": [_P],
            "hp_get_field": [_P, i32, i32, i32, _P, sz],
            "hp_get_current": [_P, i32, i32, i32, _P, sz],
            "hp_get_current_fixed": [_P, i32, i32, _P, sz],
            "hp_get_particle_count": [_P, i32, ctypes.POINTER(i64)],
            "hp_get_particles": [_P, i32, i64, _P, _P, _P, _P],
            "hp_get_particles_raw": [_P, i32, i64, _P, _P, _P, _P, _P],
            "hp_diagnostics": [_P, i32, ctypes.POINTER(Diag)],
            "hp_get_state": [_P, _P, ctypes.POINTER(sz)],
            "hp_set_state": [_P, _P, sz],
            "hp_debug_deposit": [_P, i32, i64, _P, _P, _P, _P, _P, _P, _P],
            "hp_get_fixed_params": [_P, i32, _P],
            "hp_profile": [_P, i32],
            "hp_get_kernel_times": [_P, _P, _P],
            "hp_get_push_stats": [_P, _P],
            "hp_use_graphs": [_P, i32],
            "hp_set_tiling": [_P, i32, i32, i32],
            "hp_get_tiling": [_P, _P],
            "hp_autotune": [_P, i32, _P],
            "hp_get_current_mode": [_P, i32, i32, i32, _P, sz],
            "hp_set_particles_device": [_P, i32, i32, i64, _P, _P, _P, ctypes.c_double,
                                        ctypes.c_double],
            "hp_get_field_device": [_P, i32, i32, _P, sz],
            "hp_get_particles_device": [_P, i32, i64, _P, _P, _P, _P, _P],
            "hp_get_current_device": [_P, i32, i32, i32, _P, sz],
            "hp_debug_deposit_noalloc": [_P, i32, i64, _P, _P, _P, _P, _P, _P, _P],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None if name == "hp_destroy" else (
                ctypes.c_char_p if name == "hp_last_error" else ctypes.c_int)
        _lib = L
    return _lib


def _check(code):
    if code != HP_OK:
        raise HpError(code, lib().hp_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _dptr(t, dtype, shape):
    """Device address of a contiguous device tensor (anything with data_ptr(),
    dtype, shape, is_contiguous()), checked against the expected dtype name
    and shape; None for None."""
    if t is None:
        return None
    if str(t.dtype).split(".")[-1] != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError("expected a %s tensor of shape %s, got %s %s" % (dtype, shape, t.dtype,
                                                                         tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return _P(t.data_ptr())


def config(n1, n2, dx1, dx2, dt, alpha=0.5, deriv1=0, correct=1, precision="fp32",
           shape_bits=0, weight_bits=0, sort_interval=0, n3=0, dx3=0.0, kmod=0, modes=0,
           interp=0, shape=2):
    """Configuration of one run; n3 > 0 makes it a 3D run (n1 x n2 x n3 cells);
    modes > 0 a quasi-3D run (n1 points along z of dx1, n2 radial cells of dx2,
    azimuthal modes 0..modes-1)."""
    c = Config()
    c.geom = HP_GEOM_3D if n3 > 0 else (HP_GEOM_Q3D if modes > 0 else HP_GEOM_2D)
    c.n_modes = int(modes)
    c.n[0], c.n[1], c.n[2] = int(n1), int(n2), int(n3) if n3 > 0 else 1
    c.dx[0], c.dx[1], c.dx[2] = float(dx1), float(dx2), float(dx3) if n3 > 0 else 1.0
    c.dt = float(dt)
    c.shape_order, c.interp = int(shape), int(interp)
    c.filter_frac = float(alpha)
    c.deriv1, c.correct = int(deriv1), int(correct)
    c.precision = HP_PREC_FP32_FIXED if precision == "fp32" else HP_PREC_FP64
    c.fixed_shape_bits, c.fixed_weight_bits = int(shape_bits), int(weight_bits)
    c.sort_interval = int(sort_interval)
    c.kmod = int(kmod)
    return c


class Sim:
    """One handle of the library: nruns independent 2D runs advanced together."""

    def __init__(self, configs, stream=None):
        if isinstance(configs, Config):
            configs = [configs]
        self.cfgs = list(configs)
        arr = (Config * len(self.cfgs))(*self.cfgs)
        h = _P()
        _check(lib().hp_create(arr, len(self.cfgs), ctypes.byref(h)))
        self.h = h
        if stream is not None:
            self.set_stream(stream)

    def close(self):
        if getattr(self, "h", None):
            lib().hp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, run):
        """Grid shape of a run's field arrays: (n2, n1) or (n3, n2, n1)."""
        c = self.cfgs[run]
        if c.geom == HP_GEOM_3D:
            return c.n[2], c.n[1], c.n[0]
        if c.geom == HP_GEOM_Q3D:
            return c.n[1] + 1, c.n[0]
        return c.n[1], c.n[0]

    def dim(self, run):
        """Position components of a particle: 2 (2D), 3 (3D; quasi-3D z, x, y)."""
        return 3 if self.cfgs[run].geom in (HP_GEOM_3D, HP_GEOM_Q3D) else 2

    def set_stream(self, stream):
        s = getattr(stream, "cuda_stream", stream)
        _check(lib().hp_set_stream(self.h, _P(int(s)) if s else None))

    def set_particles(self, run, x, u, w, q_over_m=-1.0, q=-1.0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        n = w.size
        assert x.shape == (self.dim(run), n) and u.shape == (3, n)
        _check(lib().hp_set_particles(self.h, run, 0, n, _ptr(x), _ptr(u), _ptr(w),
                                      float(q_over_m), float(q)))

    def set_particles_device(self, run, x, u, w, q_over_m=-1.0, q=-1.0):
        """Particles from float64 device tensors x[dim][n], u[3][n], w[n]."""
        n = int(w.shape[0])
        _check(lib().hp_set_particles_device(
            self.h, run, 0, n, _dptr(x, "float64", (self.dim(run), n)),
            _dptr(u, "float64", (3, n)), _dptr(w, "float64", (n,)), float(q_over_m), float(q)))

    def _real(self, run):
        return "float32" if self.cfgs[run].precision == HP_PREC_FP32_FIXED else "float64"

    def field_device(self, run, comp, out):
        """Real-space field component comp into the device tensor out (shape
        of the run's grid, float32 in the FP32 form, float64 in the FP64 form);
        asynchronous on the handle's stream."""
        _check(lib().hp_get_field_device(self.h, run, int(comp),
                                         _dptr(out, self._real(run), self.shape(run)),
                                         int(np.prod(self.shape(run)))))

    def current_device(self, run, comp, out, corrected=False):
        """Current component comp of the last step into the float64 device
        tensor out (shape of the run's grid), as current() returns it;
        asynchronous on the handle's stream."""
        _check(lib().hp_get_current_device(self.h, run, int(comp), int(bool(corrected)),
                                           _dptr(out, "float64", self.shape(run)),
                                           int(np.prod(self.shape(run)))))

    def particles_device(self, run, cell=None, off=None, u=None, qw=None, pid=None):
        """Particle state into device tensors (any may be None): cell int32
        [dim][n], off [dim][n], u [3][n], qw [n] in the form's real type, pid
        int32 [n]; asynchronous on the handle's stream."""
        n, d, r = self.count(run), self.dim(run), self._real(run)
        _check(lib().hp_get_particles_device(
            self.h, run, n, _dptr(cell, "int32", (d, n)), _dptr(off, r, (d, n)),
            _dptr(u, r, (3, n)), _dptr(qw, r, (n,)), _dptr(pid, "int32", (n,))))

    def set_fields_mode(self, run, mode, E, B):
        """Quasi-3D: complex E, B [3][n2+1][n1] of azimuthal mode `mode`."""
        sh = (3,) + self.shape(run)
        E = np.ascontiguousarray(E, dtype=np.complex128)
        B = np.ascontiguousarray(B, dtype=np.complex128)
        assert E.shape == sh and B.shape == sh
        _check(lib().hp_set_fields(self.h, run, int(mode), _ptr(E), _ptr(B)))

    def field_mode(self, run, comp, mode):
        """Quasi-3D: complex field component comp of mode `mode`, [n2+1][n1]."""
        out = np.empty(self.shape(run), dtype=np.complex128)
        _check(lib().hp_get_field(self.h, run, comp, int(mode), _ptr(out), 2 * out.size))
        return out

    def set_fields(self, run, E, B):
        sh = (3,) + self.shape(run)
        E = np.ascontiguousarray(E, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        assert E.shape == sh and B.shape == sh
        _check(lib().hp_set_fields(self.h, run, 0, _ptr(E), _ptr(B)))

    def set_background(self, run, rho_from_particles=True, jbg=(0.0, 0.0, 0.0)):
        """rho_from_particles: False/0 none, True/1 rho_bg = -rho_e(now), 2
        (quasi-3D) also the co-drifting current of the particles."""
        j = np.ascontiguousarray(jbg, dtype=np.float64)
        _check(lib().hp_set_background(self.h, run, int(rho_from_particles), _ptr(j)))

    def set_antenna(self, run, x0=None, v=0.0, t0=0.0, T=1.0, K0=0.0, omega=0.0, phase=0.0,
                    x2c=0.0, waist=0.0):
        """Moving antenna of a 2D run (see hp_set_antenna); x0=None removes it."""
        if x0 is None:
            _check(lib().hp_set_antenna(self.h, run, None))
            return
        a = Antenna(float(x0), float(v), float(t0), float(T), float(K0), float(omega),
                    float(phase), float(x2c), float(waist))
        _check(lib().hp_set_antenna(self.h, run, ctypes.byref(a)))

    def step(self, n=1):
        _check(lib().hp_step(self.h, int(n)))

    def set_tiling(self, tile1, tile2, sort_interval):
        _check(lib().hp_set_tiling(self.h, int(tile1), int(tile2), int(sort_interval)))

    def tiling(self):
        t = Tune()
        _check(lib().hp_get_tiling(self.h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, nsteps):
        t = Tune()
        _check(lib().hp_autotune(self.h, int(nsteps), ctypes.byref(t)))
        return t.as_dict()

    def use_graphs(self, enable=True):
        _check(lib().hp_use_graphs(self.h, int(bool(enable))))

    def synchronize(self):
        _check(lib().hp_synchronize(self.h))

    def field(self, run, comp):
        out = np.empty(self.shape(run))
        _check(lib().hp_get_field(self.h, run, comp, 0, _ptr(out), out.size))
        return out

    def fields(self, run):
        F = np.stack([self.field(run, c) for c in range(6)])
        return F[:3], F[3:]

    def current(self, run, comp, corrected=False):
        out = np.empty(self.shape(run))
        _check(lib().hp_get_current(self.h, run, comp, int(corrected), _ptr(out), out.size))
        return out

    def current_mode(self, run, comp, mode):
        """Quasi-3D: deposited current density of the last step, mode `mode`,
        complex [n2+1][n1] (before correction and filter)."""
        out = np.empty(self.shape(run), dtype=np.complex128)
        _check(lib().hp_get_current_mode(self.h, run, comp, int(mode), _ptr(out), 2 * out.size))
        return out

    def current_fixed(self, run):
        out = np.empty((3,) + self.shape(run), dtype=np.int64)
        for c in range(3):
            _check(lib().hp_get_current_fixed(self.h, run, c, _ptr(out[c]), out[c].size))
        return out

    def count(self, run):
        n = ctypes.c_int64()
        _check(lib().hp_get_particle_count(self.h, run, ctypes.byref(n)))
        return n.value

    def particles(self, run):
        n = self.count(run)
        x = np.empty((self.dim(run), n))
        u = np.empty((3, n))
        w = np.empty(n)
        pid = np.empty(n, dtype=np.int64)
        _check(lib().hp_get_particles(self.h, run, n, _ptr(x), _ptr(u), _ptr(w), _ptr(pid)))
        return dict(x=x, u=u, w=w, id=pid)

    def particles_raw(self, run):
        n = self.count(run)
        cell = np.empty((self.dim(run), n), dtype=np.int32)
        off = np.empty((self.dim(run), n), dtype=np.float32)
        u = np.empty((3, n), dtype=np.float32)
        qw = np.empty(n, dtype=np.float32)
        pid = np.empty(n, dtype=np.int32)
        _check(lib().hp_get_particles_raw(self.h, run, n, _ptr(cell), _ptr(off), _ptr(u),
                                          _ptr(qw), _ptr(pid)))
        return dict(cell=cell, off=off, u=u, qw=qw, id=pid)

    def diagnostics(self, run):
        d = Diag()
        _check(lib().hp_diagnostics(self.h, run, ctypes.byref(d)))
        return dict(W_E=list(d.W_E), W_B=list(d.W_B), kinetic=d.kinetic, gauss_l2=d.gauss_l2,
                    gauss_linf=d.gauss_linf, gauss_ref_l2=d.gauss_ref_l2, cont_linf=d.cont_linf,
                    cont_int=d.cont_int, charge_total=d.charge_total, step=d.step)

    def get_state(self):
        size = ctypes.c_size_t(0)
        _check(lib().hp_get_state(self.h, None, ctypes.byref(size)))
        buf = np.empty(size.value, dtype=np.uint8)
        _check(lib().hp_get_state(self.h, _ptr(buf), ctypes.byref(size)))
        return buf[:size.value].tobytes()

    def set_state(self, blob):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        _check(lib().hp_set_state(self.h, _ptr(buf), buf.size))

    def debug_deposit(self, run, cell0, off0, cell1, off1, v3, qw, noalloc=False):
        """Deposit alone on given moves (hp_debug_deposit, or with noalloc
        hp_debug_deposit_noalloc, which stages in the library's fixed region)."""
        n2, n1 = self.shape(run)
        c0 = np.ascontiguousarray(cell0, dtype=np.int32)
        c1 = np.ascontiguousarray(cell1, dtype=np.int32)
        o0 = np.ascontiguousarray(off0, dtype=np.float32)
        o1 = np.ascontiguousarray(off1, dtype=np.float32)
        v3 = np.ascontiguousarray(v3, dtype=np.float32)
        qw = np.ascontiguousarray(qw, dtype=np.float32)
        n = qw.size
        assert c0.shape == (2, n) and o0.shape == (2, n) and c1.shape == (2, n) and o1.shape == (2, n)
        J = np.empty((3, n2, n1), dtype=np.int64)
        fn = lib().hp_debug_deposit_noalloc if noalloc else lib().hp_debug_deposit
        _check(fn(self.h, run, n, _ptr(c0), _ptr(o0), _ptr(c1), _ptr(o1), _ptr(v3), _ptr(qw),
                  _ptr(J)))
        return J

    def fixed_params(self, run):
        out = np.empty(4)
        _check(lib().hp_get_fixed_params(self.h, run, _ptr(out)))
        return dict(P=int(out[0]), inv_wunit=np.float32(out[1]), c3=np.float32(out[2]),
                    cj=np.float32(out[2]), Q=int(out[3]))

    def profile(self, enable=True):
        _check(lib().hp_profile(self.h, int(bool(enable))))

    def push_stats(self):
        out = np.zeros(2, dtype=np.int64)
        _check(lib().hp_get_push_stats(self.h, _ptr(out)))
        return dict(fallback_tiles=int(out[0]), tiles=int(out[1]))

    def kernel_times(self):
        ms = np.zeros(HP_NK)
        n = np.zeros(HP_NK, dtype=np.int64)
        _check(lib().hp_get_kernel_times(self.h, _ptr(ms), _ptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}


def from_workloads(ds, precision="fp32", alpha=None, deriv1=0, correct=1, background=True,
                   stream=None, **cfg_kw):
    """Handle with one run per ``workloads`` dict of ``ds`` (particles, fields,
    background current and charge), all advanced together."""
    cfgs = []
    for d in ds:
        n1, n2, n3 = d["n"]
        dx1, dx2, dx3 = d["dx"]
        three = d.get("geom", 2) == 3
        cfgs.append(config(n1, n2, dx1, dx2, d["dt"], alpha=d["alpha"] if alpha is None else alpha,
                           deriv1=deriv1, correct=correct, precision=precision,
                           n3=n3 if three else 0, dx3=dx3 if three else 0.0, **cfg_kw))
    sim = Sim(cfgs, stream=stream)
    for r, d in enumerate(ds):
        dim = 3 if d.get("geom", 2) == 3 else 2
        x = np.stack([d["xi"][k] * d["dx"][k] for k in range(dim)])
        sim.set_particles(r, x, d["u"], d["w"], d["qm"], d["q"])
        if np.any(d["E"]) or np.any(d["B"]):
            sim.set_fields(r, d["E"], d["B"])
        if background:
            sim.set_background(r, True, d["jbg"])
        if d.get("antenna"):
            sim.set_antenna(r, **d["antenna"])
    return sim


def from_workload(d, precision="fp32", alpha=None, deriv1=0, correct=1, background=True,
                  stream=None, **cfg_kw):
    """Handle with one run loaded from a ``workloads`` dict."""
    return from_workloads([d], precision, alpha, deriv1, correct, background, stream, **cfg_kw)
