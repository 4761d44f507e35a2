"""FP64 CPU oracle of the hybrid Yee-FFT particle-in-cell step (arXiv:1502.01376).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It wraps the
plain C library ``libhpic_oracle.so`` (built from ``hpic_oracle.c`` by
``oracle/_build.py``) with numpy arrays; it shares no code with the GPU library.

Array conventions follow ``hpic_oracle.h``: field components are ``[3][n2][n1]``
float64 arrays on the Yee-staggered nodes, particle positions are in cell units.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.environ.get("HPIC_ORACLE_LIB", os.path.join(_HERE, "libhpic_oracle.so"))
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


class Grid2(ctypes.Structure):
    """Mirror of ``or_grid2`` (2D grid and solver options)."""

    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("dx1", ctypes.c_double), ("dx2", ctypes.c_double), ("dt", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("deriv1", ctypes.c_int32), ("correct", ctypes.c_int32),
        ("jbg", ctypes.c_double * 3), ("kmod", ctypes.c_int32), ("interp", ctypes.c_int32),
        ("shape", ctypes.c_int32),
    ]


class Grid3(ctypes.Structure):
    """Mirror of ``or_grid3`` (3D grid and solver options)."""

    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
        ("dx1", ctypes.c_double), ("dx2", ctypes.c_double), ("dx3", ctypes.c_double),
        ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
        ("deriv1", ctypes.c_int32), ("correct", ctypes.c_int32),
        ("jbg", ctypes.c_double * 3), ("kmod", ctypes.c_int32), ("interp", ctypes.c_int32),
    ]


class GridQ(ctypes.Structure):
    """Mirror of ``or_gridq`` (quasi-3D r-z grid with azimuthal modes)."""

    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("nmodes", ctypes.c_int32),
        ("dz", ctypes.c_double), ("dr", ctypes.c_double), ("dt", ctypes.c_double),
        ("alpha", ctypes.c_double), ("deriv1", ctypes.c_int32), ("correct", ctypes.c_int32),
        ("kmod", ctypes.c_int32), ("interp", ctypes.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from oracle import _build
            _build.build()
        L = ctypes.CDLL(_LIBPATH)
        G = ctypes.POINTER(Grid2)
        G3 = ctypes.POINTER(Grid3)
        GQ = ctypes.POINTER(GridQ)
        sig = {
            "or_set_threads": (None, [ctypes.c_int32]),
            "or_get_threads": (ctypes.c_int32, []),
            "or_fft": (ctypes.c_int, [ctypes.c_int32, _D, _D, ctypes.c_int32]),
            "or_rfft_rows": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _D, _D, _D]),
            "or_irfft_rows": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _D, _D, _D]),
            "or_gather2": (None, [G, _D, _D, ctypes.c_int64, _D, _D, _D, _D]),
            "or_boris": (None, [ctypes.c_int64, ctypes.c_double, ctypes.c_double, _D, _D, _D, _D, _D]),
            "or_deposit2": (ctypes.c_int, [G, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D]),
            "or_rho2": (None, [G, ctypes.c_int64, _D, _D, _D, _D]),
            "or_field_update2": (ctypes.c_int, [G, _D, _D, _D]),
            "or_yee_update2": (None, [G, _D, _D, _D]),
            "or_step2": (ctypes.c_int, [G, ctypes.c_double, ctypes.c_int64, _D, _D, _D, _D, _D,
                                        _D, _D, _D, _D, ctypes.c_void_p, ctypes.c_double]),
            "or_antenna2": (None, [G, ctypes.c_void_p, ctypes.c_double, _D]),
            "or_gauss2": (ctypes.c_int, [G, _D, _D, _D, _D]),
            "or_deposit2_fixed": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_float, ctypes.c_float, ctypes.c_int64,
                                                 _I32, _I32, _F, _F, _I32, _I32, _F, _F, _F, _F,
                                                 _I64]),
            "or_rho2_fixed": (None, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_int64, _I32, _I32, _F, _F, _F, _I64]),
            "or_gather3": (None, [G3, _D, _D, ctypes.c_int64, _D, _D, _D, _D, _D]),
            "or_deposit3": (ctypes.c_int, [G3, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]),
            "or_rho3": (None, [G3, ctypes.c_int64, _D, _D, _D, _D, _D]),
            "or_field_update3": (ctypes.c_int, [G3, _D, _D, _D]),
            "or_yee_update3": (None, [G3, _D, _D, _D]),
            "or_step3": (ctypes.c_int, [G3, ctypes.c_double, ctypes.c_int64, _D, _D, _D, _D, _D,
                                        _D, _D, _D, _D, _D]),
            "or_gauss3": (ctypes.c_int, [G3, _D, _D, _D, _D]),
            "or_field_update_q": (ctypes.c_int, [GQ, _D, _D, _D]),
            "or_yee_update_q": (ctypes.c_int, [GQ, _D, _D, _D]),
            "or_gauss_q": (ctypes.c_int, [GQ, _D, _D, _D]),
            "or_gather_q": (ctypes.c_int, [GQ, _D, _D, ctypes.c_int64, _D, _D, _D, _D, _D]),
            "or_deposit_q": (ctypes.c_int, [GQ, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]),
            "or_rho_q": (ctypes.c_int, [GQ, ctypes.c_int64, _D, _D, _D, _D, _D]),
            "or_jbg_q": (ctypes.c_int, [GQ, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D]),
            "or_step_q": (ctypes.c_int, [GQ, ctypes.c_double, ctypes.c_int64, _D, _D, _D, _D, _D,
                                         _D, _D, _D, _D, _D, _D]),
            "or_deposit3_fixed": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_float, ctypes.c_float, ctypes.c_int64,
                                                 _I32, _F, _I32, _F, _F, _I64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's OpenMP loops (results do not depend on it)."""
    lib().or_set_threads(int(n))


def threads():
    return int(lib().or_get_threads())


def _p(a, kind=_D):
    return a.ctypes.data_as(kind)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def grid2(n1, n2, dx1, dx2, dt, alpha=1.0, deriv1=0, correct=1, jbg=(0.0, 0.0, 0.0), kmod=0,
          interp=0, shape=2):
    g = Grid2()
    g.kmod = int(kmod)
    g.interp = int(interp)
    g.shape = int(shape)
    g.n1, g.n2 = int(n1), int(n2)
    g.dx1, g.dx2, g.dt = float(dx1), float(dx2), float(dt)
    g.alpha = float(alpha)
    g.deriv1, g.correct = int(deriv1), int(correct)
    for c in range(3):
        g.jbg[c] = float(jbg[c])
    return g


# ---------------------------------------------------------------- transforms
def fft(x, sign=-1):
    """Complex FFT of a power-of-two length vector (no 1/n for sign=+1)."""
    x = np.asarray(x, dtype=np.complex128)
    re, im = np.ascontiguousarray(x.real), np.ascontiguousarray(x.imag)
    if lib().or_fft(len(x), _p(re), _p(im), int(sign)) != 0:
        raise ValueError("length is not a power of two")
    return re + 1j * im


def rfft_rows(f):
    """Forward transform of each row (last axis) of a real array: kappa = 0..n1/2."""
    f = _f64(f)
    n1 = f.shape[-1]
    rows = f.size // n1
    nk = n1 // 2 + 1
    re = np.zeros(rows * nk)
    im = np.zeros(rows * nk)
    if lib().or_rfft_rows(n1, rows, _p(f), _p(re), _p(im)) != 0:
        raise ValueError("bad row length")
    return (re + 1j * im).reshape(f.shape[:-1] + (nk,))


def irfft_rows(F, n1):
    F = np.asarray(F, dtype=np.complex128)
    nk = F.shape[-1]
    rows = F.size // nk
    re, im = _f64(F.real).ravel(), _f64(F.imag).ravel()
    f = np.zeros(rows * n1)
    if lib().or_irfft_rows(int(n1), rows, _p(re), _p(im), _p(f)) != 0:
        raise ValueError("bad row length")
    return f.reshape(F.shape[:-1] + (n1,))


# ----------------------------------------------------------------- particles
def gather2(g, E, B, xi1, xi2):
    E, B, xi1, xi2 = _f64(E), _f64(B), _f64(xi1), _f64(xi2)
    n = len(xi1)
    Ep = np.zeros((3, n))
    Bp = np.zeros((3, n))
    lib().or_gather2(ctypes.byref(g), _p(E), _p(B), n, _p(xi1), _p(xi2), _p(Ep), _p(Bp))
    return Ep, Bp


def boris(qm, dt, Ep, Bp, u):
    """Returns the pushed momenta ([3][np]); the input is not modified."""
    u = _f64(u).copy()
    Ep, Bp = _f64(Ep), _f64(Bp)
    n = u.shape[1]
    u1, u2, u3 = (np.ascontiguousarray(u[c]) for c in range(3))
    lib().or_boris(n, float(qm), float(dt), _p(Ep), _p(Bp), _p(u1), _p(u2), _p(u3))
    return np.stack([u1, u2, u3])


def deposit2(g, xa1, xa2, xb1, xb2, v3, qw):
    xa1, xa2, xb1, xb2, v3, qw = map(_f64, (xa1, xa2, xb1, xb2, v3, qw))
    J = np.zeros((3, g.n2, g.n1))
    st = lib().or_deposit2(ctypes.byref(g), len(xa1), _p(xa1), _p(xa2), _p(xb1), _p(xb2),
                           _p(v3), _p(qw), _p(J))
    if st != 0:
        raise ValueError("a particle moved a cell or more in one step")
    return J


def rho2(g, xi1, xi2, qw):
    xi1, xi2, qw = map(_f64, (xi1, xi2, qw))
    rho = np.zeros((g.n2, g.n1))
    lib().or_rho2(ctypes.byref(g), len(xi1), _p(xi1), _p(xi2), _p(qw), _p(rho))
    return rho


# ---------------------------------------------------------------- field solve
def field_update2(g, E, B, J):
    """Returns (E, B) after one hybrid (or FD-mode) update; inputs not modified."""
    E, B, J = _f64(E).copy(), _f64(B).copy(), _f64(J)
    if lib().or_field_update2(ctypes.byref(g), _p(E), _p(B), _p(J)) != 0:
        raise ValueError("bad grid")
    return E, B


def yee_update2(g, E, B, J):
    E, B, J = _f64(E).copy(), _f64(B).copy(), _f64(J)
    lib().or_yee_update2(ctypes.byref(g), _p(E), _p(B), _p(J))
    return E, B


def gauss2(g, E, rho):
    E, rho = _f64(E), _f64(rho)
    nk = g.n1 // 2 + 1
    re = np.zeros(g.n2 * nk)
    im = np.zeros(g.n2 * nk)
    lib().or_gauss2(ctypes.byref(g), _p(E), _p(rho), _p(re), _p(im))
    return (re + 1j * im).reshape(g.n2, nk)


class Antenna(ctypes.Structure):
    """Moving current-sheet antenna (see ``or_antenna`` in the C header)."""
    _fields_ = [(k, ctypes.c_double) for k in
                ("x0", "v", "t0", "T", "K0", "omega", "phase", "x2c", "waist")]


def antenna(x0, v, t0, T, K0, omega, phase=0.0, x2c=0.0, waist=0.0):
    return Antenna(float(x0), float(v), float(t0), float(T), float(K0), float(omega),
                   float(phase), float(x2c), float(waist))


def antenna2(g, a, t, J=None):
    """The antenna's current j3 at time t added to J ([3][n2][n1], zeros if None)."""
    J = np.zeros((3, g.n2, g.n1)) if J is None else _f64(J).copy()
    lib().or_antenna2(ctypes.byref(g), ctypes.byref(a), float(t), _p(J))
    return J


class State2:
    """Particles and fields of one 2D run, advanced by ``step``; ``t`` is the
    time, ``antenna`` an optional ``Antenna`` whose current is added each step."""

    def __init__(self, g, qm, xi1, xi2, u, qw, E=None, B=None, antenna=None, t=0.0):
        self.antenna, self.t = antenna, float(t)
        self.g, self.qm = g, float(qm)
        self.xi1, self.xi2 = _f64(xi1).copy(), _f64(xi2).copy()
        self.u = _f64(u).copy()
        self.qw = _f64(qw).copy()
        shape = (3, g.n2, g.n1)
        self.E = np.zeros(shape) if E is None else _f64(E).copy()
        self.B = np.zeros(shape) if B is None else _f64(B).copy()
        self.J = np.zeros(shape)

    def step(self, n=1):
        g = self.g
        u1, u2, u3 = (np.ascontiguousarray(self.u[c]) for c in range(3))
        for _ in range(n):
            ant = ctypes.byref(self.antenna) if self.antenna is not None else None
            st = lib().or_step2(ctypes.byref(g), self.qm, len(self.xi1), _p(self.xi1), _p(self.xi2),
                                _p(u1), _p(u2), _p(u3), _p(self.qw), _p(self.E), _p(self.B),
                                _p(self.J), ant, self.t)
            if st != 0:
                raise ValueError("oracle step failed (move of a cell or more)")
            self.t += g.dt
        self.u = np.stack([u1, u2, u3])
        return self


# ------------------------------------------- fixed-point deposit (kernel precision)
def deposit2_fixed(n1, n2, P, inv_wunit, c3, ca1, ca2, fa1, fa2, cb1, cb2, fb1, fb2, v3, qw):
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    ca1, ca2, cb1, cb2 = map(i32, (ca1, ca2, cb1, cb2))
    fa1, fa2, fb1, fb2, v3, qw = map(f32, (fa1, fa2, fb1, fb2, v3, qw))
    J = np.zeros((3, n2, n1), dtype=np.int64)
    st = lib().or_deposit2_fixed(int(n1), int(n2), int(P), float(inv_wunit), float(c3), len(ca1),
                                 _p(ca1, _I32), _p(ca2, _I32), _p(fa1, _F), _p(fa2, _F),
                                 _p(cb1, _I32), _p(cb2, _I32), _p(fb1, _F), _p(fb2, _F),
                                 _p(v3, _F), _p(qw, _F), _p(J, _I64))
    if st != 0:
        raise ValueError("a particle moved a cell or more in one step")
    return J


def rho2_fixed(n1, n2, P, inv_wunit, c1, c2, f1, f2, qw):
    c1 = np.ascontiguousarray(c1, dtype=np.int32)
    c2 = np.ascontiguousarray(c2, dtype=np.int32)
    f1 = np.ascontiguousarray(f1, dtype=np.float32)
    f2 = np.ascontiguousarray(f2, dtype=np.float32)
    qw = np.ascontiguousarray(qw, dtype=np.float32)
    rho = np.zeros((n2, n1), dtype=np.int64)
    lib().or_rho2_fixed(int(n1), int(n2), int(P), float(inv_wunit), len(c1), _p(c1, _I32),
                        _p(c2, _I32), _p(f1, _F), _p(f2, _F), _p(qw, _F), _p(rho, _I64))
    return rho


def courant_limit2(dx1, dx2):
    """Largest stable time step of the hybrid solver, Eq. (22)."""
    return 2.0 / np.sqrt(np.pi ** 2 / dx1 ** 2 + 4.0 / dx2 ** 2)


# ------------------------------------------------------------------------ 3D
def grid3(n1, n2, n3, dx1, dx2, dx3, dt, alpha=1.0, deriv1=0, correct=1, jbg=(0.0, 0.0, 0.0),
          kmod=0, interp=0):
    g = Grid3()
    g.interp = int(interp)
    g.kmod = int(kmod)
    g.n1, g.n2, g.n3 = int(n1), int(n2), int(n3)
    g.dx1, g.dx2, g.dx3, g.dt = float(dx1), float(dx2), float(dx3), float(dt)
    g.alpha = float(alpha)
    g.deriv1, g.correct = int(deriv1), int(correct)
    for c in range(3):
        g.jbg[c] = float(jbg[c])
    return g


def _shape3(g):
    return (3, g.n3, g.n2, g.n1)


def gather3(g, E, B, xi):
    E, B = _f64(E), _f64(B)
    x1, x2, x3 = (_f64(xi[d]) for d in range(3))
    n = len(x1)
    Ep = np.zeros((3, n))
    Bp = np.zeros((3, n))
    lib().or_gather3(ctypes.byref(g), _p(E), _p(B), n, _p(x1), _p(x2), _p(x3), _p(Ep), _p(Bp))
    return Ep, Bp


def deposit3(g, xa, xb, qw):
    """Esirkepov current of moves xa -> xb ([3][np], cell units, xb unwrapped)."""
    a = [_f64(xa[d]) for d in range(3)]
    b = [_f64(xb[d]) for d in range(3)]
    qw = _f64(qw)
    J = np.zeros(_shape3(g))
    st = lib().or_deposit3(ctypes.byref(g), len(qw), _p(a[0]), _p(a[1]), _p(a[2]), _p(b[0]),
                           _p(b[1]), _p(b[2]), _p(qw), _p(J))
    if st != 0:
        raise ValueError("a particle moved a cell or more in one step")
    return J


def rho3(g, xi, qw):
    x = [_f64(xi[d]) for d in range(3)]
    qw = _f64(qw)
    rho = np.zeros(_shape3(g)[1:])
    lib().or_rho3(ctypes.byref(g), len(qw), _p(x[0]), _p(x[1]), _p(x[2]), _p(qw), _p(rho))
    return rho


def field_update3(g, E, B, J):
    E, B, J = _f64(E).copy(), _f64(B).copy(), _f64(J)
    if lib().or_field_update3(ctypes.byref(g), _p(E), _p(B), _p(J)) != 0:
        raise ValueError("bad grid")
    return E, B


def yee_update3(g, E, B, J):
    E, B, J = _f64(E).copy(), _f64(B).copy(), _f64(J)
    lib().or_yee_update3(ctypes.byref(g), _p(E), _p(B), _p(J))
    return E, B


def gauss3(g, E, rho):
    E, rho = _f64(E), _f64(rho)
    nk = g.n1 // 2 + 1
    n = g.n3 * g.n2 * nk
    re, im = np.zeros(n), np.zeros(n)
    lib().or_gauss3(ctypes.byref(g), _p(E), _p(rho), _p(re), _p(im))
    return (re + 1j * im).reshape(g.n3, g.n2, nk)


class State3:
    """Particles and fields of one 3D run, advanced by ``step``."""

    def __init__(self, g, qm, xi, u, qw, E=None, B=None):
        self.g, self.qm = g, float(qm)
        self.xi = [_f64(xi[d]).copy() for d in range(3)]
        self.u = _f64(u).copy()
        self.qw = _f64(qw).copy()
        shape = _shape3(g)
        self.E = np.zeros(shape) if E is None else _f64(E).copy()
        self.B = np.zeros(shape) if B is None else _f64(B).copy()
        self.J = np.zeros(shape)

    def step(self, n=1):
        g = self.g
        u1, u2, u3 = (np.ascontiguousarray(self.u[c]) for c in range(3))
        for _ in range(n):
            st = lib().or_step3(ctypes.byref(g), self.qm, len(self.qw), _p(self.xi[0]),
                                _p(self.xi[1]), _p(self.xi[2]), _p(u1), _p(u2), _p(u3),
                                _p(self.qw), _p(self.E), _p(self.B), _p(self.J))
            if st != 0:
                raise ValueError("oracle step failed (move of a cell or more)")
        self.u = np.stack([u1, u2, u3])
        return self


def deposit3_fixed(n, inv_wunit, cj, ca, fa, cb, fb, qw):
    """Kernel-precision 3D deposit: ca, cb int cell indices [3][np], fa, fb FP32
    offsets [3][np]; returns int64 [3][n3][n2][n1]."""
    ca = np.ascontiguousarray(ca, dtype=np.int32)
    cb = np.ascontiguousarray(cb, dtype=np.int32)
    fa = np.ascontiguousarray(fa, dtype=np.float32)
    fb = np.ascontiguousarray(fb, dtype=np.float32)
    qw = np.ascontiguousarray(qw, dtype=np.float32)
    n1, n2, n3 = (int(v) for v in n)
    J = np.zeros((3, n3, n2, n1), dtype=np.int64)
    st = lib().or_deposit3_fixed(n1, n2, n3, float(inv_wunit), float(cj), len(qw), _p(ca, _I32),
                                 _p(fa, _F), _p(cb, _I32), _p(fb, _F), _p(qw, _F), _p(J, _I64))
    if st != 0:
        raise ValueError("a particle moved a cell or more in one step")
    return J


def courant_limit3(dx1, dx2, dx3):
    """Largest stable time step of the 3D hybrid solver: Eq. (22) with the x3
    difference added, 2 / sqrt(pi^2/dx1^2 + 4/dx2^2 + 4/dx3^2)."""
    return 2.0 / np.sqrt(np.pi ** 2 / dx1 ** 2 + 4.0 / dx2 ** 2 + 4.0 / dx3 ** 2)


# ------------------------------------------------------------------ quasi-3D
def gridq(n1, n2, nmodes, dz, dr, dt, alpha=1.0, deriv1=0, correct=1, kmod=0, interp=0):
    g = GridQ()
    g.n1, g.n2, g.nmodes = int(n1), int(n2), int(nmodes)
    g.dz, g.dr, g.dt = float(dz), float(dr), float(dt)
    g.alpha = float(alpha)
    g.deriv1, g.correct, g.kmod = int(deriv1), int(correct), int(kmod)
    g.interp = int(interp)
    return g


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def field_update_q(g, E, B, J):
    """E, B, J: complex [nmodes][3][n2+1][n1]; returns the updated (E, B)."""
    E, B, J = _c128(E).copy(), _c128(B).copy(), _c128(J)
    if lib().or_field_update_q(ctypes.byref(g), _p(E), _p(B), _p(J)) != 0:
        raise ValueError("bad grid")
    return E, B


def yee_update_q(g, E, B, J):
    E, B, J = _c128(E).copy(), _c128(B).copy(), _c128(J)
    lib().or_yee_update_q(ctypes.byref(g), _p(E), _p(B), _p(J))
    return E, B


def gauss_q(g, E, rho):
    """Gauss residual per mode on the integer nodes: [nmodes][n2+1][n1] complex."""
    E, rho = _c128(E), _c128(rho)
    R = np.zeros((g.nmodes, g.n2 + 1, g.n1), dtype=np.complex128)
    lib().or_gauss_q(ctypes.byref(g), _p(E), _p(rho), _p(R))
    return R


# ------------------------------------------------------- quasi-3D particles
def _shapeq(g):
    return (g.nmodes, 3, g.n2 + 1, g.n1)


def gather_q(g, E, B, pos):
    """Cartesian E, B (order z, x, y) at particles pos = (z, x, y)."""
    E, B = _c128(E), _c128(B)
    z, x, y = (_f64(pos[d]) for d in range(3))
    n = len(z)
    Ep = np.zeros((3, n))
    Bp = np.zeros((3, n))
    st = lib().or_gather_q(ctypes.byref(g), _p(E), _p(B), n, _p(z), _p(x), _p(y), _p(Ep), _p(Bp))
    if st != 0:
        raise ValueError("a particle is outside r < (n2 - 3) dr")
    return Ep, Bp


def deposit_q(g, pa, pb, qw):
    """Per-mode current [nmodes][3][n2+1][n1] of the moves pa -> pb (each
    (z, x, y), z unwrapped) over one step."""
    a = [_f64(pa[d]) for d in range(3)]
    b = [_f64(pb[d]) for d in range(3)]
    qw = _f64(qw)
    J = np.zeros(_shapeq(g), dtype=np.complex128)
    st = lib().or_deposit_q(ctypes.byref(g), len(qw), _p(a[0]), _p(a[1]), _p(a[2]), _p(b[0]),
                            _p(b[1]), _p(b[2]), _p(qw), _p(J))
    if st != 0:
        raise ValueError("a particle moved a cell or more, or is outside r < (n2 - 3) dr")
    return J


def rho_q(g, pos, qw):
    z, x, y = (_f64(pos[d]) for d in range(3))
    qw = _f64(qw)
    rho = np.zeros((g.nmodes, g.n2 + 1, g.n1), dtype=np.complex128)
    if lib().or_rho_q(ctypes.byref(g), len(qw), _p(z), _p(x), _p(y), _p(qw), _p(rho)) != 0:
        raise ValueError("a particle is outside r < (n2 - 3) dr")
    return rho


def jbg_q(g, pos, u, qw):
    """Co-drifting background current profile [n2+1] (m = 0, z component)."""
    x, y = _f64(pos[1]), _f64(pos[2])
    uz, ux, uy = (_f64(u[d]) for d in range(3))
    qw = _f64(qw)
    out = np.zeros(g.n2 + 1)
    if lib().or_jbg_q(ctypes.byref(g), len(qw), _p(x), _p(y), _p(uz), _p(ux), _p(uy), _p(qw),
                      _p(out)) != 0:
        raise ValueError("a particle is outside r < (n2 - 3) dr")
    return out


class StateQ:
    """Particles and per-mode fields of one quasi-3D run, advanced by ``step``."""

    def __init__(self, g, qm, pos, u, qw, E=None, B=None, jbg=None):
        self.g, self.qm = g, float(qm)
        self.pos = [_f64(pos[d]).copy() for d in range(3)]
        self.u = _f64(u).copy()
        self.qw = _f64(qw).copy()
        shape = _shapeq(g)
        self.E = np.zeros(shape, dtype=np.complex128) if E is None else _c128(E).copy()
        self.B = np.zeros(shape, dtype=np.complex128) if B is None else _c128(B).copy()
        self.J = np.zeros(shape, dtype=np.complex128)
        self.jbg = None if jbg is None else _f64(jbg).copy()

    def rho(self):
        return rho_q(self.g, self.pos, self.qw)

    def step(self, n=1):
        g = self.g
        uz, ux, uy = (np.ascontiguousarray(self.u[c]) for c in range(3))
        jb = _p(self.jbg) if self.jbg is not None else None
        for _ in range(n):
            st = lib().or_step_q(ctypes.byref(g), self.qm, len(self.qw), _p(self.pos[0]),
                                 _p(self.pos[1]), _p(self.pos[2]), _p(uz), _p(ux), _p(uy),
                                 _p(self.qw), _p(self.E), _p(self.B), _p(self.J), jb)
            if st != 0:
                raise ValueError("oracle step failed (move of a cell or more, or r too large)")
        self.u = np.stack([uz, ux, uy])
        return self
