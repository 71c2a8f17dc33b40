"""Plain FP64 CPU oracle of the S-TPLS time step (arXiv 1511.07800).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg are the only callers.  The product path never imports this
package.  The arithmetic lives in ``stp_oracle.c`` (plain loops, FP64,
``-O2 -ffp-contract=off``); this module only loads it and moves numpy arrays
in and out.  Arrays are C-contiguous float64 with shape (nz, ny, nx), x
fastest; w has nz+1 planes.
"""
import ctypes
import os
import subprocess

import numpy as np

from .schedule import srj_schedule, kappa_bounds, cycle_factor  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stp_oracle.c")
_LIB = os.path.join(_HERE, "libstp_oracle.so")


def build_oracle(force=False):
    """Compile the C oracle with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("les", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("nu", ctypes.c_double), ("dpdx", ctypes.c_double), ("dt", ctypes.c_double),
                ("cs", ctypes.c_double), ("vd_a", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("poisson_cycles", ctypes.c_int32), ("cn_sweeps", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("relres0", ctypes.c_double), ("relres", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("max_div", ctypes.c_double),
                ("u_bulk", ctypes.c_double), ("u_max", ctypes.c_double),
                ("cfl", ctypes.c_double), ("u_centre", ctypes.c_double),
                ("nut_max", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None


def lib():
    global _lib
    if _lib is None:
        # STP_ORACLE_LIB: another build of the same source (the sanitizer test)
        _lib = ctypes.CDLL(os.environ.get("STP_ORACLE_LIB") or build_oracle())
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        L = _lib
        L.or_lap_p.argtypes = [pp, dp, dp]
        L.or_diag_d.argtypes = [pp]
        L.or_diag_d.restype = ctypes.c_double
        L.or_srj_sweep.argtypes = [pp, ctypes.c_double, dp, dp, dp]
        L.or_srj_sweep_at.argtypes = [pp, ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        L.or_residual.argtypes = [pp, dp, dp, dp]
        L.or_residual.restype = ctypes.c_double
        L.or_poisson_srj.argtypes = [pp, dp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), dp, dp]
        L.or_poisson_srj.restype = ctypes.c_int
        L.or_divergence.argtypes = [pp, dp, dp, dp, dp]
        L.or_project.argtypes = [pp, dp, dp, dp, dp]
        L.or_nut.argtypes = [pp, dp, dp, dp, dp]
        L.or_nut.restype = ctypes.c_double
        L.or_visc_diff.argtypes = [pp, ctypes.c_int, dp, dp, dp]
        L.or_explicit.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        L.or_cn_solve.argtypes = [pp, ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.or_cn_solve.restype = ctypes.c_int
        L.or_diagnostics.argtypes = [pp, dp, dp, dp, ctypes.POINTER(Stats)]
        L.or_step.argtypes = [pp, dp, dp, dp, dp, ctypes.POINTER(dp), ctypes.c_int, dp, ctypes.c_int,
                              ctypes.c_double, ctypes.c_int, dp, dp, ctypes.POINTER(Stats)]
        L.or_step.restype = ctypes.c_int
        L.or_srj_cycle.argtypes = [pp, dp, ctypes.c_int, dp, dp]
        L.or_plane_stats.argtypes = [pp, dp, dp, dp, dp, dp]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = ctypes.c_int
    return _lib


def set_threads(n):
    """Threads of the oracle's plane loops (n <= 0: unchanged); returns the count in effect."""
    return lib().or_set_threads(int(n))


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, nz, lx, ly, lz, nu=1.0, dpdx=0.0, dt=1.0, les=0, cs=0.1, vd_a=25.0):
    return Params(nx, ny, nz, les, lx, ly, lz, nu, dpdx, dt, cs, vd_a)


def cell_shape(P):
    return (P.nz, P.ny, P.nx)


def wface_shape(P):
    return (P.nz + 1, P.ny, P.nx)


def lap_p(P, p):
    out = np.empty(cell_shape(P))
    lib().or_lap_p(ctypes.byref(P), _p(np.ascontiguousarray(p, np.float64)), _p(out))
    return out


def diag_d(P):
    return lib().or_diag_d(ctypes.byref(P))


def srj_sweep(P, omega, p, b):
    out = np.empty(cell_shape(P))
    lib().or_srj_sweep(ctypes.byref(P), float(omega), _p(np.ascontiguousarray(p, np.float64)),
                       _p(np.ascontiguousarray(b, np.float64)), _p(out))
    return out


def srj_cycle(P, omega, p, b):
    """The sweeps omega applied to p in order (a new array; no residual test)."""
    out = np.array(p, dtype=np.float64, order="C", copy=True)
    om = np.ascontiguousarray(omega, np.float64)
    lib().or_srj_cycle(ctypes.byref(P), _p(om), len(om), _p(out), _p(np.ascontiguousarray(b, np.float64)))
    return out


def srj_sweep_at(P, omega, p, b, cells):
    """Sweep values at the flat cell indices `cells` only."""
    cells = np.ascontiguousarray(cells, np.int64)
    out = np.empty(len(cells))
    lib().or_srj_sweep_at(ctypes.byref(P), float(omega), _p(np.ascontiguousarray(p, np.float64)),
                          _p(np.ascontiguousarray(b, np.float64)),
                          cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(cells), _p(out))
    return out


def residual(P, p, b):
    r = np.empty(cell_shape(P))
    s = lib().or_residual(ctypes.byref(P), _p(np.ascontiguousarray(p, np.float64)),
                          _p(np.ascontiguousarray(b, np.float64)), _p(r))
    return r, s


def poisson_srj(P, b, p0, omega, rtol, maxit):
    """SRJ solve; returns (p, status, cycles, relres0, relres)."""
    p = np.array(p0, dtype=np.float64, order="C", copy=True)
    om = np.ascontiguousarray(omega, np.float64)
    cyc = ctypes.c_int(0)
    r0 = ctypes.c_double(0)
    r1 = ctypes.c_double(0)
    st = lib().or_poisson_srj(ctypes.byref(P), _p(np.ascontiguousarray(b, np.float64)), _p(p), _p(om),
                              len(om), float(rtol), int(maxit), ctypes.byref(cyc), ctypes.byref(r0),
                              ctypes.byref(r1))
    return p, st, cyc.value, r0.value, r1.value


def poisson_srj_adaptive(P, b, p0, rtol, maxit, floor=1e-10):
    """SRJ solve whose every cycle is sized from the reduction still needed
    (schedule.adaptive_degree); returns (p, status, cycles, sweeps, relres0, relres)."""
    from .schedule import kappa_bounds as kb, adaptive_degree, schedule_of_degree
    a, bb = kb(P.nx, P.ny, P.nz, P.lx, P.ly, P.lz)
    p = np.array(p0, dtype=np.float64, order="C", copy=True)
    bn = float(np.sqrt(np.sum(b * b)))
    fb = bn if bn > 1e-300 else 1e-300
    rn = float(np.sqrt(residual(P, p, b)[1]))
    relres0 = rn / fb
    cycles = sweeps = 0
    status = 0
    while not (rn <= rtol * fb):
        if not np.isfinite(rn):
            status = -5
            break
        if cycles >= maxit:
            status = -4
            break
        om = schedule_of_degree(a, bb, adaptive_degree(a, bb, rtol, fb, rn, floor))
        p, _, _, _, _ = poisson_srj(P, b, p, om, 0.0, 1)
        cycles += 1
        sweeps += len(om)
        rn = float(np.sqrt(residual(P, p, b)[1]))
    p -= p.mean()
    return p, status, cycles, sweeps, relres0, rn / fb


def divergence(P, u, v, w):
    out = np.empty(cell_shape(P))
    lib().or_divergence(ctypes.byref(P), _p(u), _p(v), _p(w), _p(out))
    return out


def project(P, p, u, v, w):
    u, v, w = u.copy(), v.copy(), w.copy()
    lib().or_project(ctypes.byref(P), _p(p), _p(u), _p(v), _p(w))
    return u, v, w


def nut(P, u, v, w):
    out = np.empty(cell_shape(P))
    mx = lib().or_nut(ctypes.byref(P), _p(u), _p(v), _p(w), _p(out))
    return out, mx


def visc_diff(P, comp, nut_, f):
    out = np.empty_like(f)
    lib().or_visc_diff(ctypes.byref(P), int(comp), _p(nut_), _p(np.ascontiguousarray(f)), _p(out))
    return out


def explicit(P, u, v, w, nut_):
    eu = np.empty(cell_shape(P))
    ev = np.empty(cell_shape(P))
    ew = np.empty(wface_shape(P))
    lib().or_explicit(ctypes.byref(P), _p(u), _p(v), _p(w), _p(nut_), _p(eu), _p(ev), _p(ew))
    return eu, ev, ew


def cn_solve(P, comp, nut_, nut_max, R):
    x = np.empty_like(R)
    s = lib().or_cn_solve(ctypes.byref(P), int(comp), _p(nut_), float(nut_max), _p(R), _p(x))
    return x, s


def diagnostics(P, u, v, w):
    st = Stats()
    lib().or_diagnostics(ctypes.byref(P), _p(u), _p(v), _p(w), ctypes.byref(st))
    return st.as_dict()


PLANE_STATS = ("u", "v", "uu", "vv", "nut", "w", "ww", "uw")


def plane_stats(P, u, v, w, nut_):
    """x-y means at every height (or_plane_stats): dict of u, v, uu, vv, nut
    (nz cell planes) and w, ww, uw (nz + 1 face planes)."""
    out = np.zeros(8 * (P.nz + 1))
    lib().or_plane_stats(ctypes.byref(P), _p(np.ascontiguousarray(u, np.float64)),
                         _p(np.ascontiguousarray(v, np.float64)), _p(np.ascontiguousarray(w, np.float64)),
                         _p(np.ascontiguousarray(nut_, np.float64)), _p(out))
    out = out.reshape(8, P.nz + 1)
    return {name: (out[q, :P.nz].copy() if q < 5 else out[q].copy()) for q, name in enumerate(PLANE_STATS)}


class Solver:
    """Multi-step driver over ``or_step``: state {u, v, w, p, E^{n-1}, E^{n-2}, n}."""

    def __init__(self, P, u, v, w, p=None, omega=None, rtol=1e-10, maxit=1000, reduction=1e-3,
                 warm_start="prev"):
        self.P = P
        self.u = np.array(u, np.float64, order="C", copy=True)
        self.v = np.array(v, np.float64, order="C", copy=True)
        self.w = np.array(w, np.float64, order="C", copy=True)
        self.p = np.zeros(cell_shape(P)) if p is None else np.array(p, np.float64, order="C", copy=True)
        self.omega = (srj_schedule(P.nx, P.ny, P.nz, P.lx, P.ly, P.lz, reduction)
                      if omega is None else np.ascontiguousarray(omega, np.float64))
        self.rtol, self.maxit = rtol, maxit
        self.warm_start = warm_start
        self.hist = [np.zeros(cell_shape(P)), np.zeros(cell_shape(P)), np.zeros(wface_shape(P)),
                     np.zeros(cell_shape(P)), np.zeros(cell_shape(P)), np.zeros(wface_shape(P))]
        self.nut = np.zeros(cell_shape(P))
        self.b = np.zeros(cell_shape(P))
        self.n = 0

    def step(self):
        st = Stats()
        if self.warm_start == "zero":
            self.p[...] = 0.0
        harr = (ctypes.POINTER(ctypes.c_double) * 6)(*[_p(h) for h in self.hist])
        lib().or_step(ctypes.byref(self.P), _p(self.u), _p(self.v), _p(self.w), _p(self.p), harr, self.n,
                      _p(self.omega), len(self.omega), float(self.rtol), int(self.maxit), _p(self.nut),
                      _p(self.b), ctypes.byref(st))
        self.n += 1
        return st.as_dict()
