"""ctypes wrapper around the plain FP64 CPU oracle (``wd_oracle.c``).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It never
imports the GPU package, and the GPU package never imports it.

Arrays are numpy float64, dense, x index fastest; 2D grids use shape
``(n1, n0)`` and 3D grids ``(n2, n1, n0)``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwdoracle.so")

WALL, NEUMANN, OUTFLOW, PERIODIC = 0, 1, 2, 3
EIKONAL, HJ, POISSON = 0, 1, 2
GAMMA_LINEAR, GAMMA_LAD = 0, 1
E2, E4, E6, C4, C6, UW = 0, 1, 2, 3, 4, 5
RK3, RK4 = 0, 1
SCHEMES = {"E2": E2, "E4": E4, "E6": E6, "C4": C4, "C6": C6, "UW": UW}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math; OpenMP shares
    the independent line and point loops among threads)."""
    src = os.path.join(HERE, "wd_oracle.c")
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3),
                ("bc", (C.c_int * 2) * 3), ("uniform", C.c_int),
                ("h", C.c_double * 3), ("coords", C.POINTER(C.c_double)),
                ("period", (C.c_double * 3) * 3),
                ("mask", C.POINTER(C.c_ubyte)), ("metric_form", C.c_int)]


class _Method(C.Structure):
    _fields_ = [("equation", C.c_int), ("gamma", C.c_int),
                ("curvature", C.c_int), ("eps", C.c_double),
                ("C", C.c_double), ("nu0", C.c_double), ("eps0", C.c_double),
                ("scheme", C.c_int), ("filter", C.c_int),
                ("alpha_f", C.c_double), ("rk", C.c_int),
                ("sigma", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("lad_raw", C.c_int),
                ("uw_printed", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.wdo_deriv_line.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, dp, dp]
        L.wdo_filter_line.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
        L.wdo_metrics.argtypes = [C.POINTER(_Grid), C.c_int, dp]
        L.wdo_eval.argtypes = [C.POINTER(_Grid), C.POINTER(_Method), dp, dp,
                               dp, dp, dp, dp, dp, dp, dp]
        L.wdo_lad_field.argtypes = [C.POINTER(_Grid), C.POINTER(_Method), dp, dp, dp]
        L.wdo_gauss_line.argtypes = [C.c_int, C.c_int, dp, dp]
        L.wdo_set_threads.argtypes = [C.c_int]
        L.wdo_apply_bc.argtypes = [C.POINTER(_Grid), dp]
        L.wdo_apply_bc.restype = None
        L.wdo_solve.argtypes = [C.POINTER(_Grid), C.POINTER(_Method), dp,
                                C.c_int, dp, C.c_int, C.POINTER(C.c_int)]
        L.wdo_poisson_distance.argtypes = [C.POINTER(_Grid), C.c_int, dp, dp, dp]
        L.wdo_brute_force.argtypes = [C.c_int, C.c_int, dp, C.c_int, dp, dp]
        L.wdo_brute_force.restype = None
        L.wdo_signed_distance.argtypes = [C.c_long, C.POINTER(C.c_ubyte), dp, dp, dp]
        L.wdo_signed_distance.restype = None
        L.wdo_levelset_advance.argtypes = [C.POINTER(_Grid), C.c_double, C.c_double, C.c_int, dp]
        L.wdo_level_length.argtypes = [C.POINTER(_Grid), dp, C.c_double]
        L.wdo_level_length.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleGrid:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, spec):
        self.spec = spec
        g = _Grid()
        g.ndim = spec.ndim
        for i in range(3):
            g.n[i] = spec.n[i] if i < spec.ndim else 1
            for s in range(2):
                g.bc[i][s] = spec.bc[i][s] if i < spec.ndim else WALL
            g.h[i] = spec.h[i] if spec.h is not None and i < spec.ndim else 0.0
            for m in range(3):
                g.period[i][m] = 0.0
        if spec.period is not None:
            for l in range(spec.ndim):
                for m in range(spec.ndim):
                    g.period[l][m] = float(spec.period[l][m])
        g.uniform = 1 if spec.coords is None else 0
        g.metric_form = int(getattr(spec, "metric_form", 0))
        self._coords = None
        if spec.coords is not None:
            self._coords = np.ascontiguousarray(spec.coords, dtype=np.float64)
            g.coords = _ptr(self._coords)
        self._mask = None
        if spec.mask is not None:
            self._mask = np.ascontiguousarray(spec.mask, dtype=np.uint8)
            g.mask = self._mask.ctypes.data_as(C.POINTER(C.c_ubyte))
        self.g = g

    @property
    def shape(self):
        return tuple(reversed(self.spec.n[: self.spec.ndim]))


def make_method(equation=HJ, gamma=GAMMA_LINEAR, curvature=0, eps=0.1, C_lad=0.1,
                nu0=1e-3, eps0=1e-6, scheme=E4, filter=1, alpha_f=0.495,
                rk=RK4, sigma=1.0, tol=1e-10, max_iter=100000, fixed_iters=0, lad_raw=0,
                uw_printed=0):
    m = _Method()
    m.equation, m.gamma, m.curvature = equation, gamma, curvature
    m.eps, m.C, m.nu0, m.eps0 = eps, C_lad, nu0, eps0
    m.scheme = SCHEMES[scheme] if isinstance(scheme, str) else scheme
    m.filter, m.alpha_f, m.rk = filter, alpha_f, rk
    m.sigma, m.tol, m.max_iter, m.fixed_iters = sigma, tol, max_iter, fixed_iters
    m.lad_raw = lad_raw
    m.uw_printed = uw_printed
    return m


def deriv_line(f, scheme, periodic=False, jump=0.0):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    s = SCHEMES[scheme] if isinstance(scheme, str) else scheme
    rc = lib().wdo_deriv_line(f.size, int(periodic), s, jump, _ptr(f), _ptr(out))
    if rc:
        raise ValueError("wdo_deriv_line failed")
    return out


def filter_line(f, alpha_f, periodic=False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    rc = lib().wdo_filter_line(f.size, int(periodic), alpha_f, _ptr(f), _ptr(out))
    if rc:
        raise ValueError("wdo_filter_line failed")
    return out


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's grid-wide loops (0: keep); the count in force."""
    return int(lib().wdo_set_threads(int(n)))


def gauss_line(f, periodic=False):
    """The nine-point smoothing of the LAD diffusivity along one line."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    if lib().wdo_gauss_line(f.size, int(periodic), _ptr(f), _ptr(out)):
        raise ValueError("wdo_gauss_line failed")
    return out


def metrics(spec, scheme):
    og = OracleGrid(spec)
    d = spec.ndim
    met = np.empty((d * d,) + og.shape, dtype=np.float64)
    s = SCHEMES[scheme] if isinstance(scheme, str) else scheme
    rc = lib().wdo_metrics(C.byref(og.g), s, _ptr(met))
    if rc:
        raise ValueError("wdo_metrics failed")
    return met


def evaluate(spec, method, phi, met=None):
    """Return dict with R, g, gamma, lap, kappa, dt at phi."""
    og = OracleGrid(spec)
    if met is None:
        met = metrics(spec, method.scheme)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    outs = {k: np.empty(og.shape) for k in ("R", "g", "gamma", "lap", "kappa", "dt")}
    rc = lib().wdo_eval(C.byref(og.g), C.byref(method), _ptr(met), _ptr(phi), None,
                        *(_ptr(outs[k]) for k in ("R", "g", "gamma", "lap", "kappa", "dt")))
    if rc:
        raise ValueError("wdo_eval failed")
    return outs


def lad_field(spec, method, phi, met=None):
    og = OracleGrid(spec)
    if met is None:
        met = metrics(spec, method.scheme)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.empty(og.shape)
    lib().wdo_lad_field(C.byref(og.g), C.byref(method), _ptr(met), _ptr(phi), _ptr(out))
    return out


def apply_bc(spec, phi):
    og = OracleGrid(spec)
    phi = np.array(phi, dtype=np.float64, copy=True)
    lib().wdo_apply_bc(C.byref(og.g), _ptr(phi))
    return phi


def solve(spec, method, phi0=None, hist_cap=None):
    """Run the oracle.  Returns (phi, status, iters, hist[iters, 2])."""
    og = OracleGrid(spec)
    warm = phi0 is not None
    phi = np.zeros(og.shape) if phi0 is None else \
        np.array(phi0, dtype=np.float64, copy=True)
    if hist_cap is None:
        hist_cap = method.fixed_iters if method.fixed_iters > 0 else method.max_iter
    hist = np.zeros((max(hist_cap, 1), 2))
    iters = C.c_int(0)
    status = lib().wdo_solve(C.byref(og.g), C.byref(method), _ptr(phi), int(warm),
                             _ptr(hist), hist_cap, C.byref(iters))
    n = iters.value
    return phi, status, n, hist[: min(n, hist_cap)].copy()


def poisson_distance(spec, scheme, phip, met=None):
    og = OracleGrid(spec)
    if met is None:
        met = metrics(spec, scheme)
    phip = np.ascontiguousarray(phip, dtype=np.float64)
    d = np.empty(og.shape)
    s = SCHEMES[scheme] if isinstance(scheme, str) else scheme
    rc = lib().wdo_poisson_distance(C.byref(og.g), s, _ptr(met), _ptr(phip), _ptr(d))
    if rc:
        raise ValueError("wdo_poisson_distance failed")
    return d


def brute_force(points, wall):
    points = np.ascontiguousarray(points, dtype=np.float64)
    wall = np.ascontiguousarray(wall, dtype=np.float64)
    ndim = points.shape[1]
    out = np.empty(points.shape[0])
    lib().wdo_brute_force(ndim, points.shape[0], _ptr(points), wall.shape[0],
                          _ptr(wall), _ptr(out))
    return out


def signed_distance(solid, d_solid, d_gas):
    """Sec. 5.5: phi_s = d_solid on solid points, -d_gas elsewhere."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    d_solid = np.ascontiguousarray(d_solid, dtype=np.float64)
    d_gas = np.ascontiguousarray(d_gas, dtype=np.float64)
    out = np.empty_like(d_solid)
    lib().wdo_signed_distance(out.size, solid.ctypes.data_as(C.POINTER(C.c_ubyte)),
                              _ptr(d_solid), _ptr(d_gas), _ptr(out))
    return out


def levelset_advance(spec, phi, speed, dt, nsteps):
    """Eq. levelset (right-hand side read as 0), RK4, zero-gradient faces."""
    og = OracleGrid(spec)
    phi = np.array(phi, dtype=np.float64, copy=True)
    rc = lib().wdo_levelset_advance(C.byref(og.g), speed, dt, nsteps, _ptr(phi))
    if rc:
        raise ValueError("wdo_levelset_advance failed")
    return phi


def level_length(spec, phi, level):
    """Length of the 2D iso-line phi = level (marching squares)."""
    og = OracleGrid(spec)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    v = lib().wdo_level_length(C.byref(og.g), _ptr(phi), level)
    if v < 0:
        raise ValueError("wdo_level_length needs a uniform 2D grid")
    return v
