"""ctypes binding of libwd.so (include/wd.h), argument marshalling only.

Every function here has the name of the C entry point it wraps.  Device
memory and streams come from PyTorch (``torch.Tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``); all computation happens in the
library's HIP kernels.  Importing this module fails loudly when the built
library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwd.so")

WD_OK, WD_NOT_CONVERGED, WD_STAGNATED, WD_PENDING = 0, 1, 2, 3
WD_ERR_INVALID_ARG, WD_ERR_UNSUPPORTED, WD_ERR_DIVERGED = -1, -2, -3
WD_ERR_NO_MEMORY, WD_ERR_HIP, WD_ERR_CANCELLED, WD_ERR_NOT_FOUND = -4, -5, -6, -7
WD_ERR_WARM_RUNAWAY = -8

WD_BC_WALL, WD_BC_NEUMANN, WD_BC_OUTFLOW, WD_BC_PERIODIC = 0, 1, 2, 3
WD_METRIC_UNIFORM, WD_METRIC_FIELDS = 0, 1
WD_EQ_EIKONAL, WD_EQ_HJ, WD_EQ_POISSON = 0, 1, 2
WD_GAMMA_LINEAR, WD_GAMMA_LAD = 0, 1
WD_E2, WD_E4, WD_E6, WD_C4, WD_C6, WD_UW = 0, 1, 2, 3, 4, 5
WD_RK3_SSP, WD_RK4 = 0, 1
WD_FP32, WD_FP64 = 0, 1

SCHEMES = {"E2": WD_E2, "E4": WD_E4, "E6": WD_E6, "C4": WD_C4, "C6": WD_C6, "UW": WD_UW}


class wd_grid_desc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("bc", (C.c_int * 2) * 3),
                ("metric_mode", C.c_int), ("h", C.c_double * 3),
                ("metrics", C.c_void_p), ("mask", C.c_void_p)]


class wd_method(C.Structure):
    _fields_ = [("equation", C.c_int), ("gamma", C.c_int), ("curvature", C.c_int),
                ("eps", C.c_double), ("c_lad", C.c_double), ("nu0", C.c_double),
                ("eps0", C.c_double), ("scheme", C.c_int), ("filter", C.c_int),
                ("alpha_f", C.c_double), ("rk", C.c_int), ("sigma", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_int), ("stall_window", C.c_int),
                ("precision", C.c_int), ("warm_start", C.c_int), ("warm_probe", C.c_int)]


class wd_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_longlong), ("total_ms", C.c_double),
                ("alg_bytes", C.c_double)]


class WDError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where} failed with {code}: {wd_last_error()}")


_lib = None


def lib():
    """Load libwd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or paper_2111_09859_amd/csrc/build.py")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    szp = C.POINTER(C.c_size_t)
    gd, me = C.POINTER(wd_grid_desc), C.POINTER(wd_method)
    sig = {
        "wd_version": ([], C.c_char_p),
        "wd_last_error": ([], C.c_char_p),
        "wd_method_default": ([me], C.c_int),
        "wd_ctx_create": ([C.c_int, C.POINTER(vp)], C.c_int),
        "wd_ctx_destroy": ([vp], C.c_int),
        "wd_compute_metrics": ([vp, gd, C.c_int, vp, dp, vp, C.c_int, vp], C.c_int),
        "wd_compute_metrics_form": ([vp, gd, C.c_int, C.c_int, vp, dp, vp, C.c_int, vp], C.c_int),
        "wd_workspace_bytes": ([vp, C.c_int, gd, me, szp], C.c_int),
        "wd_solve": ([vp, gd, me, vp, vp, dp, C.c_int, ip, vp, C.c_size_t, vp], C.c_int),
        "wd_solve_batched": ([vp, C.c_int, gd, me, C.POINTER(vp), C.POINTER(vp),
                              C.POINTER(dp), C.c_int, ip, ip, vp, C.c_size_t, vp], C.c_int),
        "wd_poisson_distance": ([vp, gd, C.c_int, C.c_int, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "wd_autotune": ([vp, gd, me, vp, vp, C.c_size_t, C.c_int, ip, vp], C.c_int),
        "wd_levelset_workspace_bytes": ([vp, gd, C.c_int, szp], C.c_int),
        "wd_signed_distance": ([vp, C.c_longlong, C.c_int, vp, vp, vp, vp, vp], C.c_int),
        "wd_levelset_advance": ([vp, gd, C.c_int, C.c_double, C.c_double, C.c_int, vp, vp,
                                 C.c_size_t, vp], C.c_int),
        "wd_level_lengths": ([vp, gd, C.c_int, vp, dp, C.c_int, dp, vp, C.c_size_t, vp],
                             C.c_int),
        "wd_tune_get": ([vp, gd, C.c_int, ip], C.c_int),
        "wd_tune_set": ([vp, gd, C.c_int, ip], C.c_int),
        "wd_ctx_profile": ([vp, C.c_int], C.c_int),
        "wd_ctx_profile_read": ([vp, C.POINTER(wd_kernel_stat), C.c_int, ip], C.c_int),
        "wd_ctx_set_segmented": ([vp, C.c_int], C.c_int),
        "wd_ctx_set_explicit_onepass": ([vp, C.c_int], C.c_int),
        "wd_ctx_set_lad_tiles": ([vp, C.c_int], C.c_int),
        "wd_solve_noalloc": ([vp, C.POINTER(wd_grid_desc), C.POINTER(wd_method), vp, vp, dp,
                              C.c_int, ip, vp], C.c_int),
        "wd_seg_solve_host": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                               dp, dp, ip], C.c_int),
        "wd_line_solve_host": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, dp,
                                dp, ip], C.c_int),
        "wd_server_create": ([vp, C.c_size_t, C.c_int, C.POINTER(vp)], C.c_int),
        "wd_server_submit": ([vp, gd, me, vp, C.c_longlong, C.c_int,
                              C.POINTER(C.c_longlong)], C.c_int),
        "wd_server_poll": ([vp, C.c_longlong, ip, dp, dp, dp, ip], C.c_int),
        "wd_server_wait": ([vp, C.c_longlong, C.c_double], C.c_int),
        "wd_server_history": ([vp, C.c_longlong, dp, C.c_int, ip], C.c_int),
        "wd_server_cancel": ([vp, C.c_longlong], C.c_int),
        "wd_server_stats": ([vp, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong), szp, ip,
                             C.POINTER(C.c_longlong)],
                            C.c_int),
        "wd_server_destroy": ([vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc, where, ok=(WD_OK, WD_NOT_CONVERGED, WD_STAGNATED)):
    if rc not in ok:
        raise WDError(rc, where)
    return rc


# ---- thin wrappers with the C names ----------------------------------
def wd_version() -> str:
    return lib().wd_version().decode()


def wd_last_error() -> str:
    return lib().wd_last_error().decode() if _lib is not None else ""


def wd_method_default() -> wd_method:
    m = wd_method()
    _check(lib().wd_method_default(C.byref(m)), "wd_method_default")
    return m


def wd_ctx_create(device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().wd_ctx_create(device, C.byref(h)), "wd_ctx_create")
    return h


def wd_ctx_destroy(ctx) -> None:
    lib().wd_ctx_destroy(ctx)


WD_METRICS_INVERSE, WD_METRICS_CONSERVATIVE = 0, 1


def _period_arg(period):
    if period is None:
        return None
    arr = (C.c_double * 9)(*[float(period[l][m]) if l < len(period) and m < len(period[l])
                              else 0.0 for l in range(3) for m in range(3)])
    return C.cast(arr, C.POINTER(C.c_double))


def wd_compute_metrics(ctx, desc, scheme, coords_ptr, period, out_ptr, out_precision,
                       stream=None):
    return _check(lib().wd_compute_metrics(ctx, C.byref(desc), scheme, coords_ptr,
                                           _period_arg(period), out_ptr, out_precision, stream),
                  "wd_compute_metrics")


def wd_compute_metrics_form(ctx, desc, scheme, form, coords_ptr, period, out_ptr, out_precision,
                            stream=None):
    return _check(lib().wd_compute_metrics_form(ctx, C.byref(desc), scheme, form, coords_ptr,
                                                _period_arg(period), out_ptr, out_precision,
                                                stream),
                  "wd_compute_metrics_form")


def wd_workspace_bytes(ctx, descs, methods) -> int:
    n = len(descs)
    DA = (wd_grid_desc * n)(*descs)
    MA = (wd_method * n)(*methods)
    out = C.c_size_t()
    _check(lib().wd_workspace_bytes(ctx, n, DA, MA, C.byref(out)), "wd_workspace_bytes")
    return out.value


def wd_solve(ctx, desc, method, phi_ptr, aux_ptr, hist, hist_cap, ws_ptr, ws_bytes,
             stream=None, check=True):
    """hist: ctypes double array of 2*hist_cap (or None). Returns (rc, iters)."""
    it = C.c_int(0)
    hp = C.cast(hist, C.POINTER(C.c_double)) if hist is not None else None
    rc = lib().wd_solve(ctx, C.byref(desc), C.byref(method), phi_ptr, aux_ptr, hp, hist_cap,
                        C.byref(it), ws_ptr, ws_bytes, stream)
    if check:
        _check(rc, "wd_solve")
    return rc, it.value


def wd_solve_noalloc(ctx, desc, method, phi_ptr, aux_ptr, hist, hist_cap, stream=None,
                     check=True):
    """wd_solve without any device allocation (the library's static scratch
    holds workspace and tables).  Returns (rc, iters)."""
    it = C.c_int(0)
    hp = C.cast(hist, C.POINTER(C.c_double)) if hist is not None else None
    rc = lib().wd_solve_noalloc(ctx, C.byref(desc), C.byref(method), phi_ptr, aux_ptr, hp,
                                hist_cap, C.byref(it), stream)
    if check:
        _check(rc, "wd_solve_noalloc")
    return rc, it.value


def wd_solve_batched(ctx, descs, methods, phi_ptrs, aux_ptrs, hists, hist_cap, ws_ptr,
                     ws_bytes, stream=None, check=True):
    n = len(descs)
    DA = (wd_grid_desc * n)(*descs)
    MA = (wd_method * n)(*methods)
    PA = (C.c_void_p * n)(*phi_ptrs)
    AA = (C.c_void_p * n)(*(aux_ptrs or [None] * n))
    HA = (C.POINTER(C.c_double) * n)(*[C.cast(h, C.POINTER(C.c_double)) if h is not None
                                         else None for h in (hists or [None] * n)])
    iters = (C.c_int * n)()
    status = (C.c_int * n)()
    rc = lib().wd_solve_batched(ctx, n, DA, MA, PA, AA, HA, hist_cap, iters, status, ws_ptr,
                                ws_bytes, stream)
    if check:
        _check(rc, "wd_solve_batched")
    return rc, list(iters), list(status)


def wd_poisson_distance(ctx, desc, scheme, precision, phip_ptr, dist_ptr, ws_ptr, ws_bytes,
                        stream=None):
    return _check(lib().wd_poisson_distance(ctx, C.byref(desc), scheme, precision, phip_ptr,
                                            dist_ptr, ws_ptr, ws_bytes, stream),
                  "wd_poisson_distance")


def wd_levelset_workspace_bytes(ctx, desc, precision):
    b = C.c_size_t(0)
    _check(lib().wd_levelset_workspace_bytes(ctx, C.byref(desc), precision, C.byref(b)),
           "wd_levelset_workspace_bytes")
    return b.value


def wd_signed_distance(ctx, n, precision, solid_ptr, d_solid_ptr, d_gas_ptr, out_ptr,
                       stream=None):
    return _check(lib().wd_signed_distance(ctx, n, precision, solid_ptr, d_solid_ptr,
                                           d_gas_ptr, out_ptr, stream), "wd_signed_distance")


def wd_levelset_advance(ctx, desc, precision, speed, dt, nsteps, phi_ptr, ws_ptr, ws_bytes,
                        stream=None):
    return _check(lib().wd_levelset_advance(ctx, C.byref(desc), precision, speed, dt, nsteps,
                                            phi_ptr, ws_ptr, ws_bytes, stream),
                  "wd_levelset_advance")


def wd_level_lengths(ctx, desc, precision, phi_ptr, levels, ws_ptr, ws_bytes, stream=None):
    n = len(levels)
    lv = (C.c_double * max(n, 1))(*[float(v) for v in levels])
    out = (C.c_double * max(n, 1))()
    _check(lib().wd_level_lengths(ctx, C.byref(desc), precision, phi_ptr, lv, n, out, ws_ptr,
                                  ws_bytes, stream), "wd_level_lengths")
    return [out[k] for k in range(n)]


def wd_autotune(ctx, desc, method, phi_ptr, ws_ptr, ws_bytes, iters=20, stream=None):
    w = (C.c_int * 3)()
    _check(lib().wd_autotune(ctx, C.byref(desc), C.byref(method), phi_ptr, ws_ptr, ws_bytes,
                             iters, w, stream), "wd_autotune", ok=(WD_OK,))
    return list(w)[: desc.ndim]


def wd_tune_get(ctx, desc, precision):
    w = (C.c_int * 3)()
    _check(lib().wd_tune_get(ctx, C.byref(desc), precision, w), "wd_tune_get", ok=(WD_OK,))
    return list(w)[: desc.ndim]


def wd_tune_set(ctx, desc, precision, widths):
    w = (C.c_int * 3)(*(list(widths) + [1] * (3 - len(widths))))
    _check(lib().wd_tune_set(ctx, C.byref(desc), precision, w), "wd_tune_set", ok=(WD_OK,))


def wd_ctx_profile(ctx, enable: bool) -> None:
    _check(lib().wd_ctx_profile(ctx, int(bool(enable))), "wd_ctx_profile", ok=(WD_OK,))


def wd_ctx_profile_read(ctx):
    arr = (wd_kernel_stat * 64)()
    n = C.c_int(0)
    _check(lib().wd_ctx_profile_read(ctx, arr, 64, C.byref(n)), "wd_ctx_profile_read", ok=(WD_OK,))
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches,
             "total_ms": arr[i].total_ms, "alg_bytes": arr[i].alg_bytes}
            for i in range(min(n.value, 64))]


def wd_line_solve_host(kind, rhs, periodic, scheme="C6", alpha_f=0.495, fp64=True):
    import numpy as np
    r = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.empty_like(r)
    nlev = C.c_int(0)
    sch = L_SCHEME(scheme)
    _check(lib().wd_line_solve_host(kind, r.size, int(periodic), sch, alpha_f, int(fp64),
                                    r.ctypes.data_as(C.POINTER(C.c_double)),
                                    x.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nlev)),
           "wd_line_solve_host", ok=(WD_OK,))
    return x, nlev.value


def wd_seg_solve_host(kind, rhs, periodic, scheme="C6", alpha_f=0.495, M=0):
    """Host FP64 run of the segmented line solve; returns (x, (segments,
    segment length))."""
    import numpy as np
    r = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.empty_like(r)
    su = C.c_int(0)
    _check(lib().wd_seg_solve_host(kind, r.size, int(periodic), L_SCHEME(scheme), alpha_f,
                                   M, r.ctypes.data_as(C.POINTER(C.c_double)),
                                   x.ctypes.data_as(C.POINTER(C.c_double)), C.byref(su)),
           "wd_seg_solve_host", ok=(WD_OK,))
    return x, (su.value // 100, su.value % 100)


def wd_ctx_set_segmented(ctx, enable) -> None:
    """enable: False (reduction-level passes), True (segmented), or 16/24/32
    (segmented, that segment length tried first)."""
    v = int(enable) if not isinstance(enable, bool) else int(enable)
    _check(lib().wd_ctx_set_segmented(ctx, v), "wd_ctx_set_segmented", ok=(WD_OK,))


def wd_ctx_set_lad_tiles(ctx, enable) -> None:
    """enable: the LAD field of uniform Cartesian grids in two tile passes
    (True, the default) or per-direction line passes (False)."""
    _check(lib().wd_ctx_set_lad_tiles(ctx, int(bool(enable))), "wd_ctx_set_lad_tiles",
           ok=(WD_OK,))


def wd_ctx_set_explicit_onepass(ctx, enable) -> None:
    """enable: one pointwise pass per RK stage for explicit schemes on
    uniform Cartesian grids (True, the default) or the line passes (False)."""
    _check(lib().wd_ctx_set_explicit_onepass(ctx, int(bool(enable))),
           "wd_ctx_set_explicit_onepass", ok=(WD_OK,))


def L_SCHEME(s):
    return SCHEMES[s] if isinstance(s, str) else s


def wd_server_create(ctx, budget_bytes: int, max_slots: int):
    h = C.c_void_p()
    _check(lib().wd_server_create(ctx, budget_bytes, max_slots, C.byref(h)), "wd_server_create")
    return h


def wd_server_submit(srv, desc, method, phi_ptr, session=-1, hist_cap=0) -> int:
    rid = C.c_longlong(0)
    _check(lib().wd_server_submit(srv, C.byref(desc), C.byref(method), phi_ptr, session,
                                  hist_cap, C.byref(rid)), "wd_server_submit")
    return rid.value


def wd_server_poll(srv, req_id):
    st, it = C.c_int(0), C.c_int(0)
    ts, ta, td = C.c_double(0), C.c_double(0), C.c_double(0)
    _check(lib().wd_server_poll(srv, req_id, C.byref(st), C.byref(ts), C.byref(ta),
                                C.byref(td), C.byref(it)), "wd_server_poll",
           ok=(WD_OK,))
    return {"status": st.value, "t_submit": ts.value, "t_admit": ta.value,
            "t_done": td.value, "iters": it.value}


def wd_server_wait(srv, req_id, timeout_s=-1.0) -> int:
    return lib().wd_server_wait(srv, req_id, timeout_s)


def wd_server_history(srv, req_id, cap):
    buf = (C.c_double * (2 * max(cap, 1)))()
    n = C.c_int(0)
    _check(lib().wd_server_history(srv, req_id, buf, cap, C.byref(n)), "wd_server_history",
           ok=(WD_OK,))
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]


def wd_server_cancel(srv, req_id) -> int:
    return lib().wd_server_cancel(srv, req_id)


def wd_server_stats(srv):
    d, it, act, rs = C.c_longlong(0), C.c_longlong(0), C.c_int(0), C.c_longlong(0)
    pk = C.c_size_t(0)
    _check(lib().wd_server_stats(srv, C.byref(d), C.byref(it), C.byref(pk), C.byref(act),
                                 C.byref(rs)),
           "wd_server_stats", ok=(WD_OK,))
    return {"done": d.value, "iterations": it.value, "peak_bytes": pk.value,
            "peak_active": act.value, "restarts": rs.value}


def wd_server_destroy(srv) -> None:
    lib().wd_server_destroy(srv)
