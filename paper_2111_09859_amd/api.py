"""Convenience layer over the C ABI: builds descriptors from
:class:`~paper_2111_09859_amd.grids.GridSpec` objects, places coordinates,
masks, metrics, fields and the workspace in device memory with PyTorch, and
calls the library.  Argument marshalling only -- every arithmetic step of the
solve runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib as L
from .grids import GridSpec

EQUATIONS = {"EIKONAL": L.WD_EQ_EIKONAL, "HJ": L.WD_EQ_HJ, "POISSON": L.WD_EQ_POISSON}
GAMMAS = {"LINEAR": L.WD_GAMMA_LINEAR, "LAD": L.WD_GAMMA_LAD}
RKS = {"RK3": L.WD_RK3_SSP, "RK4": L.WD_RK4}
PRECISIONS = {"fp32": L.WD_FP32, "fp64": L.WD_FP64}


def _torch():
    import torch
    return torch


def make_method(equation="HJ", gamma="LAD", curvature=False, eps=0.2, c_lad=0.1,
                nu0=1e-3, eps0=1e-6, scheme="C6", filter=True, alpha_f=0.48, rk="RK4",
                sigma=1.0, tol=1e-10, max_iter=100000, stall_window=0, precision="fp64",
                warm_start=False, warm_probe=300) -> L.wd_method:
    m = L.wd_method()
    m.equation = EQUATIONS[equation] if isinstance(equation, str) else equation
    m.gamma = GAMMAS[gamma] if isinstance(gamma, str) else gamma
    m.curvature = int(bool(curvature))
    m.eps, m.c_lad, m.nu0, m.eps0 = eps, c_lad, nu0, eps0
    m.scheme = L.SCHEMES[scheme] if isinstance(scheme, str) else scheme
    m.filter = int(bool(filter))
    m.alpha_f = alpha_f
    m.rk = RKS[rk] if isinstance(rk, str) else rk
    m.sigma, m.tol, m.max_iter, m.stall_window = sigma, tol, max_iter, stall_window
    m.precision = PRECISIONS[precision] if isinstance(precision, str) else precision
    m.warm_start = int(bool(warm_start))
    m.warm_probe = int(warm_probe)
    return m


@dataclass
class Prepared:
    """A grid placed on the device: descriptor plus the tensors it points at."""
    spec: GridSpec
    desc: L.wd_grid_desc
    metrics: Optional[object]
    mask: Optional[object]
    dtype: object


class Solver:
    """One library context on one device."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = L.wd_ctx_create(device)
        self._ws = None

    def close(self):
        if self.ctx:
            L.wd_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    # -- placement -----------------------------------------------------
    def prepare(self, spec: GridSpec, scheme="C6", precision="fp64") -> Prepared:
        torch = self.torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        d = L.wd_grid_desc()
        d.ndim = spec.ndim
        for i in range(3):
            d.n[i] = spec.n[i] if i < spec.ndim else 1
            for s in range(2):
                d.bc[i][s] = spec.bc[i][s] if i < spec.ndim else L.WD_BC_WALL
        met = None
        if spec.coords is None:
            d.metric_mode = L.WD_METRIC_UNIFORM
            for i in range(3):
                d.h[i] = spec.h[i] if i < spec.ndim else 1.0
        else:
            d.metric_mode = L.WD_METRIC_FIELDS
            coords = torch.as_tensor(np.ascontiguousarray(spec.coords, dtype=np.float64),
                                     device=self.device)
            met = torch.empty((spec.ndim * spec.ndim,) + spec.shape, dtype=dt,
                              device=self.device)
            L.wd_compute_metrics_form(self.ctx, d, L.SCHEMES[scheme] if isinstance(scheme, str)
                                      else scheme, int(getattr(spec, "metric_form", 0)),
                                      C.c_void_p(coords.data_ptr()), spec.period,
                                      C.c_void_p(met.data_ptr()), PRECISIONS[precision],
                                      self.stream())
            d.metrics = met.data_ptr()
        mask = None
        if spec.mask is not None:
            mask = torch.as_tensor(np.ascontiguousarray(spec.mask, dtype=np.uint8),
                                   device=self.device)
            d.mask = mask.data_ptr()
        return Prepared(spec, d, met, mask, dt)

    def workspace(self, nbytes: int):
        torch = self.torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return self._ws

    # -- solves --------------------------------------------------------
    def solve(self, prep: Prepared, method: L.wd_method, phi=None, hist_cap=None,
              aux=False, check=True):
        """Returns dict(phi, status, iters, hist[, aux])."""
        torch = self.torch
        if phi is None:
            phi = torch.zeros(prep.spec.shape, dtype=prep.dtype, device=self.device)
        nb = L.wd_workspace_bytes(self.ctx, [prep.desc], [method])
        ws = self.workspace(nb)
        cap = method.max_iter if hist_cap is None else hist_cap
        cap = max(1, min(cap, 1 << 20))
        hist = (C.c_double * (2 * cap))()
        auxt = torch.empty_like(phi) if aux else None
        rc, iters = L.wd_solve(self.ctx, prep.desc, method, C.c_void_p(phi.data_ptr()),
                               C.c_void_p(auxt.data_ptr()) if aux else None, hist, cap,
                               C.c_void_p(ws.data_ptr()), ws.numel(), self.stream(),
                               check=check)
        h = np.frombuffer(hist, dtype=np.float64).reshape(cap, 2)[: min(iters, cap)].copy()
        out = {"phi": phi, "status": rc, "iters": iters, "hist": h}
        if aux:
            out["aux"] = auxt
        return out

    def autotune(self, prep: Prepared, method: L.wd_method, iters: int = 20):
        """Pick and cache the fastest tile width per direction for this grid."""
        torch = self.torch
        phi = torch.zeros(prep.spec.shape, dtype=prep.dtype, device=self.device)
        ws = self.workspace(L.wd_workspace_bytes(self.ctx, [prep.desc], [method]))
        return L.wd_autotune(self.ctx, prep.desc, method, C.c_void_p(phi.data_ptr()),
                             C.c_void_p(ws.data_ptr()), ws.numel(), iters, self.stream())

    def tiles(self, prep: Prepared):
        """Tile widths used for this grid's shape and precision."""
        return L.wd_tune_get(self.ctx, prep.desc, PRECISIONS["fp64" if prep.dtype == self.torch.float64
                                                             else "fp32"])

    # -- moving walls (the unsteady cases of Sec. 5.5) ------------------
    def solve_sequence(self, specs, method: L.wd_method, scheme="E4", precision="fp64",
                       warm=True, on_step=None, probe=300):
        """Wall distance while the walls move: one pseudo-time solve per
        physical time step, on that step's grid (the same index dimensions
        at every step; metrics, mask and walls may change).  With warm,
        each solve after the first starts from the previous step's field at
        the same grid indices, the previous physical time step's solution
        being the initial estimate; without, every solve starts from zero.
        on_step(k, spec, result) is called after each step's solve (the
        result's field is overwritten by the next step).

        A warm estimate far from the new walls (a wall that moved many
        cells in one step) can start a runaway below zero beside a new
        wall; the library's runaway check (wd_method.warm_probe = probe
        iterations) then stops the solve with WD_ERR_WARM_RUNAWAY, and a
        warm solve that ends so, or that does not end converged or
        stagnated, is solved again from zero.  Returns the list of
        (status, iterations, restarted) -- iterations include a failed
        warm attempt -- and the last step's result."""
        torch = self.torch
        phi, out, steps = None, None, []
        for k, spec in enumerate(specs):
            prep = self.prepare(spec, scheme, precision)
            m = L.wd_method.from_buffer_copy(method)
            m.warm_start = int(bool(warm) and phi is not None)
            m.warm_probe = int(probe)
            if phi is None or tuple(phi.shape) != tuple(spec.shape):
                if m.warm_start:
                    raise ValueError("solve_sequence: grid dimensions changed between steps")
                phi = torch.zeros(spec.shape, dtype=prep.dtype, device=self.device)
            restarted, spent = False, 0
            if m.warm_start:
                out = self.solve(prep, m, phi=phi, hist_cap=1, check=False)
                spent = out["iters"]
                if out["status"] not in (L.WD_OK, L.WD_STAGNATED):
                    restarted = True
                    m.warm_start = 0
            if not m.warm_start:
                out = self.solve(prep, m, phi=phi, hist_cap=1)
                out["iters"] += spent
            steps.append((out["status"], out["iters"], restarted))
            if on_step is not None:
                on_step(k, spec, out)
        return steps, out

    # -- level-set burnback (Sec. 5.5) ---------------------------------
    def _prec(self, prep: Prepared):
        return L.WD_FP64 if prep.dtype == self.torch.float64 else L.WD_FP32

    def signed_distance(self, solid, d_solid, d_gas):
        """phi_s = d_solid on solid points (uint8 device mask), -d_gas elsewhere."""
        torch = self.torch
        out = torch.empty_like(d_solid)
        prec = L.WD_FP64 if d_solid.dtype == torch.float64 else L.WD_FP32
        L.wd_signed_distance(self.ctx, d_solid.numel(), prec, C.c_void_p(solid.data_ptr()),
                             C.c_void_p(d_solid.data_ptr()), C.c_void_p(d_gas.data_ptr()),
                             C.c_void_p(out.data_ptr()), self.stream())
        return out

    def levelset_advance(self, prep: Prepared, phi_s, speed: float, dt: float, nsteps: int):
        """nsteps RK4 steps of d phi_s/dt + speed |grad phi_s| = 0, in place."""
        prec = self._prec(prep)
        ws = self.workspace(L.wd_levelset_workspace_bytes(self.ctx, prep.desc, prec))
        L.wd_levelset_advance(self.ctx, prep.desc, prec, speed, dt, nsteps,
                              C.c_void_p(phi_s.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                              self.stream())
        return phi_s

    def level_lengths(self, prep: Prepared, phi_s, levels):
        """Lengths of the 2D iso-lines phi_s = level for each level."""
        prec = self._prec(prep)
        ws = self.workspace(L.wd_levelset_workspace_bytes(self.ctx, prep.desc, prec))
        return L.wd_level_lengths(self.ctx, prep.desc, prec, C.c_void_p(phi_s.data_ptr()),
                                  list(levels), C.c_void_p(ws.data_ptr()), ws.numel(),
                                  self.stream())

    def set_tiles(self, prep: Prepared, widths):
        """Use these tile widths for this grid's shape and precision."""
        L.wd_tune_set(self.ctx, prep.desc, PRECISIONS["fp64" if prep.dtype == self.torch.float64
                                                      else "fp32"], widths)

    def solve_batched(self, preps, methods, phis=None, hist_cap=0, check=True):
        torch = self.torch
        if phis is None:
            phis = [torch.zeros(p.spec.shape, dtype=p.dtype, device=self.device) for p in preps]
        nb = L.wd_workspace_bytes(self.ctx, [p.desc for p in preps], list(methods))
        ws = self.workspace(nb)
        hists = None
        if hist_cap > 0:
            hists = [(C.c_double * (2 * hist_cap))() for _ in preps]
        rc, iters, status = L.wd_solve_batched(
            self.ctx, [p.desc for p in preps], list(methods),
            [C.c_void_p(p.data_ptr()) for p in phis], None, hists, hist_cap,
            C.c_void_p(ws.data_ptr()), ws.numel(), self.stream(), check=check)
        out = {"phi": phis, "rc": rc, "iters": iters, "status": status}
        if hists is not None:
            out["hist"] = [np.frombuffer(h, dtype=np.float64).reshape(hist_cap, 2)[: min(it, hist_cap)].copy()
                           for h, it in zip(hists, iters)]
        return out


class Server:
    """Continuous-batching request loop (wd_server_*) on a Solver's device.
    Keeps the tensors of submitted requests alive until they finish."""

    def __init__(self, solver: Solver, budget_bytes: int, max_slots: int = 64):
        self.solver = solver
        self.srv = L.wd_server_create(solver.ctx, int(budget_bytes), int(max_slots))
        self._keep = {}

    def submit(self, prep: Prepared, method: L.wd_method, phi=None, session: int = -1,
               hist_cap: int = 0) -> int:
        torch = self.solver.torch
        if phi is None:
            phi = torch.zeros(prep.spec.shape, dtype=prep.dtype, device=self.solver.device)
        # phi (and the grid's metrics) must be ready before the server reads them
        torch.cuda.current_stream(self.solver.device).synchronize()
        rid = L.wd_server_submit(self.srv, prep.desc, method, C.c_void_p(phi.data_ptr()),
                                 session, hist_cap)
        self._keep[rid] = (prep, phi)
        return rid

    def wait(self, rid: int, timeout_s: float = -1.0) -> int:
        return L.wd_server_wait(self.srv, rid, timeout_s)

    def poll(self, rid: int) -> dict:
        return L.wd_server_poll(self.srv, rid)

    def result(self, rid: int):
        return self._keep[rid][1]

    def history(self, rid: int, cap: int):
        return L.wd_server_history(self.srv, rid, cap)

    def cancel(self, rid: int) -> int:
        return L.wd_server_cancel(self.srv, rid)

    def stats(self) -> dict:
        return L.wd_server_stats(self.srv)

    def close(self):
        if self.srv:
            L.wd_server_destroy(self.srv)
            self.srv = None
