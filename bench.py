"""Benchmark of the wall-distance hot path on one MI355X.

Workload (default): the 3D square duct 256^3 on [0,1]^3 (x periodic with
256 distinct points, walls y = 0, 1 and z = 0, 1), LAD pseudo-HJ (eps 0.2,
C 0.1), 6th-order compact derivatives (tridiagonal line solves along every
direction), 10th-order implicit filter (alpha_f 0.495) after every pseudo
step, RK4 with local time stepping, FP32.  One step = 200 pseudo
iterations from phi = 0 (throughput at a fixed iteration count: the march
needs thousands of iterations to converge at this size), with grid and
fields resident in HBM; nothing of an iteration is skipped.

value = grid-point updates per second (points x pseudo iterations / time);
one update is one point through one full pseudo iteration (LAD field, all
RK stages, the filter in every direction, boundary conditions, FP64
residual).

roofline: the compulsory HBM bytes of the method per grid point (27 field
accesses per RK4 iteration on a 3D uniform grid: 5 per RK stage, 2 per
filter direction, 1 for the residual) over measured time, against 8 TB/s.
The dominant unit of work is one RK stage (its directional line passes and
its pointwise finish, about three quarters of an iteration): achieved =
5 accesses x points / the mean duration of a stage's launches, timed with
HIP events on the library's stream in a second pass over the same steps.
The whole iteration's figure sits beside it.  traffic = HBM bytes per
stage from rocprofv3 FETCH_SIZE / WRITE_SIZE counters (calibrated on a
plain copy), kept in profiles/traffic.json and used only while the kernel
sources are unchanged.

Secondary fields: the same duct in FP64, and the 2D cylinder O-grid
512 x 256 (C6, LAD + curvature) solved to convergence in FP32.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_2111_09859_amd import grids as G
    if name == "cylinder":
        spec = G.cylinder(512, 256)
        kw = dict(equation="HJ", gamma="LAD", curvature=True, eps=0.2, scheme="C6", rk="RK4",
                  alpha_f=0.495)
        desc = ("cylinder O-grid 512x256, R=0.5, r_out=20, stretch 1.03 from 1e-3 (capped), "
                "C6 + F10, LAD pseudo-HJ + curvature, RK4")
    elif name == "duct":
        spec = G.duct(256)
        kw = dict(equation="HJ", gamma="LAD", eps=0.2, scheme="C6", rk="RK4", alpha_f=0.495)
        desc = ("3D square duct 256^3 on [0,1]^3, x periodic, walls y,z = 0,1; C6 + F10, "
                "LAD pseudo-HJ (eps 0.2, C 0.1), RK4; 200 pseudo iterations from phi = 0 per step")
    elif name == "channel":
        spec = G.channel(129, 65)
        kw = dict(equation="HJ", gamma="LINEAR", eps=0.1, scheme="E4", rk="RK3", alpha_f=0.495)
        desc = "2D channel 129x65, E4 + F10, standard HJ eps 0.1, RK3"
    else:
        raise SystemExit(f"unknown workload {name}")
    return spec, kw, desc


FP32_STALL = 200    # iterations without a smaller max change that end an FP32 solve


def stop_rule(prec, fixed):
    if fixed:
        return dict(tol=0.0, max_iter=fixed, stall_window=0)
    if prec == "fp32":
        return dict(tol=1e-6, max_iter=20000, stall_window=FP32_STALL)
    return dict(tol=1e-10, max_iter=20000, stall_window=0)


def run_gpu(args, spec, kw, prec, profile=False):
    import torch
    from paper_2111_09859_amd import _lib as L, api
    s = api.Solver(0)
    L.wd_ctx_set_segmented(s.ctx, args.seg)
    prep = s.prepare(spec, kw["scheme"], prec)
    m = api.make_method(precision=prec, **kw, **stop_rule(prec, args.fixed_iters))
    if args.tiles:
        s.set_tiles(prep, [int(w) for w in args.tiles.split(",")])
        tiles = s.tiles(prep)
    else:
        tiles = s.autotune(prep, m, iters=10) if args.autotune else None
    phi = torch.zeros(spec.shape, dtype=prep.dtype, device=s.device)
    for _ in range(args.warmup):
        s.solve(prep, m, phi=phi, check=False)
    torch.cuda.synchronize()
    iters = 0
    statuses = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = s.solve(prep, m, phi=phi, check=False)
        iters += out["iters"]
        statuses.append(out["status"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = []
    prof_iters, prof_time = 0, None
    if profile:
        # kernel timing pass: some of the same steps again, each launch
        # bracketed by HIP events on the library's stream (direct launches,
        # no graph), and the same steps as one graph-replayed region
        nprof = max(1, min(args.steps, args.profile_steps))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nprof):
            s.solve(prep, m, phi=phi, check=False)
        torch.cuda.synchronize()
        prof_time = time.perf_counter() - t0
        L.wd_ctx_profile(s.ctx, True)
        for _ in range(nprof):
            prof_iters += s.solve(prep, m, phi=phi, check=False)["iters"]
        torch.cuda.synchronize()
        stats = L.wd_ctx_profile_read(s.ctx)
        L.wd_ctx_profile(s.ctx, False)
    res = phi.double().cpu().numpy()
    err = float(np.abs(res - spec.exact).max()) if spec.exact is not None else None
    s.close()
    return dict(time=dt, iters=iters, statuses=statuses, err=err, stats=stats, tiles=tiles,
                prof_iters=prof_iters, prof_time=prof_time, stages=4 if kw["rk"] == "RK4" else 3)


KERNEL_SOURCES = ("wd_common.h", "wd_line.h", "wd_line.hip", "wd_kernels.hip", "wd_seg.h",
                  "wd_seg.hip")


def kernel_source_sha():
    """Hash of the device sources: a traffic record is used only while the
    kernels it was measured on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2111_09859_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def run_copy(args):
    """Calibration for the HBM byte counters: plain device copies of a
    known size (1 GiB read + 1 GiB written per copy)."""
    import torch
    n = (1 << 30) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"metric": "copy GB/s", "value": 2 * n * 4 * args.steps / dt / 1e9, "unit": "GB/s",
            "copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "steps": args.steps}


def _rocpd_files(d):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True))


def _pmc_rows(d):
    """Counter rows of a rocprofv3 --pmc output directory (SQLite results
    database or CSV): dicts with Dispatch_Id, Kernel_Name, Counter_Name,
    Counter_Value (KiB for FETCH_SIZE / WRITE_SIZE)."""
    import csv
    import glob
    rows = []
    for f in _rocpd_files(d):
        import sqlite3
        con = sqlite3.connect(f)
        for disp, name, ctr, val in con.execute(
                "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": ctr,
                         "Counter_Value": val})
        con.close()
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    if not rows:
        raise SystemExit(f"no counter rows under {d}")
    return rows


def trace_summary(d):
    """Markdown table of a rocprofv3 --kernel-trace --stats output directory
    (SQLite results database): calls, average and total duration per
    kernel."""
    import sqlite3
    files = _rocpd_files(d)
    if not files:
        raise SystemExit(f"no results database under {d}")
    con = sqlite3.connect(files[0])
    lines = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    # the database's summary view gives durations in microseconds
    for name, calls, tot, avg, pct in con.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"):
        lines.append(f"| `{_kernel_base(name)[:60]}` | {calls} | {avg:.2f} | {tot / 1e3:.3f} "
                     f"| {pct:.2f} |")
    con.close()
    return "\n".join(lines)


def _kernel_base(name):
    """'void wd::k_seg_cart<float, 32, false>(...)' -> 'k_seg_cart<float, 32, false>'."""
    n = name.split("(")[0].replace("void ", "").strip()
    return n.split("::")[-1] if "::" in n.split("<")[0] else n


def _per_dispatch(rows, counter):
    """[(kernel, counter value in KiB)] per dispatch for one counter."""
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        nm, v = _kernel_base(r["Kernel_Name"]), float(r["Counter_Value"])
        old = per.get(key, (nm, 0.0))
        per[key] = (nm, old[1] + v)
    return list(per.values())


def _per_kernel(rows, counter):
    """{kernel: [dispatches, summed counter value in KiB]} for one counter."""
    out = {}
    for nm, v in _per_dispatch(rows, counter):
        e = out.setdefault(nm, [0, 0.0])
        e[0] += 1
        e[1] += v
    return out


# kernels of one RK stage, and of the rest of a pseudo iteration
STAGE_KERNELS = ("k_seg_cart<", "k_seg_cart_fin<", "k_cart_finish<", "k_cart<", "k_d1<",
                 "k_d12<", "k_d2<", "k_uwadv<", "k_final<", "k_face<", "k_xstage<")
ITER_KERNELS = STAGE_KERNELS + ("k_seg_lad<", "k_lad<", "k_xlad", "k_seg_filter<", "k_filter<",
                                "k_resid<", "k_finalize")


def _in(name, group):
    return any(name.startswith(k) for k in group)


def pmc_summary(args):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE / WRITE_SIZE of a run of
    exactly --pmc-iters pseudo iterations of the workload, the same of the
    copy calibration) into HBM bytes per RK stage and per iteration, written
    to profiles/traffic.json."""
    wl, dfetch, dwrite, cfetch, cwrite = args.pmc_summary
    copy_bytes = float(1 << 30)
    factors = {}
    for d, ctr in ((cfetch, "FETCH_SIZE"), (cwrite, "WRITE_SIZE")):
        # the largest copy dispatch is one 1 GiB device copy
        big = [v for nm, v in _per_dispatch(_pmc_rows(d), ctr) if "copy" in nm.lower()]
        if not big:
            raise SystemExit(f"no copy kernel in {d}")
        factors[ctr] = copy_bytes / (max(big) * 1024.0)
    its, stages = args.pmc_iters, args.pmc_iters * args.pmc_stages
    rec = {"iters": its, "stages": stages, "kernels": {},
           "copy_factor_fetch": factors["FETCH_SIZE"], "copy_factor_write": factors["WRITE_SIZE"],
           "source_sha256": kernel_source_sha()}
    for d, ctr in ((dfetch, "FETCH_SIZE"), (dwrite, "WRITE_SIZE")):
        rows = _pmc_rows(d)
        # the solve starts at its initial field: dispatches before it (the
        # FP64 metric helpers of a curvilinear grid) are set-up, not iterations
        inits = [int(r["Dispatch_Id"]) for r in rows if _kernel_base(r["Kernel_Name"]).startswith("k_init<")]
        if inits:
            rows = [r for r in rows if int(r["Dispatch_Id"]) > min(inits)]
        per = _per_kernel(rows, ctr)
        key = "fetch" if ctr == "FETCH_SIZE" else "write"
        for nm, (n, v) in per.items():
            if not _in(nm, ITER_KERNELS):
                continue
            k = rec["kernels"].setdefault(nm, {"dispatches": n})
            k[f"{key}_bytes_per_dispatch"] = v / n * 1024.0 * factors[ctr]
        for grp, div in (("stage", stages), ("iteration", its)):
            tot = sum(v for nm, (n, v) in per.items()
                      if _in(nm, STAGE_KERNELS if grp == "stage" else ITER_KERNELS))
            rec[f"{key}_bytes_per_{grp}"] = tot * 1024.0 * factors[ctr] / div
    for grp in ("stage", "iteration"):
        rec[f"hbm_bytes_per_{grp}"] = rec[f"fetch_bytes_per_{grp}"] + rec[f"write_bytes_per_{grp}"]
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    allrec = json.load(open(tpath)) if os.path.exists(tpath) else {}
    allrec[wl] = rec
    with open(tpath, "w") as f:
        json.dump(allrec, f, indent=1, sort_keys=True)
        f.write("\n")
    return rec


# Compulsory field accesses per grid point (bytes = accesses x value size):
# each live RK state field read or written once per stage, the local step
# stored once, one read and one write per filter direction, one read for
# the residual; curvilinear 2D grids read their 4 metric fields per stage.
def compulsory_accesses(ndim, uniform, rk4):
    stage = 5 if rk4 else 11.0 / 3.0
    met = 0 if uniform else ndim * ndim
    stages = 4 if rk4 else 3
    per_stage = stage + met
    return per_stage, per_stage * stages + 2 * ndim + 1


def roofline(r, spec, prec, workload_key):
    """Achieved HBM bandwidth of the compulsory bytes of one RK stage (the
    dominant unit of work) and of the whole pseudo iteration.

    The durations come from HIP events recorded around every launch of a
    second, non-graph pass over the same steps.  Each event pair also holds
    the launch's dispatch latency, which the graph replay of the timed
    region hides; that overhead per launch is (sum of the event-timed
    durations - the same steps timed as graph replays) / launches, and it is
    removed from every launch."""
    stats = r["stats"]
    if not stats or not r["prof_iters"]:
        return None
    S = 8.0 if prec == "fp64" else 4.0
    acc_stage, acc_iter = compulsory_accesses(spec.ndim, spec.coords is None, r["stages"] == 4)
    n_it = r["prof_iters"]
    n_st = n_it * r["stages"]
    tot_ms = sum(k["total_ms"] for k in stats)
    nl = sum(k["launches"] for k in stats)
    over_s = max(0.0, (tot_ms * 1e-3 - r["prof_time"]) / nl) if r["prof_time"] else 0.0
    kern = {}
    for k in stats:
        avg = k["total_ms"] * 1e-3 / k["launches"] - over_s
        kern[k["name"]] = {"launches": k["launches"], "avg_us": round(avg * 1e6, 2),
                           "avg_us_events": round(k["total_ms"] * 1e3 / k["launches"], 2)}
    base = lambda nm: nm.split("/")[0] + "<"          # library name -> kernel prefix
    stage_names = [nm for nm in kern if _in(base(nm), STAGE_KERNELS)]
    stage_s = sum(kern[nm]["avg_us"] * kern[nm]["launches"] for nm in stage_names) * 1e-6 / n_st
    iter_s = sum(v["avg_us"] * v["launches"] for v in kern.values()) * 1e-6 / n_it
    alg_stage = acc_stage * S * spec.npoints
    alg_iter = acc_iter * S * spec.npoints
    achieved = alg_stage / stage_s / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        rec = json.load(open(tpath)).get(workload_key, {})
        if rec.get("source_sha256") == kernel_source_sha():
            traffic = rec.get("hbm_bytes_per_stage")
    out = {"bound": "hbm",
           "kernel": "one RK stage: " + " + ".join(sorted(set(nm for nm in stage_names))),
           "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
           "alg_bytes_per_launch": alg_stage, "alg_accesses_per_point": acc_stage,
           "avg_launch_us": stage_s * 1e6,
           "iteration": {"alg_accesses_per_point": acc_iter, "alg_bytes": alg_iter,
                         "avg_us": iter_s * 1e6, "achieved": alg_iter / iter_s / 1e9,
                         "frac": alg_iter / iter_s / 1e9 / HBM_PEAK_GBS},
           "event_overhead_us": over_s * 1e6, "profiled_iters": n_it,
           "kernels": kern}
    if traffic:
        out["hbm_GBps_measured_traffic"] = traffic / stage_s / 1e9
        out["traffic_efficiency"] = alg_stage / traffic
    return out


def cpu_info():
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def run_cpu_baseline(spec, kw, iters, threads):
    """The FP64 oracle on the same grid and method for `iters` pseudo
    iterations from phi = 0 on `threads` threads: (point-updates/s, seconds,
    threads used)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    O.build(force=False)
    used = O.set_threads(threads)
    m = O.make_method(equation={"HJ": O.HJ, "EIKONAL": O.EIKONAL, "POISSON": O.POISSON}[kw["equation"]],
                      gamma={"LAD": O.GAMMA_LAD, "LINEAR": O.GAMMA_LINEAR}[kw["gamma"]],
                      curvature=int(kw.get("curvature", False)), eps=kw["eps"], scheme=kw["scheme"],
                      rk={"RK4": O.RK4, "RK3": O.RK3}[kw["rk"]], alpha_f=kw["alpha_f"],
                      fixed_iters=iters)
    t0 = time.perf_counter()
    O.solve(spec, m)
    dt = time.perf_counter() - t0
    return spec.npoints * iters / dt, dt, used


ALPHA_F = 0.48   # filter coefficient of the batch and serving workloads
BATCH_TOL = 1e-6
BATCH_STALL = 200


def method_for(spec, scheme, prec, **over):
    from paper_2111_09859_amd import api
    # the paper's convergence criterion (Eq. Con-criter): max change <= 1e-5
    # L_ref, the same stated target for both precisions; the FP32 stall
    # window is only a safety net at the rounding floor
    kw = dict(equation="HJ", gamma="LAD", eps=0.2, scheme=scheme, rk="RK4",
              curvature=spec.coords is not None, precision=prec, alpha_f=ALPHA_F,
              tol=1e-5, max_iter=20000, stall_window=1000 if prec == "fp32" else 0)
    kw.update(over)
    return api.make_method(**kw)


def batch_tiles(spec, target=2048):
    """Tile widths holding about `target` points (whole lines)."""
    n0, n1 = spec.n[0], spec.n[1]
    return [max(1, min(n1, target // n0)), max(1, min(n0, target // n1, 64))]


def run_batch(args):
    """The batch workload: 64 seeded 2D grids (channel / cylinder / ellipse O-grids,
    E6 / C6, LAD pseudo-HJ + curvature on O-grids) solved as ONE FP32 batch
    versus the same grids solved one at a time in FP64."""
    import torch
    from paper_2111_09859_amd import api, grids as G
    mix = G.batch_mix(args.batch_count)
    s = api.Solver(0)
    p32 = [s.prepare(spec, sch, "fp32") for spec, sch in mix]
    # the batch's stopping rule: max change <= 1e-6 in both precisions (FP32
    # with the stall window at its rounding floor), tight enough that the
    # two runs' distances from their fixed points stay below the 1e-5
    # accuracy bar
    m32 = [method_for(spec, sch, "fp32", tol=BATCH_TOL, stall_window=BATCH_STALL) for spec, sch in mix]
    # tiles of about 2048 points: a full batch is throughput bound, so each
    # shape gets fewer, larger tiles than its solo latency optimum
    for p in p32:
        s.set_tiles(p, batch_tiles(p.spec))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = s.solve_batched(p32, m32, check=False)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    print(f"[batch] FP32 batched: {t32:.1f} s", file=sys.stderr, flush=True)
    e32 = [G.linf_error(sp, ph.double().cpu().numpy()) for ph, (sp, _) in zip(out["phi"], mix)]
    t64, e64, it64, st64, d3264, max_abs64 = 0.0, [], [], [], [], []
    seen = set()
    for (spec, sch), ph32 in zip(mix, out["phi"]):
        p = s.prepare(spec, sch, "fp64")
        m = method_for(spec, sch, "fp64", tol=BATCH_TOL)
        if spec.n not in seen:      # same tile tuning as the batched run
            seen.add(spec.n)
            s.autotune(p, m, iters=4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve(p, m, check=False)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t0
        f64 = r["phi"].cpu().numpy()
        e64.append(G.linf_error(spec, f64))
        print(f"[batch] FP64 plain grid {len(e64)}/{len(mix)}: {r['iters']} its", file=sys.stderr,
              flush=True)
        it64.append(r["iters"])
        st64.append(r["status"])
        keep = G.scored(spec)
        d3264.append(float(np.abs(ph32.double().cpu().numpy() - f64)[keep].max()))
        max_abs64.append(float(np.abs(f64).max()))
    pts = sum(sp.npoints for sp, _ in mix)
    # "same stated accuracy": both runs finished (no divergence) and their
    # L-inf errors against the exact distance agree within 5 % or within the
    # FP32 accuracy bar, 1e-5 of the field's largest value (the relative
    # L-inf of every parity statement); beside it, the FP32 field within
    # 1e-5 relative of the FP64 one
    ok = [i for i in range(len(mix)) if out["status"][i] >= 0 and st64[i] >= 0
          and abs(e32[i] - e64[i]) <= 0.05 * e64[i] + 1e-5 * max_abs64[i]]
    close = [i for i in range(len(mix)) if d3264[i] <= 1e-5 * max_abs64[i]]
    return {
        "metric": "solves/s (FP32 batched)", "value": len(mix) / t32, "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * t32,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(mix)} seeded 2D grids (channel/cylinder/ellipse, E6/C6, "
                               "LAD pseudo-HJ + curvature on O-grids), 65x33..1025x513",
                   "points": pts, "batched_fp32_s": t32, "plain_fp64_s": t64,
                   "plain_fp64_solves_per_s": len(mix) / t64,
                   "speedup_fp32_batched_vs_fp64_plain": t64 / t32,
                   "fp32_iters": out["iters"], "fp64_iters": it64,
                   "fp32_status": out["status"], "fp64_status": st64,
                   "linf_fp32_minus_fp64": d3264,
                   "max_abs_fp64": max_abs64,
                   "linf_err_fp32": e32, "linf_err_fp64": e64,
                   "grids_same_accuracy": len(ok),
                   "grids_fp32_within_1e-5_rel_of_fp64": len(close),
                   "linf_err_median_same_accuracy": float(np.median([e64[i] for i in ok])) if ok else None}}


def run_ratios(args):
    """GPU counterpart of the paper's timing comparisons (Sec. 5.2, 5.3):
    time per 100 pseudo iterations of the first-order upwind baseline (no
    filter) and of the central schemes (with the filter, alpha_f 0.48), and
    time / iterations / error to the paper's criterion (max change <= 1e-5),
    FP64, default tiles: the 129x65 channel with standard HJ (eps 0.1) and
    with LAD HJ, and a 129x129 2-D box with the Eikonal equation."""
    import torch
    from paper_2111_09859_amd import api, grids as G
    s = api.Solver(0)
    cases = [("channel129x65_hj", G.channel(129, 65), dict(equation="HJ", gamma="LINEAR", eps=0.1)),
             ("channel129x65_lad", G.channel(129, 65), dict(equation="HJ", gamma="LAD", eps=0.2)),
             ("box129_eikonal", G.box2d(129), dict(equation="EIKONAL"))]
    # the central Eikonal on the four-wall box grows without bound from its
    # corners at alpha_f >= 0.48 with Courant number 1 (the oracle does the
    # same); a stronger filter, alpha_f 0.45, keeps every scheme stable there
    alpha = {"box129_eikonal": 0.45}
    out = {}
    for name, spec, kw in cases:
        row = {}
        for sch in ("UW", "E2", "E4", "C4", "C6"):
            filt = sch != "UW"
            prep = s.prepare(spec, sch, "fp64")
            af = alpha.get(name, 0.48)
            m = api.make_method(scheme=sch, filter=filt, alpha_f=af, tol=0.0, max_iter=300,
                                precision="fp64", rk="RK4", **kw)
            s.solve(prep, m, check=False)               # warm-up (graphs, tables)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve(prep, m, check=False)
            torch.cuda.synchronize()
            per100 = (time.perf_counter() - t0) / 3.0
            mc = api.make_method(scheme=sch, filter=filt, alpha_f=af, tol=1e-5, max_iter=50000,
                                 precision="fp64", rk="RK4", **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.solve(prep, mc, check=False)
            torch.cuda.synchronize()
            tc = time.perf_counter() - t0
            row[sch] = {"ms_per_100_iters": 1e3 * per100, "iters_to_1e-5": r["iters"],
                        "status": r["status"], "s_to_1e-5": tc,
                        "linf_err": float(np.abs(r["phi"].cpu().numpy() - spec.exact).max())}
            print(f"[ratios] {name} {sch}: {1e3 * per100:.2f} ms/100 its, {r['iters']} its, "
                  f"{tc:.3f} s to 1e-5", file=sys.stderr, flush=True)
        for sch in row:
            row[sch]["uw_time_per_iter_over_this"] = (row["UW"]["ms_per_100_iters"]
                                                      / row[sch]["ms_per_100_iters"])
        out[name] = row
    return {"metric": "time per 100 pseudo iterations, central vs upwind", "value": None,
            "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
            "data": "synthetic", "vs_baseline": None,
            "config": {"workload": "channel 129x65 (HJ standard, HJ LAD), box 129x129 (Eikonal); "
                                   "UW without filter, E2/E4/C4/C6 with F10 alpha_f 0.48 "
                                   "(0.45 on the Eikonal box), RK4",
                       "results": out}}


def run_burnback(args):
    """Level-set burnback of the star grain (Sec. 5.5): the signed distance
    from two FP32 E4 LAD pseudo-HJ solves (gas side, propellant side, to the
    paper's 1e-5), then RK4 steps of d phi_s/dt + F |grad phi_s| = 0 at
    F = 0.3 with dt = h / (2 F), the lengths of the levels 0, 0.05, 0.1 and
    -0.02 every 50 steps (the burning perimeter S_b per unit depth is the
    level 0).  March-only runs on a 4096^2 grid from the analytic six-lobed
    front and on a 256^3 grid (x periodic) from a wavy tube give the stage
    kernels' bandwidth in 2D and 3D."""
    import torch
    from paper_2111_09859_amd import api, grids as G
    s = api.Solver(0)
    n = args.burn_n
    gas, sol = G.star_grain(n), G.star_grain_solid(n)
    m = method_for(gas, "E4", "fp32", eps=0.2)
    pg, ps_ = s.prepare(gas, "E4", "fp32"), s.prepare(sol, "E4", "fp32")
    for p in (pg, ps_):
        s.autotune(p, m, iters=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rg = s.solve(pg, m, check=False)
    rs = s.solve(ps_, m, check=False)
    mask = torch.as_tensor(gas.mask, device=s.device).contiguous()
    phi = s.signed_distance(mask, rs["phi"], rg["phi"])
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    print(f"[burnback] init {t_init:.2f} s ({rg['iters']} + {rs['iters']} iterations)",
          file=sys.stderr, flush=True)
    F, dt = 0.3, 0.5 * gas.h[0] / 0.3
    levels = [0.0, 0.05, 0.1, -0.02]
    series = [(0.0, s.level_lengths(pg, phi, levels))]
    t_march = 0.0
    done = 0
    while done < args.burn_steps:
        k = min(50, args.burn_steps - done)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.levelset_advance(pg, phi, F, dt, k)
        torch.cuda.synchronize()
        t_march += time.perf_counter() - t1
        done += k
        series.append((done * dt, s.level_lengths(pg, phi, levels)))
    print(f"[burnback] {done} steps in {t_march:.3f} s", file=sys.stderr, flush=True)
    # bandwidth of the march on a large grid (no solves)
    big = G.square(args.burn_big, 0.5)
    X, Y = G.square_xy(big)
    front = np.hypot(X, Y) - 0.2 * (1 + 0.3 * np.cos(6 * np.arctan2(Y, X)))
    pb = s.prepare(big, "UW", "fp32")
    pbig = torch.as_tensor(front, dtype=torch.float32, device=s.device).contiguous()
    bdt = 0.5 * big.h[0] / F
    s.levelset_advance(pb, pbig, F, bdt, 4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.levelset_advance(pb, pbig, F, bdt, args.burn_big_steps)
    torch.cuda.synchronize()
    t_big = time.perf_counter() - t2
    # compulsory bytes of one step's stage kernels: stage 0 reads phi and
    # writes the stage value and the accumulator; stages 1 and 2 read the
    # stage value, phi and the accumulator and write two; stage 3 reads two
    # and writes phi: 64 B per point (FP32), faces excluded
    nb = big.npoints
    step_bytes = 16.0 * 4 * nb
    bw = step_bytes * args.burn_big_steps / t_big / 1e9
    # and a 3D march: the 256^3 duct grid (x periodic) from a wavy tube
    cube = G.duct(args.burn_big3)
    k, j, i = np.meshgrid(*(np.arange(n) for n in reversed(cube.n)), indexing="ij")
    tube = (np.hypot(j * cube.h[1] - 0.5, k * cube.h[2] - 0.5) - 0.25
            + 0.05 * np.sin(2 * np.pi * i / cube.n[0]))
    del k, j, i
    pc = s.prepare(cube, "UW", "fp32")
    p3 = torch.as_tensor(tube, dtype=torch.float32, device=s.device).contiguous()
    del tube
    cdt = 0.5 * min(cube.h) / F
    s.levelset_advance(pc, p3, F, cdt, 4)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    s.levelset_advance(pc, p3, F, cdt, args.burn_big_steps)
    torch.cuda.synchronize()
    t_3d = time.perf_counter() - t3
    bw3 = 16.0 * 4 * cube.npoints * args.burn_big_steps / t_3d / 1e9
    return {
        "metric": "level-set point-updates/s", "value": gas.npoints * done / t_march,
        "unit": "point-updates/s", "n_gpus": 1, "steps": done, "warmup": 0,
        "ms_per_step": 1e3 * t_march / done, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"star-grain burnback {n}x{n}: signed distance from two E4 LAD "
                               f"pseudo-HJ solves, {done} RK4 level-set steps at F = 0.3",
                   "init_s": t_init, "init_iters": [rg["iters"], rs["iters"]],
                   "init_status": [rg["status"], rs["status"]],
                   "levels": levels, "lengths": [[t, l] for t, l in series],
                   "march_4096_ms_per_step": 1e3 * t_big / args.burn_big_steps,
                   "march_4096_point_updates_per_s": nb * args.burn_big_steps / t_big,
                   "march_4096_stage_GBps": bw, "march_4096_frac_of_8TBps": bw / HBM_PEAK_GBS,
                   "march_3d_grid": list(cube.n),
                   "march_3d_ms_per_step": 1e3 * t_3d / args.burn_big_steps,
                   "march_3d_stage_GBps": bw3, "march_3d_frac_of_8TBps": bw3 / HBM_PEAK_GBS}}


def run_moving(args):
    """Moving walls (the unsteady cases of Sec. 5.5), FP32, E4 LAD pseudo-HJ
    at eps 0.15 and sigma 0.5, stopped at max change <= 1e-5: a piston in
    an annular bore (128 x 49 x 97 O-grid, half a stroke, h 1.4 -> 0.6 in
    24 physical steps) and a cube bouncing between a floor and a ceiling
    (129^3 Cartesian grid, the cube a moving mask, 24 steps over 6 time
    units: three bounces).  Each sequence runs cold (every step from zero)
    and warm (every step from the previous step's field); grids are built
    before the timed region, placing them (coordinates, metrics, mask) is
    inside it."""
    import torch
    from paper_2111_09859_amd import api, grids as G
    s = api.Solver(0)
    steps = args.moving_steps
    m = api.make_method(equation="HJ", gamma="LAD", eps=0.15, scheme="E4", alpha_f=ALPHA_F,
                        sigma=0.5, tol=1e-5, max_iter=20000, stall_window=1000,
                        precision="fp32")
    hs = G.piston_stroke(2 * steps)[: steps + 1]
    zs = G.bounce_heights(steps, 6.0)
    cases = {
        "piston": [G.piston(128, 49, 97, h) for h in hs],
        "cube": [G.bouncing_cube(129, z) for z in zs],
    }

    def probe(name, spec, phi):
        """Field and exact distance at a fixed point off the ridges: the
        piston's at r = 0.5 (0.25 from the rod), theta = 0, z = 0.5, linear
        in z between grid planes; the cube's at the node (0.25, 0.5, 0.5)
        beside its path."""
        if name == "piston":
            hz = spec.meta["h"] / (spec.n[2] - 1)
            k = min(int(0.5 / hz), spec.n[2] - 2)
            w = 0.5 / hz - k
            j = (spec.n[1] - 1) // 3
            v = (1 - w) * phi[k, j, 0] + w * phi[k + 1, j, 0]
            return float(v), min(0.25, 0.5, spec.meta["h"] - 0.5)
        n = spec.n[0] - 1
        q = (n // 2, n // 2, n // 4)
        return float(phi[q]), float(spec.exact[q])

    out = {}
    total_steps, total_warm = 0, 0.0
    for name, specs in cases.items():
        s.autotune(s.prepare(specs[0], "E4", "fp32"), m, iters=10)
        rec = {"points": specs[0].npoints}
        for mode in ("cold", "warm"):
            probes = []

            def on_step(k, spec, res, name=name, probes=probes):
                if k % 4 == 0 or k == len(specs) - 1:
                    v, e = probe(name, spec, res["phi"].cpu().numpy())
                    probes.append([k, round(v, 5), round(e, 5)])

            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _ = s.solve_sequence(specs, m, "E4", "fp32", warm=mode == "warm",
                                     on_step=on_step)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            its = [i for _, i, _ in st]
            rec[mode] = {"s": dt, "iters_total": int(sum(its)), "iters_first": its[0],
                         "iters_later_mean": float(np.mean(its[1:])),
                         "status": sorted(set(c for c, _, _ in st)),
                         "restarted_cold": [k for k, (_, _, r) in enumerate(st) if r],
                         "probe": probes}
            print(f"[moving {name} {mode}] {dt:.2f} s, iterations {its}", file=sys.stderr,
                  flush=True)
        rec["warm_speedup_s"] = rec["cold"]["s"] / rec["warm"]["s"]
        rec["warm_iters_ratio_later"] = (rec["cold"]["iters_later_mean"]
                                         / rec["warm"]["iters_later_mean"])
        out[name] = rec
        total_steps += len(specs)
        total_warm += rec["warm"]["s"]
    return {
        "metric": "moving-wall physical steps/s", "value": total_steps / total_warm,
        "unit": "steps/s", "n_gpus": 1, "steps": total_steps, "warmup": 0,
        "ms_per_step": 1e3 * total_warm / total_steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"piston 128x49x97 ({steps + 1} positions, half a stroke) and "
                               f"bouncing cube 129^3 ({steps + 1} positions over three bounces), "
                               "E4 LAD pseudo-HJ to 1e-5, warm-started",
                   "cases": out}}


def run_serve(args):
    """The serving workload: open-loop Poisson arrivals (--serve-rate, default
    200 req/s; a rate at or below the server's measured capacity
    gives latencies of the server rather than of an overloaded queue) of
    --serve-count 2D grids 129^2..2049^2 and 3D ducts 64^3..192^3 into the
    continuous-batching server, beside 4 closed-loop warm-started
    star-grain sessions of --serve-steps steps.  FP32, LAD pseudo-HJ, stop
    at max change <= 1e-5 (the paper's criterion)."""
    import threading
    import torch
    from paper_2111_09859_amd import api, grids as G
    s = api.Solver(0)
    srv = api.Server(s, budget_bytes=args.serve_budget << 20, max_slots=64)
    stream = G.serving_stream(count=args.serve_count, rate=args.serve_rate)
    over = dict(tol=1e-5, stall_window=500, max_iter=20000)
    ids = []
    sess_lat = []

    def sessions():
        ss = api.Solver(0)
        phis = {}
        for k in range(args.serve_steps):
            rids = []
            for sid in range(4):
                spec = G.star_grain(512, step=k + 5 * sid)
                p = ss.prepare(spec, "E6", "fp32")
                if sid not in phis:
                    phis[sid] = torch.zeros(spec.shape, dtype=torch.float32, device=ss.device)
                m = method_for(spec, "E6", "fp32", eps=0.15, warm_start=k > 0, **over)
                rids.append((srv.submit(p, m, phi=phis[sid], session=100 + sid), p))
            for rid, p in rids:
                srv.wait(rid, 600.0)
                info = srv.poll(rid)
                sess_lat.append((info["t_done"] - info["t_submit"], info["iters"], k))
            print(f"[serve] session step {k + 1}/{args.serve_steps} done", file=sys.stderr,
                  flush=True)
        ss.close()

    th = threading.Thread(target=sessions)
    t0 = time.perf_counter()
    th.start()
    for req in stream:
        delay = req["t"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        spec = G.build_request(req)
        p = s.prepare(spec, req["scheme"], "fp32")
        ids.append((srv.submit(p, method_for(spec, req["scheme"], "fp32", **over)), spec))
        if len(ids) % 10 == 0:
            print(f"[serve] {len(ids)}/{len(stream)} requests submitted at "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    # requests finish out of order (smallest first): report the count done
    pending = [rid for rid, _ in ids]
    while pending:
        srv.wait(pending[0], 10.0)
        pending = [rid for rid in pending if srv.poll(rid)["status"] == api.L.WD_PENDING]
        print(f"[serve] {len(ids) - len(pending)}/{len(ids)} requests done at "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if time.perf_counter() - t0 > 3600:
            raise RuntimeError("serving run did not finish")
    th.join()
    wall = time.perf_counter() - t0
    lat, qwait, its, pts = [], [], [], 0
    for rid, spec in ids:
        info = srv.poll(rid)
        lat.append(info["t_done"] - info["t_submit"])
        qwait.append(info["t_admit"] - info["t_submit"])
        its.append(info["iters"])
        pts += spec.npoints * info["iters"]
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    cold = [l for l, it, k in sess_lat if k == 0]
    warm = [l for l, it, k in sess_lat if k > 0]
    warm_it = [it for l, it, k in sess_lat if k > 0]
    cold_it = [it for l, it, k in sess_lat if k == 0]
    n = len(ids) + len(sess_lat)
    return {
        "metric": "served solves/s", "value": n / wall, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": 1e3 * wall, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(ids)} Poisson-arrival requests ({args.serve_rate:g}/s) "
                               f"+ 4 warm-started star-grain sessions x {args.serve_steps} steps",
                   "arrival_rate_per_s": args.serve_rate, "requests": len(ids),
                   "session_steps": args.serve_steps,
                   "warm_restarts": st.get("restarts"),
                   "p50_latency_s": float(np.percentile(lat, 50)),
                   "p99_latency_s": float(np.percentile(lat, 99)),
                   "p50_queue_wait_s": float(np.percentile(qwait, 50)),
                   "point_updates_per_s": pts / wall,
                   "session_cold_latency_s": float(np.mean(cold)) if cold else None,
                   "session_warm_latency_s": float(np.mean(warm)) if warm else None,
                   "session_cold_iters": float(np.mean(cold_it)) if cold_it else None,
                   "session_warm_iters": float(np.mean(warm_it)) if warm_it else None,
                   "peak_arena_bytes": st["peak_bytes"], "peak_active": st["peak_active"],
                   "budget_bytes": args.serve_budget << 20}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="duct")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--fixed-iters", type=int, default=None,
                    help="pseudo iterations per step (default: 200 for the duct, a full "
                         "solve otherwise; 0 = full solve)")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle iterations of the all-core CPU baseline (default: "
                         "2 x 256^3 point-updates' worth, at least 2)")
    ap.add_argument("--cpu-iters-1t", type=int, default=None,
                    help="oracle iterations of the one-thread CPU baseline (default: "
                         "256^3 point-updates' worth, at least 1)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core baseline (0: OMP_NUM_THREADS, else all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the cylinder O-grid secondary measurement")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default tile widths (no tuning before the timed steps)")
    ap.add_argument("--tiles", default=None,
                    help="tile widths per direction, e.g. 1,2 (skips the autotuner)")
    ap.add_argument("--no-profile", action="store_true",
                    help="no per-kernel event timing (roofline is then null)")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="steps of the per-launch event timing pass")
    ap.add_argument("--pmc-summary", nargs=5, metavar=("KEY", "FETCH_DIR", "WRITE_DIR",
                                                       "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="derive HBM bytes per RK stage from rocprofv3 --pmc output")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="print the kernel table of a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--pmc-iters", type=int, default=2,
                    help="pseudo iterations in the counted runs")
    ap.add_argument("--pmc-stages", type=int, default=4)
    ap.add_argument("--alpha-f", type=float, default=None,
                    help="filter coefficient (default: the workload's)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--serve-count", type=int, default=200)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="arrivals per second")
    ap.add_argument("--serve-budget", type=int, default=4096, help="arena MiB")
    ap.add_argument("--burn-n", type=int, default=1024)
    ap.add_argument("--burn-steps", type=int, default=500)
    ap.add_argument("--burn-big", type=int, default=4096)
    ap.add_argument("--burn-big-steps", type=int, default=40)
    ap.add_argument("--burn-big3", type=int, default=256)
    ap.add_argument("--moving-steps", type=int, default=24)
    ap.add_argument("--stall-window", type=int, default=None,
                    help="FP32 solves: iterations without a smaller max change that end them")
    ap.add_argument("--scheme", default=None,
                    help="derivative scheme in place of the workload's (E2, E4, E6, C4, C6)")
    ap.add_argument("--seg", type=int, default=1,
                    help="segmented Cartesian passes: 0 off, 1 auto, 16/24/32 segment length")
    args = ap.parse_args()
    global ALPHA_F, FP32_STALL
    if args.alpha_f is not None:
        ALPHA_F = args.alpha_f
    if args.stall_window is not None:
        FP32_STALL = args.stall_window
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(grids are independent; see the multi-GPU design notes)", file=sys.stderr)
        raise SystemExit(2)

    if args.pmc_summary:
        print(json.dumps(pmc_summary(args)), flush=True)
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary), flush=True)
        return
    if args.workload == "copy":
        print(json.dumps(run_copy(args)), flush=True)
        return
    if args.workload == "ratios":
        print(json.dumps(run_ratios(args)), flush=True)
        return
    if args.workload == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.workload == "burnback":
        print(json.dumps(run_burnback(args)), flush=True)
        return
    if args.workload == "moving":
        print(json.dumps(run_moving(args)), flush=True)
        return
    if args.fixed_iters is None:
        args.fixed_iters = 200 if args.workload == "duct" else 0
    spec, kw, desc = workload(args.workload)
    if args.alpha_f is not None:
        kw["alpha_f"] = args.alpha_f
    if args.scheme:
        kw["scheme"] = args.scheme
        desc += f", scheme {args.scheme} in place of the above"
    desc += f", alpha_f {kw['alpha_f']}"
    print(f"[bench] {args.workload} {args.precision}: {args.warmup} + {args.steps} steps",
          file=sys.stderr, flush=True)
    r = run_gpu(args, spec, kw, args.precision, profile=not args.no_profile)
    ups = spec.npoints * r["iters"] / r["time"]
    line = {
        "metric": "grid-point updates/s",
        "value": ups,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["time"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "points": spec.npoints,
                   "iters_per_step": r["iters"] / args.steps,
                   "ms_per_iter": 1e3 * r["time"] / r["iters"],
                   "status": r["statuses"][-1], "linf_err_vs_exact": r["err"],
                   "tile_widths": r["tiles"],
                   "stop": stop_rule(args.precision, args.fixed_iters)},
    }
    if not args.fixed_iters:
        line["config"]["solves_per_s"] = args.steps / r["time"]
    print(f"[bench] {ups:.4g} point-updates/s", file=sys.stderr, flush=True)
    if not args.no_fp64 and args.precision == "fp32":
        a64 = argparse.Namespace(**vars(args))
        a64.steps, a64.warmup = max(1, min(args.steps, args.fp64_steps)), 1
        r64 = run_gpu(a64, spec, kw, "fp64")
        line["config"]["fp64"] = {"value": spec.npoints * r64["iters"] / r64["time"],
                                  "steps": a64.steps,
                                  "ms_per_iter": 1e3 * r64["time"] / r64["iters"],
                                  "iters_per_step": r64["iters"] / a64.steps,
                                  "linf_err_vs_exact": r64["err"],
                                  "status": r64["statuses"][-1]}
        print("[bench] fp64 leg done", file=sys.stderr, flush=True)
    if args.workload == "duct" and not args.no_secondary:
        cspec, ckw, cdesc = workload("cylinder")
        ca = argparse.Namespace(**vars(args))
        ca.steps, ca.warmup, ca.fixed_iters = 3, 1, 0
        rc = run_gpu(ca, cspec, ckw, "fp32")
        line["config"]["cylinder"] = {
            "workload": cdesc + ", alpha_f 0.495; one step = one full solve from phi = 0",
            "value": cspec.npoints * rc["iters"] / rc["time"], "unit": "point-updates/s",
            "solves_per_s": ca.steps / rc["time"], "ms_per_solve": 1e3 * rc["time"] / ca.steps,
            "iters_per_solve": rc["iters"] / ca.steps, "status": rc["statuses"][-1],
            "linf_err_vs_exact": rc["err"], "stop": stop_rule("fp32", 0)}
        print("[bench] cylinder leg done", file=sys.stderr, flush=True)
        # the same duct with the explicit E6 scheme (one pointwise pass per
        # RK stage), FP32, 200 iterations per step
        ea = argparse.Namespace(**vars(args))
        ea.steps, ea.warmup = max(1, min(args.steps, 3)), 1
        ekw = dict(kw, scheme="E6")
        re6 = run_gpu(ea, spec, ekw, "fp32", profile=not args.no_profile)
        line["config"]["duct_e6"] = {
            "workload": "the same duct and method with E6 explicit derivatives "
                        "(one pass per RK stage: k_xstage, fast and edge tiles)",
            "value": spec.npoints * re6["iters"] / re6["time"], "unit": "point-updates/s",
            "ms_per_iter": 1e3 * re6["time"] / re6["iters"], "steps": ea.steps,
            "iters_per_step": re6["iters"] / ea.steps,
            "roofline": roofline(re6, spec, "fp32", "duct-e6-fp32")}
        print("[bench] duct E6 leg done", file=sys.stderr, flush=True)
    line["roofline"] = roofline(r, spec, args.precision, f"{args.workload}-{args.precision}")
    if not args.no_cpu:
        model, ncpu, avail = cpu_info()
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS") or 0) or avail
        # a bounded sample of the workload: about as many point-updates as
        # 2 (all cores) and 1 (one thread) iterations of the 256^3 duct, a
        # few seconds to some tens of seconds of host work whatever the grid
        if args.cpu_iters is None:
            args.cpu_iters = max(2, round(2 * 256 ** 3 / spec.npoints))
        if args.cpu_iters_1t is None:
            args.cpu_iters_1t = max(1, round(256 ** 3 / spec.npoints))
        v, dt, used = run_cpu_baseline(spec, kw, args.cpu_iters, threads)
        print(f"[bench] oracle, {used} threads: {dt:.1f} s", file=sys.stderr, flush=True)
        v1, dt1, _ = run_cpu_baseline(spec, kw, args.cpu_iters_1t, 1)
        print(f"[bench] oracle, 1 thread: {dt1:.1f} s", file=sys.stderr, flush=True)
        line["cpu_baseline"] = {
            "value": v, "unit": "point-updates/s", "cores": used, "kind": "oracle",
            "sample": f"{args.cpu_iters} pseudo iterations of the same workload (full grid) "
                      f"from phi = 0, FP64, {used} threads: {dt:.1f} s",
            "one_thread": {"value": v1, "seconds": dt1,
                           "sample": f"{args.cpu_iters_1t} pseudo iteration(s), full grid"},
            "host": {"cpu_model": model, "nproc": ncpu, "cpus_available": avail}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
