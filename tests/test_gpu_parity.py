"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.

FP64: element-wise relative L-inf <= 1e-12 (max |gpu - oracle| / max |oracle|)
at an equal number of pseudo iterations.  FP32: <= 1e-5 against the
oracle's FP64 result (fixed iterations) or FP64 fixed point (converged).
"""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_09859_amd import api
    s = api.Solver(0)
    yield s
    s.close()


def say(*a):
    print(*a, flush=True)


def omethod(O, eq="HJ", gamma="LINEAR", curv=0, eps=0.2, scheme="C6", rk="RK4",
            alpha_f=0.495, filt=1, tol=1e-10, fixed=0, max_iter=100000):
    return O.make_method(equation={"EIKONAL": O.EIKONAL, "HJ": O.HJ, "POISSON": O.POISSON}[eq],
                         gamma={"LINEAR": O.GAMMA_LINEAR, "LAD": O.GAMMA_LAD}[gamma],
                         curvature=curv, eps=eps, scheme=scheme,
                         rk={"RK3": O.RK3, "RK4": O.RK4}[rk], alpha_f=alpha_f, filter=filt,
                         tol=tol, fixed_iters=fixed, max_iter=max_iter)


def gmethod(eq="HJ", gamma="LINEAR", curv=0, eps=0.2, scheme="C6", rk="RK4", alpha_f=0.495,
            filt=1, tol=1e-10, max_iter=100000, precision="fp64", stall=0):
    from paper_2111_09859_amd import api
    return api.make_method(equation=eq, gamma=gamma, curvature=curv, eps=eps, scheme=scheme,
                           rk=rk, alpha_f=alpha_f, filter=filt, tol=tol, max_iter=max_iter,
                           precision=precision, stall_window=stall)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_fixed(solver, spec, n_iter, precision="fp64", **kw):
    m = gmethod(tol=0.0, max_iter=n_iter, precision=precision, **kw)
    prep = solver.prepare(spec, kw.get("scheme", "C6"), precision)
    out = solver.solve(prep, m)
    assert out["iters"] == n_iter, out
    return out["phi"].double().cpu().numpy(), out


def oracle_fixed(O, spec, n_iter, **kw):
    phi, st, it, h = O.solve(spec, omethod(O, fixed=n_iter, **kw))
    assert it == n_iter
    return phi, h


CASES = [
    # name, spec builder, method kwargs, iterations
    ("channel37x29_E2_hj", lambda: G.channel(37, 29), dict(eq="HJ", scheme="E2", eps=0.1), 40),
    ("channel37x29_E4_hj_rk3", lambda: G.channel(37, 29), dict(eq="HJ", scheme="E4", eps=0.1, rk="RK3"), 40),
    ("channel37x29_E6_lad", lambda: G.channel(37, 29), dict(eq="HJ", gamma="LAD", scheme="E6"), 40),
    ("channel37x29_C4_eik", lambda: G.channel(37, 29), dict(eq="EIKONAL", scheme="C4"), 40),
    ("channel37x29_C6_poisson", lambda: G.channel(37, 29), dict(eq="POISSON", scheme="C6"), 40),
    ("channel37x29_C6_lad", lambda: G.channel(37, 29), dict(eq="HJ", gamma="LAD", scheme="C6"), 40),
    ("box33_C6_lad", lambda: G.box2d(33), dict(eq="HJ", gamma="LAD", scheme="C6"), 40),
    # curvature on Cartesian boxes amplifies rounding while the normal is
    # ill-defined in the flat interior: compare after few iterations
    ("box33_E4_curv_cart", lambda: G.box2d(33), dict(eq="HJ", curv=1, scheme="E4"), 4),
    ("cyl48x40_C6_lad_curv", lambda: G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12),
     dict(eq="HJ", gamma="LAD", curv=1, scheme="C6"), 40),
    ("cyl48x40_E4_lin_curv_neumann", lambda: G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12,
                                                         far=G.NEUMANN),
     dict(eq="HJ", curv=1, scheme="E4"), 40),
    # annulus between two walls: no extrapolated face, so the finishing pass
    # forms the next stage's F from values it holds in LDS before any face step
    ("cyl48x40_E6_lad_walls", lambda: G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12,
                                                  far=G.WALL),
     dict(eq="HJ", gamma="LAD", scheme="E6"), 40),
    ("ell40x33_E6_eik", lambda: G.ellipse(40, 33, axis_ratio=2.0, ratio=1.15, rout=5.0, dr1=1e-2),
     dict(eq="EIKONAL", scheme="E6"), 40),
    ("ell40x33_C6_poisson", lambda: G.ellipse(40, 33, axis_ratio=2.0, ratio=1.15, rout=5.0, dr1=1e-2),
     dict(eq="POISSON", scheme="C6"), 30),
    ("star64_E6_lad_mask", lambda: G.star_grain(64), dict(eq="HJ", gamma="LAD", scheme="E6", eps=0.15), 40),
    ("duct17x17x12_C6_lad", lambda: G.duct(17, nx=12), dict(eq="HJ", gamma="LAD", scheme="C6"), 25),
    ("duct17x17x12_E4_poisson", lambda: G.duct(17, nx=12), dict(eq="POISSON", scheme="E4"), 25),
    ("duct17x17x12_C4_curv", lambda: G.duct(17, nx=12), dict(eq="HJ", curv=1, scheme="C4"), 3),
    # the upwind baseline (Eqs. UW1-UW5), run without the filter as the paper's
    ("channel37x29_UW_eik", lambda: G.channel(37, 29), dict(eq="EIKONAL", scheme="UW", filt=0), 40),
    ("channel37x29_UW_hj_rk3", lambda: G.channel(37, 29),
     dict(eq="HJ", scheme="UW", eps=0.1, rk="RK3", filt=0), 40),
    ("box33_UW_lad", lambda: G.box2d(33), dict(eq="HJ", gamma="LAD", scheme="UW", filt=0), 40),
    ("cyl48x40_UW_hj_neumann", lambda: G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12,
                                                   far=G.NEUMANN),
     dict(eq="HJ", scheme="UW", filt=0), 40),
    ("ell40x33_UW_eik", lambda: G.ellipse(40, 33, axis_ratio=2.0, ratio=1.15, rout=5.0, dr1=1e-2),
     dict(eq="EIKONAL", scheme="UW", filt=0), 40),
    ("star64_UW_eik_mask", lambda: G.star_grain(64), dict(eq="EIKONAL", scheme="UW", filt=0), 40),
    ("duct17x17x12_UW_lad", lambda: G.duct(17, nx=12), dict(eq="HJ", gamma="LAD", scheme="UW", filt=0), 25),
]


@pytest.mark.parametrize("name,build,kw,n_iter", CASES, ids=[c[0] for c in CASES])
def test_fp64_fixed_iterations(solver, oracle, name, build, kw, n_iter):
    spec = build()
    say(f"[parity fp64] {name} shape={spec.shape} iters={n_iter}")
    g, out = gpu_fixed(solver, spec, n_iter, **kw)
    o, h = oracle_fixed(oracle, spec, n_iter, **kw)
    if kw.get("eq") == "POISSON":
        o = oracle.poisson_distance(spec, kw["scheme"], o)
    e = rel(g, o)
    say(f"   rel_linf={e:.3e}")
    assert e <= FP64_TOL
    # residual history (FP64 on both sides)
    assert np.allclose(out["hist"][:, 0], h[:, 0], rtol=1e-8, atol=1e-14)


def test_channel_129x65_converged(solver, oracle):
    """129 x 65 channel, E4, RK3, standard HJ (eps 0.1), FP64 to 1e-10:
    the GPU stops at the oracle's iteration and matches its field."""
    spec = G.channel(129, 65)
    kw = dict(eq="HJ", scheme="E4", eps=0.1, rk="RK3")
    say("[parity fp64] channel 129x65 converged")
    prep = solver.prepare(spec, "E4", "fp64")
    out = solver.solve(prep, gmethod(tol=1e-10, **kw))
    o, st, it, h = oracle.solve(spec, omethod(oracle, tol=1e-10, **kw))
    say(f"   gpu iters={out['iters']} oracle iters={it}")
    assert out["status"] == 0 and st == 0
    assert abs(out["iters"] - it) <= 1
    o2, _ = oracle_fixed(oracle, spec, out["iters"], **kw)
    e = rel(out["phi"].cpu().numpy(), o2)
    say(f"   rel_linf={e:.3e}")
    assert e <= FP64_TOL


@pytest.mark.parametrize("name,build,kw,n_iter", [
    ("channel65x33_C6_hj", lambda: G.channel(65, 33), dict(eq="HJ", scheme="C6", eps=0.1), 60),
    ("cyl48x40_C6_lad_curv", lambda: G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12),
     dict(eq="HJ", gamma="LAD", curv=1, scheme="C6"), 60),
    ("duct17_E6_lad", lambda: G.duct(17, nx=12), dict(eq="HJ", gamma="LAD", scheme="E6"), 30),
], ids=lambda v: v if isinstance(v, str) else None)
def test_fp32_fixed_iterations(solver, oracle, name, build, kw, n_iter):
    spec = build()
    say(f"[parity fp32] {name} iters={n_iter}")
    g, _ = gpu_fixed(solver, spec, n_iter, precision="fp32", **kw)
    o, _ = oracle_fixed(oracle, spec, n_iter, **kw)
    e = rel(g, o)
    say(f"   rel_linf={e:.3e}")
    assert e <= FP32_TOL


def test_fp32_converged_vs_fp64_fixed_point(solver, oracle):
    spec = G.cylinder(64, 48, rout=5.0, dr1=1e-2, ratio=1.1)
    kw = dict(eq="HJ", gamma="LAD", curv=1, scheme="C6")
    say("[parity fp32 converged] cylinder 64x48 LAD+curvature")
    o, st, it, h = oracle.solve(spec, omethod(oracle, tol=1e-12, max_iter=20000, **kw))
    assert st == 0
    prep = solver.prepare(spec, "C6", "fp32")
    out = solver.solve(prep, gmethod(tol=1e-6, stall=300, max_iter=20000, precision="fp32", **kw))
    e = rel(out["phi"].double().cpu().numpy(), o)
    say(f"   gpu status={out['status']} iters={out['iters']} oracle iters={it} rel_linf={e:.3e}")
    assert out["status"] in (0, 2)
    assert e <= FP32_TOL


def test_metrics_parity(solver, oracle):
    import torch
    from paper_2111_09859_amd import _lib as L
    for spec, scheme in ((G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12), "C6"),
                         (G.ellipse(33, 29, axis_ratio=3.0, ratio=1.2, rout=5.0, dr1=1e-2), "E4"),
                         (G.channel_curvilinear(24, 17), "C4"),
                         (G.channel_curvilinear(24, 17), "E6")):
        prep = solver.prepare(spec, scheme, "fp64")
        g = prep.metrics.cpu().numpy()
        o = oracle.metrics(spec, scheme)
        e = rel(g, o)
        say(f"[metrics] {spec.name} {scheme} rel_linf={e:.3e}")
        assert e <= FP64_TOL


def test_poisson_distance_entry(solver, oracle):
    import ctypes as C
    import torch
    from paper_2111_09859_amd import _lib as L, api
    spec = G.ellipse(40, 33, axis_ratio=2.0, ratio=1.15, rout=5.0, dr1=1e-2)
    rng = np.random.default_rng(7)
    phip = np.abs(rng.standard_normal(spec.shape)) + spec.exact ** 2
    prep = solver.prepare(spec, "C6", "fp64")
    src = torch.as_tensor(phip, device=solver.device)
    dst = torch.empty_like(src)
    m = gmethod(eq="POISSON", scheme="C6")
    ws = solver.workspace(L.wd_workspace_bytes(solver.ctx, [prep.desc], [m]))
    L.wd_poisson_distance(solver.ctx, prep.desc, L.WD_C6, L.WD_FP64, C.c_void_p(src.data_ptr()),
                          C.c_void_p(dst.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                          solver.stream())
    o = oracle.poisson_distance(spec, "C6", phip)
    e = rel(dst.cpu().numpy(), o)
    say(f"[poisson distance] rel_linf={e:.3e}")
    assert e <= FP64_TOL


def test_warm_start_resumes(solver, oracle):
    spec = G.channel(33, 17)
    kw = dict(eq="HJ", scheme="E4", eps=0.1)
    prep = solver.prepare(spec, "E4", "fp64")
    first = solver.solve(prep, gmethod(tol=1e-11, **kw))
    from paper_2111_09859_amd import api
    m = gmethod(tol=1e-11, **kw)
    m.warm_start = 1
    again = solver.solve(prep, m, phi=first["phi"].clone())
    say(f"[warm start] first={first['iters']} again={again['iters']}")
    assert again["iters"] <= 2
    assert rel(again["phi"].cpu().numpy(), first["phi"].cpu().numpy()) < 1e-10


def test_failure_paths(solver):
    import torch
    from paper_2111_09859_amd import _lib as L
    spec = G.channel(33, 17)
    prep = solver.prepare(spec, "E4", "fp64")
    # non-finite guess -> diverged
    m = gmethod(scheme="E4", tol=1e-10, max_iter=50)
    m.warm_start = 1
    phi = torch.full(spec.shape, float("nan"), dtype=torch.float64, device=solver.device)
    out = solver.solve(prep, m, phi=phi, check=False)
    assert out["status"] == L.WD_ERR_DIVERGED
    # iteration limit -> not converged, valid history
    out = solver.solve(prep, gmethod(scheme="E4", tol=1e-14, max_iter=3))
    assert out["status"] == L.WD_NOT_CONVERGED and out["iters"] == 3 and len(out["hist"]) == 3
    # bad descriptor
    bad = L.wd_grid_desc()
    bad.ndim = 4
    with pytest.raises(L.WDError):
        L.wd_workspace_bytes(solver.ctx, [bad], [gmethod()])
    # workspace too small
    rc, _ = L.wd_solve(solver.ctx, prep.desc, gmethod(scheme="E4"),
                       torch.zeros(spec.shape, dtype=torch.float64, device=solver.device).data_ptr(),
                       None, None, 0, solver.workspace(16).data_ptr(), 16, solver.stream(),
                       check=False)
    assert rc == L.WD_ERR_NO_MEMORY


def test_batched_equals_alone_bitwise(solver):
    """Each grid of a mixed batch (sizes, geometries, schemes, equations)
    gives bitwise the field it gives when solved alone."""
    specs = [(G.channel(65, 33), dict(eq="HJ", gamma="LAD", scheme="E6")),
             (G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12),
              dict(eq="HJ", gamma="LAD", curv=1, scheme="C6")),
             (G.ellipse(40, 33, axis_ratio=2.0, ratio=1.15, rout=5.0, dr1=1e-2),
              dict(eq="EIKONAL", scheme="C6")),
             (G.channel(37, 29), dict(eq="POISSON", scheme="E4")),
             (G.duct(17, nx=12), dict(eq="HJ", gamma="LAD", scheme="C6"))]
    for prec in ("fp32", "fp64"):
        preps, meths, alone = [], [], []
        for spec, kw in specs:
            p = solver.prepare(spec, kw["scheme"], prec)
            m = gmethod(tol=0.0, max_iter=35, precision=prec, **kw)
            preps.append(p)
            meths.append(m)
            alone.append(solver.solve(p, m)["phi"].cpu().numpy())
        out = solver.solve_batched(preps, meths, hist_cap=40)
        for i, (a, b) in enumerate(zip(alone, out["phi"])):
            b = b.cpu().numpy()
            say(f"[batched {prec}] grid {i} max|diff|={np.abs(a - b).max():.3e}")
            assert np.array_equal(a, b)


def test_autotune_keeps_results_bitwise(solver):
    """Tile widths change speed only: a solve after autotuning gives bitwise
    the field of the untuned solve."""
    from paper_2111_09859_amd import api
    spec = G.cylinder(96, 64, rout=6.0, dr1=1e-2, ratio=1.08)
    m = gmethod(eq="HJ", gamma="LAD", curv=1, scheme="C6", tol=0.0, max_iter=40, precision="fp32")
    fresh = api.Solver(0)
    try:
        prep = fresh.prepare(spec, "C6", "fp32")
        before = fresh.solve(prep, m)["phi"].cpu().numpy()
        widths = fresh.autotune(prep, m, iters=8)
        say(f"[autotune] widths={widths}")
        after = fresh.solve(prep, m)["phi"].cpu().numpy()
        assert np.array_equal(before, after)
    finally:
        fresh.close()
