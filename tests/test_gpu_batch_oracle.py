"""Batched and served solves against the FP64 oracle, grid by grid.

A mix of uneven grids (sizes, geometries, schemes, equations, Gamma forms,
solid masks) runs at a fixed number of pseudo iterations (Sec. 3.3-3.5 per
grid) three ways -- as one batch (one set of launches per RK stage for all
of them), through the continuous-batching server, and alone -- and every
grid's field is compared element by element with the oracle's after the
same iterations: FP64 relative L-inf <= 1e-12 (and the FP64 change history
to 1e-8), FP32 <= 1e-5.  LAD cases stop after a few iterations: while the
front moves, the LAD sensor amplifies rounding-level differences between
any two summation orders (the oracle against itself included).
"""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

from test_gpu_parity import FP32_TOL, FP64_TOL, gmethod, omethod, rel, say

pytestmark = pytest.mark.gpu

MIX2D = [
    ("channel65x33_E6_lad", lambda: G.channel(65, 33), dict(eq="HJ", gamma="LAD", scheme="E6"), 12),
    ("cyl48x40_C6_lad_curv", lambda: G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12),
     dict(eq="HJ", gamma="LAD", curv=1, scheme="C6"), 12),
    ("ell40x33_C6_lad_curv", lambda: G.ellipse(40, 33, axis_ratio=2.5, ratio=1.15, rout=5.0,
                                               dr1=1e-2),
     dict(eq="HJ", gamma="LAD", curv=1, scheme="C6"), 12),
    # a uniform Cartesian grid: segmented line passes inside the batch
    ("channel129x65_C6_lad", lambda: G.channel(129, 65),
     dict(eq="HJ", gamma="LAD", scheme="C6"), 12),
    ("star64_E6_lad_mask", lambda: G.star_grain(64),
     dict(eq="HJ", gamma="LAD", scheme="E6", eps=0.15), 12),
    ("box33_E4_eikonal", lambda: G.box2d(33), dict(eq="EIKONAL", scheme="E4"), 30),
    ("channel37x29_E4_poisson", lambda: G.channel(37, 29), dict(eq="POISSON", scheme="E4"), 30),
    ("cyl40x24_E6_linear_neumann", lambda: G.cylinder(40, 24, rout=4.0, dr1=2e-2, ratio=1.1,
                                                      far=G.NEUMANN),
     dict(eq="HJ", scheme="E6"), 30),
]

MIX3D = [
    ("duct17x17x12_C6_lad", lambda: G.duct(17, nx=12), dict(eq="HJ", gamma="LAD", scheme="C6"), 10),
    ("duct40x33x33_E4_poisson", lambda: G.duct(33, nx=40), dict(eq="POISSON", scheme="E4"), 20),
    ("piston16x9x13_E4_lad", lambda: G.piston(16, 9, 13, 0.8),
     dict(eq="HJ", gamma="LAD", scheme="E4", eps=0.15), 10),
]

_REF = {}


def oracle_ref(O, name, spec, kw, n):
    """The oracle's field after n iterations (Poisson: converted to the
    distance of Eq. Poiss2, as the library returns it) and its history."""
    if name not in _REF:
        phi, st, it, h = O.solve(spec, omethod(O, fixed=n, **kw))
        assert it == n
        if kw.get("eq") == "POISSON":
            phi = O.poisson_distance(spec, kw["scheme"], phi)
        _REF[name] = (phi, h)
    return _REF[name]


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_09859_amd import api
    s = api.Solver(0)
    yield s
    s.close()


def _check(O, name, spec, kw, n, phi, prec, hist=None, tag=""):
    ref, h = oracle_ref(O, name, spec, kw, n)
    e = rel(phi, ref)
    say(f"[{tag} {prec}] {name}: rel_linf={e:.2e}")
    assert e <= (FP64_TOL if prec == "fp64" else FP32_TOL), name
    if hist is not None and prec == "fp64":
        assert np.allclose(hist[:, 0], h[:, 0], rtol=1e-8, atol=1e-14), name


@pytest.mark.parametrize("mix", ["2d", "3d"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_grids_vs_oracle(solver, oracle, mix, prec):
    cases = MIX2D if mix == "2d" else MIX3D
    specs = [build() for _, build, _, _ in cases]
    preps = [solver.prepare(sp, kw["scheme"], prec) for sp, (_, _, kw, _) in zip(specs, cases)]
    meths = [gmethod(tol=0.0, max_iter=n, precision=prec, **kw) for _, _, kw, n in cases]
    out = solver.solve_batched(preps, meths, hist_cap=64)
    for i, ((name, _, kw, n), spec) in enumerate(zip(cases, specs)):
        assert out["iters"][i] == n
        _check(oracle, name, spec, kw, n, out["phi"][i].double().cpu().numpy(), prec,
               out["hist"][i], tag=f"batch {mix}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_served_grids_vs_oracle(solver, oracle, prec):
    """The 2D and 3D mixes submitted together to the server (grids of both
    kinds iterate side by side, each group in its own launches)."""
    from paper_2111_09859_amd import api, _lib as L
    cases = MIX2D + MIX3D
    srv = api.Server(solver, budget_bytes=512 << 20, max_slots=16)
    try:
        ids, specs = [], []
        for name, build, kw, n in cases:
            spec = build()
            specs.append(spec)
            p = solver.prepare(spec, kw["scheme"], prec)
            ids.append(srv.submit(p, gmethod(tol=0.0, max_iter=n, precision=prec, **kw),
                                  hist_cap=64))
        for rid, spec, (name, _, kw, n) in zip(ids, specs, cases):
            st = srv.wait(rid, 120.0)
            info = srv.poll(rid)
            assert st == L.WD_NOT_CONVERGED and info["iters"] == n, (name, st, info)
            hist = np.array(srv.history(rid, 64)).reshape(-1, 2)
            _check(oracle, name, spec, kw, n, srv.result(rid).double().cpu().numpy(), prec,
                   hist, tag="served")
        assert srv.stats()["peak_active"] > 1
    finally:
        srv.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_served_warm_session_step_vs_oracle(solver, oracle, prec):
    """A warm-started session step through the server (the receding star
    grain of Sec. 5.5): the previous step's field is the oracle's converged
    field of the grain at step 0; the server advances the grain at step 4
    from it for a fixed number of iterations, the oracle does the same from
    the same start, and the two fields agree element by element."""
    import torch
    from paper_2111_09859_amd import api
    kw = dict(eq="HJ", gamma="LAD", scheme="E6", eps=0.15)
    s0, s1 = G.star_grain(64, step=0), G.star_grain(64, step=4)
    prev, st, _, _ = oracle.solve(s0, omethod(oracle, tol=1e-10, max_iter=20000, **kw))
    assert st == 0
    n = 12
    ref, _, it, h = oracle.solve(s1, omethod(oracle, fixed=n, **kw), phi0=prev)
    dt = torch.float64 if prec == "fp64" else torch.float32
    phi = torch.as_tensor(prev, dtype=dt, device=solver.device).contiguous()
    srv = api.Server(solver, budget_bytes=256 << 20, max_slots=4)
    try:
        p = solver.prepare(s1, "E6", prec)
        m = gmethod(tol=0.0, max_iter=n, precision=prec, **kw)
        m.warm_start = 1
        rid = srv.submit(p, m, phi=phi, session=5, hist_cap=n)
        srv.wait(rid, 120.0)
        assert srv.poll(rid)["iters"] == n
        e = rel(phi.double().cpu().numpy(), ref)
        say(f"[served warm step {prec}] star64 step 4 from step 0: rel_linf={e:.2e}")
        assert e <= (FP64_TOL if prec == "fp64" else FP32_TOL)
        if prec == "fp64":
            hist = np.array(srv.history(rid, n)).reshape(-1, 2)
            assert np.allclose(hist[:, 0], h[:, 0], rtol=1e-8, atol=1e-14)
    finally:
        srv.close()


def test_served_unchanged_set_rounds_vs_oracle(solver, oracle):
    """Three grids served together for 80 iterations: five rounds of 16
    with the same set, the last four replaying the graph the server
    captures for an unchanged set (the round's states read back between
    replays); each field against the oracle after the same iterations
    (FP64, linear Gamma so that the 80 iterations stay comparable)."""
    from paper_2111_09859_amd import api, _lib as L
    cases = [
        ("channel65x33_E6_linear", lambda: G.channel(65, 33), dict(eq="HJ", scheme="E6", eps=0.1)),
        ("duct17x17x12_C6_linear", lambda: G.duct(17, nx=12), dict(eq="HJ", scheme="C6")),
        ("star64_E6_linear_mask", lambda: G.star_grain(64), dict(eq="HJ", scheme="E6", eps=0.15)),
    ]
    n = 80
    srv = api.Server(solver, budget_bytes=256 << 20, max_slots=8)
    try:
        ids, specs = [], []
        for name, build, kw in cases:
            spec = build()
            specs.append(spec)
            p = solver.prepare(spec, kw["scheme"], "fp64")
            ids.append(srv.submit(p, gmethod(tol=0.0, max_iter=n, precision="fp64", **kw),
                                  hist_cap=n))
        for rid, spec, (name, _, kw) in zip(ids, specs, cases):
            st = srv.wait(rid, 120.0)
            assert st == L.WD_NOT_CONVERGED and srv.poll(rid)["iters"] == n, (name, st)
            ref, _, it, h = oracle.solve(spec, omethod(oracle, fixed=n, **kw))
            e = rel(srv.result(rid).double().cpu().numpy(), ref)
            say(f"[served unchanged set fp64] {name}: rel_linf={e:.2e}")
            assert e <= FP64_TOL, name
            hist = np.array(srv.history(rid, n)).reshape(-1, 2)
            assert np.allclose(hist[:, 0], h[:, 0], rtol=1e-8, atol=1e-14), name
    finally:
        srv.close()
