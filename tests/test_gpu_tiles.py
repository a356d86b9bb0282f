"""GPU parity across the tile variants of the reduction-level line passes.

The same grid is solved with tile widths that put 1, 2, 4 and 8 points on
each thread (every compiled variant of the line passes, in both
precisions, with ragged last tiles), each result is compared element-wise
with the FP64 oracle after the same number of pseudo iterations, and the
variants are compared with each other.  The segmented passes, which
uniform Cartesian grids take by default, are switched off here so these
passes are the ones tested on every grid (test_gpu_seg.py covers the
segmented ones).
"""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

from test_gpu_parity import FP32_TOL, FP64_TOL, gmethod, omethod, rel, say

pytestmark = pytest.mark.gpu

# name, grid builder, method, iterations, tile widths per direction giving
# 1, 2, 4, 8 points per thread in every direction that can hold them
CASES = [
    ("channel65x33_C6_lad", lambda: G.channel(65, 33),
     dict(eq="HJ", gamma="LAD", scheme="C6"), 30,
     [(1, 4), (8, 31), (16, 62), (33, 65)]),
    ("cyl64x40_C6_lad_curv", lambda: G.cylinder(64, 40, rout=6.0, dr1=1e-2, ratio=1.12),
     dict(eq="HJ", gamma="LAD", curv=1, scheme="C6"), 30,
     [(1, 4), (9, 13), (17, 26), (40, 64)]),
    ("cyl64x40_C6_hj_walls", lambda: G.cylinder(64, 40, rout=6.0, dr1=1e-2, ratio=1.12,
                                                 far=G.WALL),
     dict(eq="HJ", scheme="C6", eps=0.2), 30,
     [(1, 4), (9, 13), (17, 26), (40, 64)]),
    ("cyl64x40_E6_poisson_neumann", lambda: G.cylinder(64, 40, rout=6.0, dr1=1e-2, ratio=1.12,
                                                       far=G.NEUMANN),
     dict(eq="POISSON", scheme="E6"), 20,
     [(1, 4), (9, 13), (17, 26), (40, 64)]),
    ("ell64x40_C4_eik", lambda: G.ellipse(64, 40, axis_ratio=2.0, ratio=1.12, rout=5.0, dr1=1e-2),
     dict(eq="EIKONAL", scheme="C4"), 30,
     [(1, 4), (9, 13), (17, 26), (40, 64)]),
    ("duct17x17x12_C6_lad", lambda: G.duct(17, nx=12),
     dict(eq="HJ", gamma="LAD", scheme="C6"), 20,
     [(1, 4, 4), (43, 12, 12), (86, 8, 8), (172, 12, 12)]),
    ("cyl64x40_UW_lad", lambda: G.cylinder(64, 40, rout=6.0, dr1=1e-2, ratio=1.12, far=G.NEUMANN),
     dict(eq="HJ", gamma="LAD", scheme="UW", filt=0), 30,
     [(1, 4), (9, 13), (17, 26), (40, 64)]),
    # Cartesian grids whose lines do not fill a tile row: ragged tiles of
    # odd widths, lines shorter than a workgroup, 3D with an explicit scheme
    ("duct33x33x40_E4_lad", lambda: G.duct(33, nx=40),
     dict(eq="HJ", gamma="LAD", scheme="E4"), 20,
     [(8, 8, 8), (3, 5, 7), (1, 2, 2), (43, 33, 33)]),
    ("box100_C6_hj", lambda: G.box2d(100),
     dict(eq="HJ", gamma="LINEAR", scheme="C6"), 20,
     [(8, 8), (6, 3), (1, 1), (40, 40)]),
]


def points_per_thread(spec, widths):
    out = []
    for l, w in enumerate(widths):
        pts = w * spec.n[l]
        np_ = 1
        while np_ < 8 and 512 * np_ < pts:
            np_ *= 2
        out.append(np_)
    return out


@pytest.fixture(scope="module")
def fresh_solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_09859_amd import _lib as L, api
    s = api.Solver(0)
    L.wd_ctx_set_segmented(s.ctx, False)
    yield s
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,build,kw,n_iter,configs", CASES, ids=[c[0] for c in CASES])
def test_tile_variants_match_oracle(fresh_solver, oracle, precision, name, build, kw, n_iter,
                                    configs):
    spec = build()
    o, _, it, _ = oracle.solve(spec, omethod(oracle, fixed=n_iter, **kw))
    assert it == n_iter
    if kw.get("eq") == "POISSON":
        o = oracle.poisson_distance(spec, kw["scheme"], o)
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    results = []
    for widths in configs:
        nps = points_per_thread(spec, widths)
        say(f"[tiles {precision}] {name} widths={widths} points/thread={nps}")
        prep = fresh_solver.prepare(spec, kw.get("scheme", "C6"), precision)
        fresh_solver.set_tiles(prep, widths)
        assert fresh_solver.tiles(prep) == list(widths)
        out = fresh_solver.solve(prep, gmethod(tol=0.0, max_iter=n_iter, precision=precision, **kw))
        assert out["iters"] == n_iter
        g = out["phi"].double().cpu().numpy()
        e = rel(g, o)
        say(f"   rel_linf vs oracle={e:.3e}")
        assert e <= tol
        results.append(g)
    # every variant does the same arithmetic per point
    for g in results[1:]:
        d = rel(g, results[0])
        say(f"   rel_linf vs first variant={d:.3e}")
        assert d <= (1e-13 if precision == "fp64" else 1e-6)


def test_upwind_with_curvature_is_rejected(fresh_solver):
    from paper_2111_09859_amd import _lib as L
    spec = G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12)
    prep = fresh_solver.prepare(spec, "UW", "fp64")
    with pytest.raises(L.WDError):
        fresh_solver.solve(prep, gmethod(eq="HJ", curv=1, scheme="UW", filt=0, tol=0.0,
                                         max_iter=5))


def test_tile_widths_out_of_range_are_rejected(fresh_solver):
    from paper_2111_09859_amd import _lib as L
    spec = G.channel(65, 33)
    prep = fresh_solver.prepare(spec, "C6", "fp64")
    before = fresh_solver.tiles(prep)
    for bad in [(0, 4), (34, 4), (1, 66), (1, 200)]:
        with pytest.raises(L.WDError):
            fresh_solver.set_tiles(prep, bad)
    assert fresh_solver.tiles(prep) == before
