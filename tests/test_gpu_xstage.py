"""GPU parity of the one-pass explicit RK stages (uniform Cartesian grids,
E2/E4/E6, Sec. 3.2): every point forms D_l phi and D_l D_l phi from its
neighbours, closure rows included, and finishes the stage in one pass.

Each case runs with the one-pass stages (the default for these grids) and
with the directional line passes, and once on the FP64 oracle, at equal
iterations: FP64 relative L-inf <= 1e-12 against the oracle (with the
change history) and between the two GPU paths; FP32 <= 1e-5.  Lines of
4R + 2 points are the shortest the one-pass stage takes (every point then
sits within 2R of an end, where the closure rows enter the composed
stencil); one point fewer falls back to the line passes.

The stage works on 64 x 16 tiles of x-y planes marched along z in chunks:
tiles whose U positions all take the interior row go to the fast variant,
the rest to the general one, and the z queue is refilled with closure rows
near non-periodic z ends.  The 64 x 40 x 40 duct has both kinds of tile
and five z chunks (refills at both ends); the slab is periodic in x and z
(the queue wraps); the 200^2 box has fast tiles with non-periodic x.
"""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

from test_gpu_parity import FP32_TOL, FP64_TOL, gpu_fixed, oracle_fixed, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_09859_amd import api
    s = api.Solver(0)
    yield s
    s.close()


def run_both(solver, spec, n, precision, kw):
    from paper_2111_09859_amd import _lib as L
    L.wd_ctx_set_explicit_onepass(solver.ctx, True)
    one, out = gpu_fixed(solver, spec, n, precision=precision, **kw)
    L.wd_ctx_set_explicit_onepass(solver.ctx, False)
    try:
        lines, _ = gpu_fixed(solver, spec, n, precision=precision, **kw)
    finally:
        L.wd_ctx_set_explicit_onepass(solver.ctx, True)
    return one, lines, out


def oracle_ref(O, spec, n, kw):
    ref, h = oracle_fixed(O, spec, n, **kw)
    if kw.get("eq") == "POISSON":
        ref = O.poisson_distance(spec, kw["scheme"], ref)
    return ref, h


def slab(nx=64, ny=40, nz=24):
    """Uniform box periodic in x and z, walls y = 0, 1 (exact min(y, 1-y))."""
    dy = 1.0 / (ny - 1)
    y = np.arange(ny) * dy
    ex = np.broadcast_to(np.minimum(y, 1.0 - y)[None, :, None], (nz, ny, nx)).copy()
    return G.GridSpec("slab", 3, (nx, ny, nz),
                      ((G.PERIODIC, G.PERIODIC), (G.WALL, G.WALL), (G.PERIODIC, G.PERIODIC)),
                      h=(1.0 / nx, dy, 1.0 / nz), exact=ex)


CASES = [
    ("duct64x40x40_E6_lad", lambda: G.duct(40, nx=64),
     dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 12),
    ("duct64x40x40_E4_linear_rk3", lambda: G.duct(40, nx=64),
     dict(eq="HJ", gamma="LINEAR", scheme="E4", rk="RK3", eps=0.1, alpha_f=0.48), 25),
    ("duct64x40x40_E2_poisson", lambda: G.duct(40, nx=64),
     dict(eq="POISSON", scheme="E2", alpha_f=0.48), 25),
    ("slab64x40x24_E6_lad", slab, dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 12),
    # 3D at the shortest z the pass takes for E6 (4R + 2 = 14 planes: the
    # queue's refills come within reach of both ends), non-periodic and
    # periodic
    ("duct64x14x14_E6_linear", lambda: G.duct(14, nx=64),
     dict(eq="HJ", gamma="LINEAR", scheme="E6", eps=0.1, alpha_f=0.48), 20),
    ("slab64x40x14_E6_linear", lambda: slab(64, 40, 14),
     dict(eq="HJ", gamma="LINEAR", scheme="E6", eps=0.1, alpha_f=0.48), 20),
    ("slab64x40x24_E4_eikonal", slab, dict(eq="EIKONAL", scheme="E4", alpha_f=0.48), 30),
    ("box200_E6_linear", lambda: G.box2d(200),
     dict(eq="HJ", gamma="LINEAR", scheme="E6", eps=0.1, alpha_f=0.48), 20),
    # LAD on this grid: a few iterations (the sensor amplifies rounding-order
    # differences between any two summation orders while the front moves)
    ("box200_E6_lad", lambda: G.box2d(200), dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 4),
    ("duct40x33x33_E4_lad", lambda: G.duct(33, nx=40),
     dict(eq="HJ", gamma="LAD", scheme="E4", alpha_f=0.48), 25),
    ("duct40x33x33_E6_poisson", lambda: G.duct(33, nx=40),
     dict(eq="POISSON", scheme="E6", alpha_f=0.48), 25),
    ("duct40x33x33_E2_linear_rk3", lambda: G.duct(33, nx=40),
     dict(eq="HJ", gamma="LINEAR", scheme="E2", rk="RK3", eps=0.1, alpha_f=0.48), 25),
    ("duct16x256x256_E6_lad", lambda: G.duct(256, nx=16),
     dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 4),
    # the benchmarked duct's lines (256 points along y and z, fast tiles,
    # the z march in chunks with both end zones) at a quarter of its x
    ("duct64x256x256_E6_lad", lambda: G.duct(256, nx=64),
     dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 4),
    ("box100_E6_lad", lambda: G.box2d(100), dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 12),
    ("box100_E4_eikonal", lambda: G.box2d(100), dict(eq="EIKONAL", scheme="E4", alpha_f=0.48), 40),
    ("star96_E6_lad_mask", lambda: G.star_grain(96),
     dict(eq="HJ", gamma="LAD", scheme="E6", eps=0.15, alpha_f=0.48), 12),
    ("channel129x65_E4_linear_rk3", lambda: G.channel(129, 65),
     dict(eq="HJ", gamma="LINEAR", scheme="E4", rk="RK3", eps=0.1, alpha_f=0.495), 60),
    # the shortest lines the one-pass stage takes: 4R + 2 points
    ("box14_E6_linear", lambda: G.box2d(14), dict(eq="HJ", gamma="LINEAR", scheme="E6"), 30),
    ("box10_E4_lad", lambda: G.box2d(10), dict(eq="HJ", gamma="LAD", scheme="E4"), 12),
    ("box8_E2_linear", lambda: G.box2d(8), dict(eq="HJ", gamma="LINEAR", scheme="E2"), 30),
    # one point short: the line passes serve it
    ("box13_E6_linear", lambda: G.box2d(13), dict(eq="HJ", gamma="LINEAR", scheme="E6"), 30),
]


@pytest.mark.parametrize("name,mk,kw,n", CASES, ids=[c[0] for c in CASES])
def test_onepass_fp64_vs_oracle(solver, oracle, name, mk, kw, n):
    spec = mk()
    say(f"[onepass fp64] {name} {spec.n[:spec.ndim]} iters={n}")
    one, lines, out = run_both(solver, spec, n, "fp64", kw)
    ref, h = oracle_ref(oracle, spec, n, kw)
    e1, e2, e12 = rel(one, ref), rel(lines, ref), rel(one, lines)
    say(f"  one-pass vs oracle {e1:.2e}, line passes vs oracle {e2:.2e}, between {e12:.2e}")
    assert e1 <= FP64_TOL
    assert e12 <= FP64_TOL
    assert np.allclose(out["hist"][:, 0], h[:, 0], rtol=1e-8, atol=1e-14)


FP32_CASES = [c for c in CASES if c[0] in ("duct40x33x33_E4_lad", "duct16x256x256_E6_lad",
                                           "duct64x256x256_E6_lad",
                                           "box100_E6_lad", "star96_E6_lad_mask",
                                           "duct40x33x33_E6_poisson", "duct64x40x40_E6_lad",
                                           "slab64x40x24_E6_lad", "box200_E6_lad")]


@pytest.mark.parametrize("name,mk,kw,n", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_onepass_fp32_vs_oracle(solver, oracle, name, mk, kw, n):
    spec = mk()
    say(f"[onepass fp32] {name}")
    one, lines, _ = run_both(solver, spec, n, "fp32", kw)
    ref, _ = oracle_ref(oracle, spec, n, kw)
    e1 = rel(one, ref)
    say(f"  one-pass vs oracle {e1:.2e}, line passes vs oracle {rel(lines, ref):.2e}")
    assert e1 <= FP32_TOL


def test_onepass_channel_converged(solver, oracle):
    """The 129 x 65 channel (standard HJ eps 0.1, E4, RK3, FP64 to 1e-10)
    through the one-pass stages stops at the oracle's iteration with its
    field."""
    from test_gpu_parity import gmethod, omethod
    spec = G.channel(129, 65)
    kw = dict(eq="HJ", gamma="LINEAR", scheme="E4", rk="RK3", eps=0.1, alpha_f=0.495)
    prep = solver.prepare(spec, "E4", "fp64")
    out = solver.solve(prep, gmethod(tol=1e-10, **kw))
    phi = out["phi"].double().cpu().numpy()
    ref, st, it, _ = oracle.solve(spec, omethod(oracle, tol=1e-10, **kw))
    say(f"[onepass converged] channel 129x65: gpu {out['iters']} iters, oracle {it}, "
        f"rel {rel(phi, ref):.2e}")
    assert out["status"] == 0 and st == 0
    assert out["iters"] == it
    assert rel(phi, ref) <= FP64_TOL
