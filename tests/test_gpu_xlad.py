"""GPU parity of the LAD diffusivity of uniform Cartesian grids formed in
two tile passes (Eq. Gamma_form2 with the smoothing reading): the sensor
C |sum_l d4_l phi^n / h_l| over x-y tiles marched along z, then the
nine-point truncated Gaussian along x, y (in LDS) and z (a register queue
over clamped or wrapped planes).

Each case runs with the tile passes (the default) and with the per-direction
line passes, and once on the FP64 oracle, at equal iterations: FP64
relative L-inf <= 1e-12 against the oracle (with the change history) and
between the two GPU paths; FP32 <= 1e-5.  LAD runs stop after a few
iterations: while the front moves the sensor amplifies rounding-order
differences between any two summation orders.  The grids cover both
non-periodic ends in y and z (the clamped fourth-difference centre and
Gaussian ends), periodic x and z (wrapped tiles and queue), 2D grids, a
solid mask, and the shortest lines the library takes (8 points: a periodic
line then wraps within the Gaussian's reach on both sides).
"""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

from test_gpu_parity import FP32_TOL, FP64_TOL, gpu_fixed, oracle_fixed, rel, say
from test_gpu_xstage import slab

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
    L.wd_ctx_set_lad_tiles(solver.ctx, True)
    tiles, out = gpu_fixed(solver, spec, n, precision=precision, **kw)
    L.wd_ctx_set_lad_tiles(solver.ctx, False)
    try:
        lines, _ = gpu_fixed(solver, spec, n, precision=precision, **kw)
    finally:
        L.wd_ctx_set_lad_tiles(solver.ctx, True)
    return tiles, lines, out


LAD = dict(eq="HJ", gamma="LAD", alpha_f=0.48)

CASES = [
    ("duct64x40x40_C6", lambda: G.duct(40, nx=64), dict(LAD, scheme="C6"), 4),
    # the benchmarked duct's tiles and z chunks, at a quarter of its x
    ("duct64x256x256_C6", lambda: G.duct(256, nx=64), dict(LAD, scheme="C6"), 3),
    ("duct64x40x40_E6", lambda: G.duct(40, nx=64), dict(LAD, scheme="E6"), 4),
    ("slab64x40x24_C6", slab, dict(LAD, scheme="C6"), 4),
    ("duct40x33x33_E4", lambda: G.duct(33, nx=40), dict(LAD, scheme="E4"), 4),
    ("duct12x17x17_C6", lambda: G.duct(17, nx=12), dict(LAD, scheme="C6"), 4),
    ("duct8x12x12_E2", lambda: G.duct(12, nx=8), dict(LAD, scheme="E2"), 4),
    ("slab8x9x8_E2", lambda: slab(8, 9, 8), dict(LAD, scheme="E2"), 4),
    ("channel129x65_C6", lambda: G.channel(129, 65), dict(LAD, scheme="C6"), 6),
    ("box100_E6", lambda: G.box2d(100), dict(LAD, scheme="E6"), 4),
    ("star96_E6_mask", lambda: G.star_grain(96), dict(LAD, scheme="E6", eps=0.15), 4),
]


@pytest.mark.parametrize("name,mk,kw,n", CASES, ids=[c[0] for c in CASES])
def test_lad_tiles_fp64_vs_oracle(solver, oracle, name, mk, kw, n):
    spec = mk()
    say(f"[lad tiles fp64] {name} {spec.n[:spec.ndim]} iters={n}")
    tiles, lines, out = run_both(solver, spec, n, "fp64", kw)
    ref, h = oracle_fixed(oracle, spec, n, **kw)
    e1, e2, e12 = rel(tiles, ref), rel(lines, ref), rel(tiles, lines)
    say(f"  tiles vs oracle {e1:.2e}, line passes vs oracle {e2:.2e}, between {e12:.2e}")
    assert e1 <= FP64_TOL
    assert e12 <= FP64_TOL
    assert np.allclose(out["hist"][:, 0], h[:, 0], rtol=1e-8, atol=1e-14)


FP32_CASES = [c for c in CASES if c[0] in ("duct64x40x40_C6", "duct64x256x256_C6", "slab64x40x24_C6",
                                           "channel129x65_C6", "star96_E6_mask")]


@pytest.mark.parametrize("name,mk,kw,n", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_lad_tiles_fp32_vs_oracle(solver, oracle, name, mk, kw, n):
    spec = mk()
    say(f"[lad tiles fp32] {name}")
    tiles, lines, _ = run_both(solver, spec, n, "fp32", kw)
    ref, _ = oracle_fixed(oracle, spec, n, **kw)
    e1 = rel(tiles, ref)
    say(f"  tiles vs oracle {e1:.2e}, line passes vs oracle {rel(lines, ref):.2e}")
    assert e1 <= FP32_TOL


def test_lad_tiles_duct_converged(solver, oracle):
    """The 40 x 33 x 33 duct, C6 LAD to max change 1e-10 in FP64: the GPU
    (tile LAD passes) stops at the oracle's iteration with its field."""
    from test_gpu_parity import gmethod, omethod
    spec = G.duct(33, nx=40)
    kw = dict(LAD, scheme="C6")
    prep = solver.prepare(spec, "C6", "fp64")
    out = solver.solve(prep, gmethod(tol=1e-10, max_iter=20000, **kw))
    phi = out["phi"].double().cpu().numpy()
    ref, st, it, _ = oracle.solve(spec, omethod(oracle, tol=1e-10, max_iter=20000, **kw))
    say(f"[lad tiles converged] duct 40x33x33: gpu {out['iters']} iters, oracle {it}, "
        f"rel {rel(phi, ref):.2e}")
    assert out["status"] == 0 and st == 0
    assert out["iters"] == it
    assert rel(phi, ref) <= 1e-9
