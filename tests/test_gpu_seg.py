"""GPU parity of the segmented line passes (uniform Cartesian grids).

Every case runs on the GPU twice through the C ABI -- segmented passes
(the default) and the reduction-level line passes -- and once on the FP64
CPU oracle, at an equal number of pseudo iterations.  Bars: FP64 relative
L-inf <= 1e-12 against the oracle and between the two GPU paths; FP32 <=
1e-5 against the oracle.  LAD cases stop after a few iterations: while the
front moves, the LAD sensor amplifies rounding-level differences between
any two summation orders (the oracle against itself included), so later
iterates of different but correct implementations drift apart.

The shapes reach the segment geometries of the 256^3 duct's lines (256
points along y and z: 8 segments of 32; along x: 16 of 16) on grids the
oracle finishes in seconds, plus ragged segment lengths, periodic and
walled lines, extrapolated faces, solid masks and every scheme.
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


def walled(bc, n=65):
    """n x n uniform grid on [0,1]^2 with the given face kinds."""
    h = 1.0 / (n - 1)
    return G.GridSpec("walled", 2, (n, n, 1), (bc[0], bc[1], (G.WALL, G.WALL)), h=(h, h, 1.0))


def run_both(solver, spec, n, precision, kw):
    from paper_2111_09859_amd import _lib as L
    L.wd_ctx_set_segmented(solver.ctx, True)
    seg, out = gpu_fixed(solver, spec, n, precision=precision, **kw)
    L.wd_ctx_set_segmented(solver.ctx, False)
    try:
        old, _ = gpu_fixed(solver, spec, n, precision=precision, **kw)
    finally:
        L.wd_ctx_set_segmented(solver.ctx, True)
    return seg, old, out


def oracle_ref(O, spec, n, kw):
    """The oracle's field after n iterations (Poisson: converted to the
    distance of Eq. Poiss2, as the library returns it) and its history."""
    ref, h = oracle_fixed(O, spec, n, **kw)
    if kw.get("eq") == "POISSON":
        ref = O.poisson_distance(spec, kw["scheme"], ref)
    return ref, h


CASES = [
    # the 256-point y and z lines of the 256^3 duct (8 segments of 32)
    ("duct16x256x256_C6_lad", lambda: G.duct(256, nx=16),
     dict(eq="HJ", gamma="LAD", scheme="C6", alpha_f=0.48), 4),
    ("duct16x256x256_C6_poisson", lambda: G.duct(256, nx=16),
     dict(eq="POISSON", scheme="C6", alpha_f=0.48), 8),
    # the 256-point periodic x lines (16 segments of 16)
    ("duct256x16x16_C6_lad", lambda: G.duct(16, nx=256),
     dict(eq="HJ", gamma="LAD", scheme="C6", alpha_f=0.48), 20),
    ("duct256x16x16_C6_poisson", lambda: G.duct(16, nx=256),
     dict(eq="POISSON", scheme="C6", alpha_f=0.48), 20),
    # ragged segments (40 = 2 x 20 periodic, 33 = 17 + 16)
    ("duct40x33x33_C6_lad", lambda: G.duct(33, nx=40),
     dict(eq="HJ", gamma="LAD", scheme="C6", alpha_f=0.48), 25),
    ("duct40x33x33_E4_linear", lambda: G.duct(33, nx=40),
     dict(eq="HJ", gamma="LINEAR", scheme="E4", alpha_f=0.48), 25),
    ("duct40x33x33_E6_poisson", lambda: G.duct(33, nx=40),
     dict(eq="POISSON", scheme="E6", alpha_f=0.48), 25),
    ("duct40x33x33_C4_eikonal", lambda: G.duct(33, nx=40),
     dict(eq="EIKONAL", scheme="C4", alpha_f=0.48), 25),
    ("duct40x33x33_E2_lad_rk3", lambda: G.duct(33, nx=40),
     dict(eq="HJ", gamma="LAD", scheme="E2", rk="RK3", alpha_f=0.48), 25),
    # 2D: four walls, 100 = 4 x 25
    ("box100_C6_lad", lambda: G.box2d(100), dict(eq="HJ", gamma="LAD", scheme="C6", alpha_f=0.48), 12),
    ("box100_C6_linear", lambda: G.box2d(100), dict(eq="HJ", gamma="LINEAR", scheme="C6",
                                                    alpha_f=0.48), 40),
    ("box100_C4_poisson_nofilter", lambda: G.box2d(100),
     dict(eq="POISSON", scheme="C4", filt=0), 40),
    # an extrapolated (zero-gradient) face normal to the last direction, fused into its passes
    ("wall65_E6_lad_face_y", lambda: walled(((G.WALL, G.WALL), (G.WALL, G.NEUMANN))),
     dict(eq="HJ", gamma="LAD", scheme="E6", alpha_f=0.48), 12),
    # faces along x as well: applied by the face passes after the stage
    ("wall65_C6_linear_faces_xy", lambda: walled(((G.NEUMANN, G.OUTFLOW), (G.WALL, G.NEUMANN))),
     dict(eq="HJ", gamma="LINEAR", scheme="C6", alpha_f=0.48), 40),
    # solid mask (star-shaped port)
    ("star96_E6_lad_mask", lambda: G.star_grain(96), dict(eq="HJ", gamma="LAD", scheme="E6",
                                                          eps=0.15, alpha_f=0.48), 12),
    # the 129 x 65 channel (x periodic, 129 = 8 x 17 - 7; 65 = 4 x 17 - 3), RK3
    ("channel129x65_E4_linear_rk3", lambda: G.channel(129, 65),
     dict(eq="HJ", gamma="LINEAR", scheme="E4", rk="RK3", eps=0.1, alpha_f=0.495), 60),
    ("channel129x65_C6_lad", lambda: G.channel(129, 65),
     dict(eq="HJ", gamma="LAD", scheme="C6", alpha_f=0.495), 12),
]


@pytest.mark.parametrize("name,mk,kw,n", CASES, ids=[c[0] for c in CASES])
def test_segmented_fp64_vs_oracle(solver, oracle, name, mk, kw, n):
    spec = mk()
    say(f"[seg fp64] {name} {spec.n[:spec.ndim]} iters={n}")
    seg, old, out = run_both(solver, spec, n, "fp64", kw)
    ref, h = oracle_ref(oracle, spec, n, kw)
    e_seg, e_old, e_so = rel(seg, ref), rel(old, ref), rel(seg, old)
    say(f"  seg vs oracle {e_seg:.2e}, reduction-level vs oracle {e_old:.2e}, seg vs it {e_so:.2e}")
    assert e_seg <= FP64_TOL
    assert e_so <= FP64_TOL
    # FP64 residual history (max change per iteration) against the oracle's
    assert np.allclose(out["hist"][:, 0], h[:, 0], rtol=1e-8, atol=1e-14)


FP32_CASES = [c for c in CASES if c[0] in ("duct16x256x256_C6_lad", "duct256x16x16_C6_lad",
                                           "duct40x33x33_C6_lad", "box100_C6_lad",
                                           "wall65_E6_lad_face_y", "star96_E6_lad_mask",
                                           "duct16x256x256_C6_poisson")]


@pytest.mark.parametrize("name,mk,kw,n", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_segmented_fp32_vs_oracle(solver, oracle, name, mk, kw, n):
    spec = mk()
    say(f"[seg fp32] {name} {spec.n[:spec.ndim]} iters={n}")
    seg, old, _ = run_both(solver, spec, n, "fp32", kw)
    ref, _ = oracle_ref(oracle, spec, n, kw)
    e_seg, e_old = rel(seg, ref), rel(old, ref)
    say(f"  seg vs oracle {e_seg:.2e}, reduction-level vs oracle {e_old:.2e}")
    assert e_seg <= FP32_TOL


def test_segmented_converged_channel(solver, oracle):
    """The 129 x 65 channel (standard HJ eps 0.1, E4, RK3, FP64 to 1e-10)
    through the segmented passes stops at the oracle's iteration and matches
    its field."""
    from test_gpu_parity import gmethod, omethod
    spec = G.channel(129, 65)
    kw = dict(eq="HJ", gamma="LINEAR", scheme="E4", rk="RK3", eps=0.1, alpha_f=0.495)
    prep = solver.prepare(spec, "E4", "fp64")
    out = solver.solve(prep, gmethod(tol=1e-10, **kw))
    phi = out["phi"].double().cpu().numpy()
    ref, st, it, h = oracle.solve(spec, omethod(oracle, tol=1e-10, **kw))
    say(f"[seg converged] channel 129x65: gpu {out['iters']} iters, oracle {it}, "
        f"rel {rel(phi, ref):.2e}")
    assert out["status"] == 0 and st == 0
    assert out["iters"] == it
    assert rel(phi, ref) <= FP64_TOL
