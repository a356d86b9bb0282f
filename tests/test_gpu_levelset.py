"""GPU parity of the level-set burnback (Sec. 5.5, Eq. levelset read with a
zero right-hand side) against the FP64 oracle: the RK4 march with the
upwind switch of Eqs. UW3-UW5 and zero-gradient faces, the iso-line
lengths, the signed-distance combination, and the star-grain pipeline
(two wall-distance solves, signed distance, march, burning perimeter).

FP64 fields: relative L-inf <= 1e-12 after equal steps; FP32 <= 1e-5
against the oracle run from the same FP32 start values.  Lengths: the GPU
and the oracle sum the same FP64 cell lengths in different orders, 1e-12.
"""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

from test_gpu_parity import FP32_TOL, FP64_TOL, gmethod, omethod, rel, say

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


def star_front(spec):
    """A six-lobed port front, phi = r - 0.3 (1 + 0.3 cos 6 theta) (positive
    in the solid), on a `square` grid."""
    X, Y = G.square_xy(spec)
    return np.hypot(X, Y) - 0.3 * (1 + 0.3 * np.cos(6 * np.arctan2(Y, X)))


CASES = [
    # name, grid, start field, speed, steps
    ("square65_star", lambda: G.square(65, 1.0), star_front, 0.3, 25),
    ("square100_star_ragged", lambda: G.square(100, 1.0), star_front, 0.3, 17),
    # two lane blocks along x with a ragged last one, rows not a multiple
    # of the rows a thread walks; and the same with x periodic
    ("square301_star_ragged", lambda: G.square(301, 1.0), star_front, 0.3, 12),
    ("channel300x37_periodic_x", lambda: G.channel(300, 37),
     lambda s: np.fromfunction(lambda j, i: j / 36 - 0.5 + 0.1 * np.sin(2 * np.pi * i / 300),
                               s.shape), 0.3, 15),
    # 3D with no periodic face and ragged rows; 3D with two lane blocks
    ("cube19_sphere", lambda: G.bouncing_cube(19, 0.3),
     lambda s: np.fromfunction(lambda k, j, i: np.sqrt((i / 18 - 0.5) ** 2 + (j / 18 - 0.5) ** 2
                                                       + (k / 18 - 0.45) ** 2) - 0.3, s.shape),
     0.3, 10),
    ("duct9x9x300_periodic_x", lambda: G.duct(9, nx=300),
     lambda s: np.fromfunction(lambda k, j, i: np.hypot(j / 8 - 0.5, k / 8 - 0.5) - 0.25
                               + 0.05 * np.sin(2 * np.pi * i / 300), s.shape), 0.3, 8),
    ("duct17x17x12_periodic_x", lambda: G.duct(17, nx=12),
     lambda s: np.fromfunction(lambda k, j, i: np.hypot(j / 16 - 0.5, k / 16 - 0.45) - 0.2
                               + 0.05 * np.sin(2 * np.pi * i / 12), s.shape), 0.3, 20),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,build,start,speed,nsteps", CASES, ids=[c[0] for c in CASES])
def test_levelset_advance_matches_oracle(solver, oracle, precision, name, build, start, speed,
                                         nsteps):
    import torch
    spec = build()
    phi0 = np.ascontiguousarray(start(spec), dtype=np.float64)
    dt = 0.5 * min(spec.h[: spec.ndim]) / speed
    dtype = torch.float64 if precision == "fp64" else torch.float32
    phi0 = phi0.astype(np.float32).astype(np.float64) if precision == "fp32" else phi0
    say(f"[levelset {precision}] {name} shape={spec.shape} steps={nsteps}")
    prep = solver.prepare(spec, "UW", precision)
    phi = torch.as_tensor(phi0, dtype=dtype, device=solver.device).contiguous()
    solver.levelset_advance(prep, phi, speed, dt, nsteps)
    g = phi.double().cpu().numpy()
    o = oracle.levelset_advance(spec, phi0, speed, dt, nsteps)
    e = rel(g, o)
    say(f"   rel_linf vs oracle={e:.3e}")
    assert e <= (FP64_TOL if precision == "fp64" else FP32_TOL)
    if spec.ndim == 2 and spec.bc[0][0] != G.PERIODIC:
        levels = [0.0, 0.1, -0.2]
        lg = solver.level_lengths(prep, phi, levels)
        lo = [oracle.level_length(spec, g, v) for v in levels]
        say(f"   lengths gpu={np.round(lg, 6)} oracle={np.round(lo, 6)}")
        for a, b in zip(lg, lo):
            assert abs(a - b) <= 1e-12 * max(abs(b), 1.0)


def test_levelset_zero_steps_and_bad_grid(solver):
    import torch
    from paper_2111_09859_amd import _lib as L
    spec = G.square(33, 1.0)
    prep = solver.prepare(spec, "UW", "fp64")
    phi = torch.as_tensor(star_front(spec), device=solver.device).contiguous()
    before = phi.clone()
    solver.levelset_advance(prep, phi, 0.3, 0.01, 0)
    assert torch.equal(phi, before)
    cyl = G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12)
    cprep = solver.prepare(cyl, "UW", "fp64")
    cphi = torch.zeros(cyl.shape, dtype=torch.float64, device=solver.device)
    with pytest.raises(L.WDError):
        solver.levelset_advance(cprep, cphi, 0.3, 0.01, 1)
    with pytest.raises(L.WDError):
        solver.level_lengths(prep, phi, [0.0] * 9)


def test_signed_distance_entry(solver, oracle):
    import torch
    rng = np.random.default_rng(5)
    solid = (rng.random((40, 37)) < 0.4).astype(np.uint8)
    ds, dg = rng.random((40, 37)), rng.random((40, 37))
    t = lambda a: torch.as_tensor(a, device=solver.device).contiguous()
    out = solver.signed_distance(t(solid), t(ds), t(dg)).cpu().numpy()
    assert np.array_equal(out, oracle.signed_distance(solid, ds, dg))


def test_star_grain_burnback_pipeline(solver, oracle):
    """The burnback as the paper runs it, on a 64^2 star grain: E4 LAD
    pseudo-HJ distances on the gas side and on the propellant side
    (converged to 1e-10), the signed distance, 30 RK4 steps at F = 0.3 and
    the lengths of the levels 0, 0.05 and -0.02.  Both sides stop their
    solves by the same criterion, so the fields agree to about the
    tolerance."""
    import torch
    gas, sol = G.star_grain(64), G.star_grain_solid(64)
    kw = dict(eq="HJ", gamma="LAD", scheme="E4", alpha_f=0.48)
    dg_o, st1, _, _ = oracle.solve(gas, omethod(oracle, **kw))
    ds_o, st2, _, _ = oracle.solve(sol, omethod(oracle, **kw))
    assert st1 == 0 and st2 == 0
    phi_o = oracle.signed_distance(gas.mask, ds_o, dg_o)
    F, dt, n = 0.3, 0.5 * gas.h[0] / 0.3, 30
    phi_o = oracle.levelset_advance(gas, phi_o, F, dt, n)
    levels = [0.0, 0.05, -0.02]
    lo = [oracle.level_length(gas, phi_o, v) for v in levels]
    m = gmethod(**kw)
    pg, ps_ = solver.prepare(gas, "E4", "fp64"), solver.prepare(sol, "E4", "fp64")
    dg = solver.solve(pg, m)["phi"]
    ds = solver.solve(ps_, m)["phi"]
    mask = torch.as_tensor(gas.mask, device=solver.device).contiguous()
    phi = solver.signed_distance(mask, ds, dg)
    solver.levelset_advance(pg, phi, F, dt, n)
    lg = solver.level_lengths(pg, phi, levels)
    e = rel(phi.cpu().numpy(), phi_o)
    say(f"[burnback] rel_linf={e:.3e} lengths gpu={np.round(lg, 6)} oracle={np.round(lo, 6)}")
    assert e <= 1e-8
    for a, b in zip(lg, lo):
        assert abs(a - b) <= 1e-7 * b
