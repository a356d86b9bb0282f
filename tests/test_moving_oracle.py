"""Moving walls (the unsteady cases of Sec. 5.5), CPU side: the closed-form
distances of the two moving-wall geometries against a brute-force search
over sampled wall surfaces, and the oracle's warm-started march (a
physical time step starts from the previous step's field) against what
the method fixes: a field already at the steady state stays there, the
steady state does not depend on the initial estimate, walls and solid
points are zero before the first pseudo-step, and the converged field
follows the moving wall to within the grid's resolution."""
import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

SIGMA = 0.5     # the annular bore needs a halved pseudo-step (sigma = 1 stalls)


def lad(O, tol=1e-6, fixed=0, max_iter=5000):
    return O.make_method(equation=O.HJ, gamma=O.GAMMA_LAD, eps=0.15, scheme="E4",
                         alpha_f=0.48, tol=tol, fixed_iters=fixed, max_iter=max_iter,
                         sigma=SIGMA)


def piston_small(h):
    return G.piston(16, 9, 13, h)


def test_piston_exact_is_brute_force(oracle):
    spec = piston_small(0.8)
    R, Rb, h = 0.25, 1.0, 0.8
    t = np.linspace(0, 2 * np.pi, 181)[:-1]
    zs = np.linspace(0, h, 161)
    rs = np.linspace(R, Rb, 151)
    walls = []
    for rad in (R, Rb):                    # rod and bore
        T, Z = np.meshgrid(t, zs)
        walls.append(np.stack([rad * np.cos(T), rad * np.sin(T), Z], -1).reshape(-1, 3))
    for zw in (0.0, h):                    # head and piston face
        T, Rr = np.meshgrid(t, rs)
        walls.append(np.stack([Rr * np.cos(T), Rr * np.sin(T), np.full_like(T, zw)],
                              -1).reshape(-1, 3))
    pts = G.cartesian_points(spec)
    d = oracle.brute_force(pts, np.concatenate(walls)).reshape(spec.shape)
    # sampling spacing on the bore: 2 pi / 180 ~ 0.035, so <= ~0.02 above exact
    assert np.all(d >= spec.exact - 1e-12)
    assert np.abs(d - spec.exact).max() < 0.02


def test_cube_exact_is_brute_force(oracle):
    spec = G.bouncing_cube(17, 0.3)
    lo, hi = spec.meta["lo"], spec.meta["hi"]
    s = np.linspace(0, 1, 81)
    A, B = np.meshgrid(s, s)
    walls = [np.stack([A.ravel(), B.ravel(), np.full(A.size, zw)], 1) for zw in (0.0, 1.0)]
    c = np.linspace(0, 1, 41)
    U, V = np.meshgrid(c, c)
    for ax in range(3):
        for side in (lo[ax], hi[ax]):
            face = np.empty((U.size, 3))
            o = [a for a in range(3) if a != ax]
            face[:, ax] = side
            face[:, o[0]] = lo[o[0]] + (hi[o[0]] - lo[o[0]]) * U.ravel()
            face[:, o[1]] = lo[o[1]] + (hi[o[1]] - lo[o[1]]) * V.ravel()
            walls.append(face)
    pts = G.cartesian_points(spec)
    d = oracle.brute_force(pts, np.concatenate(walls)).reshape(spec.shape)
    fluid = spec.mask == 0
    assert np.all(spec.exact[~fluid] == 0.0)
    assert np.abs(d - spec.exact)[fluid].max() < 0.01


def test_bounce_heights_energy():
    """Each rebound apex is `kept` times the previous one (energy mgh)."""
    z = G.bounce_heights(4000, 8.0, z0=0.6, kept=0.8)
    assert z[0] == 0.6 and z.min() >= 0.0
    peaks = [z[i] for i in range(1, len(z) - 1) if z[i] >= z[i - 1] and z[i] > z[i + 1]]
    assert len(peaks) >= 3
    for a, b in zip([0.6] + peaks[:-1], peaks[:3]):
        assert abs(b / a - 0.8) < 2e-3


def test_warm_start_at_steady_state_stays(oracle):
    spec = piston_small(1.0)
    phi, st, it, _ = oracle.solve(spec, lad(oracle, tol=1e-10, max_iter=20000))
    assert st == 0
    again, st2, it2, _ = oracle.solve(spec, lad(oracle, tol=1e-10), phi0=phi)
    assert st2 == 0 and it2 <= 2
    assert np.abs(again - phi).max() < 1e-10


def test_warm_start_reaches_cold_steady_state(oracle):
    """The next piston position from the previous field: the same steady
    state as a cold start (to the stopping tolerance's scale), in fewer
    pseudo-steps when the wall moved by a fraction of a cell."""
    h0, h1 = 1.0, 0.99
    prev, _, _, _ = oracle.solve(piston_small(h0), lad(oracle, tol=1e-10, max_iter=20000))
    spec = piston_small(h1)
    cold, st, it_c, _ = oracle.solve(spec, lad(oracle, tol=1e-10, max_iter=20000))
    warm, st2, it_w, _ = oracle.solve(spec, lad(oracle, tol=1e-10, max_iter=20000), phi0=prev)
    assert st == 0 and st2 == 0
    assert it_w < it_c
    assert np.abs(warm - cold).max() < 1e-7


def test_warm_start_zeroes_new_walls(oracle):
    """Walls and the cube's new position are zero before the first step."""
    old = G.bouncing_cube(17, 0.5)
    new = G.bouncing_cube(17, 0.25)
    phi0 = np.full(new.shape, 0.3)
    out, st, it, _ = oracle.solve(new, lad(oracle, fixed=1), phi0=phi0)
    assert it == 1
    assert np.all(out[new.mask == 1] == 0.0)
    assert np.all(out[0] == 0.0) and np.all(out[-1] == 0.0)
    moved = (old.mask == 1) & (new.mask == 0)
    assert moved.any() and np.all(out[moved] > 0.0)


@pytest.mark.parametrize("h", [1.4, 0.6])
def test_piston_converged_follows_wall(oracle, h):
    """Converged E4 LAD pseudo-HJ distance within half a cell (the larger
    spacing, 0.117 in z at h = 1.4, 0.094 in r at h = 0.6) of the exact
    field at every point (the error peaks on the ridges where two walls are
    equally near), and within a quarter cell on the mid-radius line near
    the head."""
    spec = piston_small(h)
    phi, st, it, _ = oracle.solve(spec, lad(oracle))
    assert st == 0
    cell = max(h / (spec.n[2] - 1), 0.75 / (spec.n[1] - 1))
    err = np.abs(phi - spec.exact)
    assert err.max() < 0.5 * cell
    k = np.arange(spec.n[2])
    near_head = k * h / (spec.n[2] - 1) < 0.3
    assert err[near_head, 4, :].max() < 0.25 * cell


@pytest.mark.parametrize("n,level,runaway", [(129, 0.3, True), (65, 0.3, False),
                                              (129, 0.1, False)])
def test_steep_warm_estimate_runs_away(oracle, n, level, runaway):
    """A warm estimate that jumps from the wall's zero to `level` within one
    cell: with a jump of 0.3 over 1/128 the central march undershoots below
    zero beside the wall, Gamma = max(0, eps phi) vanishes there and the
    point runs away (far below -0.1 of the field's maximum within 300
    pseudo-steps, the bound the moving-wall sequences restart at); half the
    jump per cell, or a third of it, recovers and stays non-negative."""
    spec = G.box2d(n)
    phi, st, it, hist = oracle.solve(spec, lad(oracle, fixed=300),
                                     phi0=np.full(spec.shape, level))
    assert it == 300
    if runaway:
        assert phi.min() < -0.1 * np.abs(phi).max()
        assert hist[-1, 0] > 10 * hist[100, 0]
    else:
        assert phi.min() >= 0.0
        assert hist[-1, 0] < hist[100, 0]
