"""Pins of the FP64 CPU oracle against facts the paper and the mathematics
fix independently of the oracle's own code: Fourier symbols of the central
schemes and of the implicit filter, polynomial exactness, the exact Poisson
channel solution, the metric identities of an O-grid, the standard-HJ
channel ODE under grid refinement, RK amplification factors, closed-form
distances and brute-force nearest-wall search.

A plausible slip in the oracle (a coefficient, a sign, an index, a
transposed metric) breaks at least one of these."""
import math

import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

SCHEMES = ["E2", "E4", "E6", "C4", "C6"]


def symbol(scheme, w):
    """Modified wavenumber k'(w) of each first-derivative scheme (Sec. 3.2
    interior relation with its standard coefficients)."""
    s = np.sin
    return {"E2": s(w),
            "E4": 4 / 3 * s(w) - 1 / 6 * s(2 * w),
            "E6": 1.5 * s(w) - 0.3 * s(2 * w) + s(3 * w) / 30,
            "C4": 1.5 * s(w) / (1 + 0.5 * np.cos(w)),
            "C6": (14 / 9 * s(w) + 1 / 18 * s(2 * w)) / (1 + 2 / 3 * np.cos(w))}[scheme]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("n", [32, 129])
def test_derivative_fourier_symbol(oracle, scheme, n):
    j = np.arange(n)
    for k in (1, 5, n // 3):
        w = 2 * np.pi * k / n
        d = oracle.deriv_line(np.sin(w * j + 0.3), scheme, periodic=True)
        assert np.abs(d - symbol(scheme, w) * np.cos(w * j + 0.3)).max() < 1e-13


@pytest.mark.parametrize("scheme,deg", [("E2", 2), ("E4", 4), ("E6", 4), ("C4", 4), ("C6", 4)])
def test_derivative_polynomial_exactness(oracle, scheme, deg):
    n = 24
    x = np.arange(n, dtype=float)
    for k in range(deg + 1):
        d = oracle.deriv_line((x / n) ** k, scheme)
        exact = k * (x / n) ** max(k - 1, 0) / n
        assert np.abs(d - exact).max() < 1e-12, (scheme, k)
    # one degree higher is not reproduced (the closures have that order)
    d = oracle.deriv_line((x / n) ** (deg + 1), scheme)
    assert np.abs(d - (deg + 1) * (x / n) ** deg / n).max() > 1e-9


@pytest.mark.parametrize("scheme,deg", [("E4", 4), ("E6", 6)])
def test_explicit_interior_order(oracle, scheme, deg):
    n = 40
    x = np.arange(n, dtype=float) / n
    d = oracle.deriv_line(x ** deg, scheme)
    exact = deg * x ** (deg - 1) / n
    r = {"E4": 2, "E6": 3}[scheme]
    assert np.abs(d[r:-r] - exact[r:-r]).max() < 1e-12


def test_periodic_seam_jump(oracle):
    n = 20
    x = np.arange(n) * 0.1
    for s in SCHEMES:
        d = oracle.deriv_line(x, s, periodic=True, jump=n * 0.1)
        assert np.abs(d - 0.1).max() < 1e-13


def transfer(alpha, N, w):
    return 1 - (1 - 2 * alpha) * np.sin(w / 2) ** (2 * N) / (1 + 2 * alpha * np.cos(w))


@pytest.mark.parametrize("alpha", [0.48, 0.49, 0.495])
def test_filter_transfer_function(oracle, alpha):
    n = 64
    j = np.arange(n)
    for k in (1, 7, 20, 31):
        w = 2 * np.pi * k / n
        f = np.cos(w * j + 0.1)
        out = oracle.filter_line(f, alpha, periodic=True)
        assert np.abs(out - transfer(alpha, 5, w) * f).max() < 1e-12
    pi_mode = (-1.0) ** j
    assert np.abs(oracle.filter_line(pi_mode, alpha, periodic=True)).max() < 1e-12
    const = np.full(n, 3.25)
    assert np.abs(oracle.filter_line(const, alpha, periodic=True) - const).max() < 1e-13


def test_filter_near_boundary_orders(oracle):
    """Rows at distance k from a wall apply the order-2k member: the residual
    of the left-hand side applied to (filtered - input) must equal the
    closed-form correction -(1-2a)(-1)^N delta^{2N} f / 4^N with N = min(k, 5)."""
    a = 0.49
    n = 30
    x = np.arange(n, dtype=float) / n
    rng = np.random.default_rng(3)
    f = np.sin(3 * x) + 0.2 * rng.standard_normal(n)
    out = oracle.filter_line(f, a, periodic=False)
    e = out - f
    assert e[0] == 0.0 and e[-1] == 0.0
    for i in range(1, n - 1):
        lhs = a * e[i - 1] + e[i] + a * e[i + 1]
        N = min(i, n - 1 - i, 5)
        coef = [math.comb(2 * N, N + t) * (-1) ** (N + t) for t in range(-N, N + 1)]
        d2n = sum(c * f[i + t] for c, t in zip(coef, range(-N, N + 1)))
        want = -(1 - 2 * a) * (-1) ** N * d2n / 4 ** N
        assert abs(lhs - want) < 1e-13, i


def test_filter_identity_and_linear(oracle):
    n = 25
    lin = 2.0 + 0.7 * np.arange(n)
    assert np.abs(oracle.filter_line(lin, 0.495, periodic=False) - lin).max() < 1e-12


def test_metrics_uniform_from_coordinates(oracle):
    spec = G.channel_curvilinear(24, 17)
    for s in SCHEMES:
        met = oracle.metrics(spec, s)
        dx, dy = 2.0 / 24, 1.0 / 16
        assert np.abs(met[0] - 1 / dx).max() < 1e-9
        assert np.abs(met[3] - 1 / dy).max() < 1e-9
        assert np.abs(met[1]).max() < 1e-9 and np.abs(met[2]).max() < 1e-9


@pytest.mark.parametrize("scheme", SCHEMES)
def test_ogrid_metric_identities(oracle, scheme):
    """On a uniform-theta O-grid, phi = r - R gives U = (cos, sin), |U| = 1,
    lap = 1/r and kappa = 1/(r (1 + eps0)) for ANY radial distribution."""
    spec = G.cylinder(48, 20, rout=6.0, dr1=2e-2, ratio=1.15)
    m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LINEAR, curvature=1,
                           eps0=1e-6, scheme=scheme)
    ev = oracle.evaluate(spec, m, spec.exact)
    r = spec.exact + 0.5
    assert np.abs(ev["g"] - 1).max() < 1e-12
    assert np.abs(ev["lap"] - 1 / r).max() < 1e-10
    assert np.abs(ev["kappa"] - 1 / (r * (1 + 1e-6))).max() < 1e-10


def test_ellipse_metric_identities(oracle):
    """Normal offsets of an ellipse: the exact distance rho_j has |grad| = 1
    up to the derivative truncation error (not exactly: the theta spacing of
    the wall is not uniform in arc length)."""
    spec = G.ellipse(128, 24, axis_ratio=2.0, ratio=1.1, rout=4.0, dr1=1e-2)
    m = oracle.make_method(equation=oracle.EIKONAL, scheme="C6")
    ev = oracle.evaluate(spec, m, spec.exact)
    assert np.abs(ev["g"] - 1).max() < 1e-3


def test_poisson_channel_exact(oracle):
    """phi' = y(1-y)/2 solves lap phi' = -1 exactly for every scheme, and
    Eq. Poiss2 with the minus sign turns it into min(y, 1-y)."""
    spec = G.channel(16, 17)
    y = np.arange(17) / 16.0
    phip = np.broadcast_to((y * (1 - y) / 2)[:, None], spec.shape).copy()
    for s in SCHEMES:
        m = oracle.make_method(equation=oracle.POISSON, scheme=s)
        ev = oracle.evaluate(spec, m, phip)
        assert np.abs(ev["R"][1:-1]).max() < 1e-11
        d = oracle.poisson_distance(spec, s, phip)
        assert np.abs(d - spec.exact).max() < 1e-12


def test_poisson_channel_march(oracle):
    spec = G.channel(12, 13)
    m = oracle.make_method(equation=oracle.POISSON, scheme="E4", filter=0, tol=1e-13)
    phi, st, it, h = oracle.solve(spec, m)
    y = np.arange(13) / 12.0
    assert st == 0
    assert np.abs(phi - (y * (1 - y) / 2)[:, None]).max() < 1e-11


@pytest.mark.parametrize("rk", [0, 1])
def test_rk_amplification(oracle, rk):
    """Poisson on a doubly periodic grid without filter: a Fourier mode of
    amplitude A obeys A' = P(z) A with z = -k'(w)^2 dt / h^2 and P the RK
    stability polynomial; the mean grows by exactly dt per step."""
    n0, n1, h = 16, 8, 0.1
    spec = G.GridSpec("periodic", 2, (n0, n1, 1),
                      ((G.PERIODIC, G.PERIODIC), (G.PERIODIC, G.PERIODIC), (0, 0)),
                      h=(h, h, 1.0))
    w = 2 * np.pi * 3 / n0
    x = np.arange(n0)
    phi0 = np.broadcast_to(0.5 + 0.1 * np.cos(w * x)[None, :], (n1, n0)).copy()
    m = oracle.make_method(equation=oracle.POISSON, scheme="C6", filter=0, rk=rk,
                           fixed_iters=1)
    out, st, it, hist = oracle.solve(spec, m, phi0=phi0)
    kp = 1.989
    dt = 1.0 / (kp * kp * 2 / h ** 2)
    z = -symbol("C6", w) ** 2 * dt / h ** 2
    P = 1 + z + z ** 2 / 2 + z ** 3 / 6 + (z ** 4 / 24 if rk == 1 else 0.0)
    want = 0.5 + dt + 0.1 * P * np.cos(w * x)
    assert np.abs(out - want[None, :]).max() < 1e-13


def test_neumann_bc_quadratic(oracle):
    """phi_b = (4 phi_1 - phi_2)/3 is exact for quadratics with zero normal
    derivative at the face."""
    n = 12
    spec = G.GridSpec("nb", 2, (n, n, 1),
                      ((G.PERIODIC, G.PERIODIC), (G.WALL, G.NEUMANN), (0, 0)),
                      h=(0.1, 0.1, 1.0))
    y = np.arange(n) * 0.1
    phi = np.broadcast_to(((y - y[-1]) ** 2 + 0.3)[:, None], (n, n)).copy()
    out = oracle.apply_bc(spec, phi)
    assert out[0].max() == 0.0
    assert np.abs(out[-1] - 0.3).max() < 1e-14


def _hj_ode(eps):
    """Continuum standard-HJ channel profile: (phi')^2 = 1 + eps phi phi'',
    phi(0) = 0, phi'(1/2) = 0 (shooting from the centre)."""
    from scipy.integrate import solve_ivp
    from scipy.optimize import brentq

    def run(pc, dense=False):
        ev = lambda y, u: u[0] - 1e-9
        ev.terminal = True
        s = solve_ivp(lambda y, u: [u[1], (u[1] ** 2 - 1) / (eps * u[0])], [0.5, 0.0],
                      [pc, 0.0], rtol=1e-12, atol=1e-14, events=ev, dense_output=dense,
                      method="LSODA")
        return s if dense else (s.t_events[0][0] if len(s.t_events[0]) else -1.0)

    pc = brentq(run, 0.3, 0.5, xtol=1e-14)
    return run(pc, True)


@pytest.mark.parametrize("scheme,rate", [("E4", 12.0), ("C6", 40.0)])
def test_channel_hj_converges_to_ode(oracle, scheme, rate):
    """Standard HJ (eps = 0.1) in the channel converges to the 1-D ODE
    solution under refinement; the converged field is x-independent and
    symmetric about y = 1/2."""
    sol = _hj_ode(0.1)
    errs = []
    for ny in (33, 65):
        spec = G.channel(16, ny)
        m = oracle.make_method(equation=oracle.HJ, eps=0.1, scheme=scheme, tol=1e-12)
        phi, st, it, h = oracle.solve(spec, m)
        assert st == 0
        y = np.arange(ny) / (ny - 1)
        yy = np.minimum(y, 1 - y)
        ref = np.array([sol.sol(v)[0] if v > sol.t_events[0][0] else 0.0 for v in yy])
        errs.append(np.abs(phi[:, 5] - ref).max())
        assert np.abs(phi - phi[:, :1]).max() < 1e-12
        assert np.abs(phi - phi[::-1]).max() < 1e-12
    assert errs[1] < errs[0] / rate
    assert errs[1] < 1e-3


def test_channel_hj_positive_bias(oracle):
    """Standard HJ under-predicts the distance away from the walls."""
    spec = G.channel(16, 33)
    m = oracle.make_method(equation=oracle.HJ, eps=0.1, scheme="E4", rk=oracle.RK3, tol=1e-10)
    phi, st, it, h = oracle.solve(spec, m)
    assert st == 0
    # the largest error sits at the centre line, where phi < d_true
    err = phi - spec.exact
    j = np.argmax(np.abs(err[:, 0]))
    assert j == 16 and err[j, 0] < -0.02
    assert np.abs(err).max() < 0.05


def test_cylinder_lad_curvature_fixed_point(oracle):
    """d = r - R is a discrete fixed point of the LAD + curvature HJ form on
    an O-grid with outflow far field; marching from zero converges to it."""
    spec = G.cylinder(64, 48, rout=5.0, dr1=1e-2, ratio=1.1)
    m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, curvature=1,
                           eps=0.2, scheme="C6", tol=1e-10, max_iter=5000)
    ev = oracle.evaluate(spec, m, spec.exact)
    assert np.abs(ev["R"][1:]).max() < 1e-8
    phi, st, it, h = oracle.solve(spec, m)
    assert st == 0
    assert np.abs(phi - spec.exact).max() < 1e-3
    assert np.abs(phi - phi[:, :1]).max() < 1e-8


def test_lad_gamma_vanishes_on_cubics(oracle):
    spec = G.channel(16, 17)
    y = np.arange(17) / 16.0
    phi = np.broadcast_to((0.3 * y + y ** 3)[:, None], spec.shape).copy()
    m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, eps=0.2)
    ev = oracle.evaluate(spec, m, phi)
    assert np.abs(ev["gamma"]).max() < 1e-12
    phi4 = np.broadcast_to(((np.arange(17.0)) ** 4 / 24)[:, None], spec.shape).copy()
    ev = oracle.evaluate(spec, m, phi4)
    inner = ev["gamma"][3:-3]
    lad = 0.1 * 16.0  # C |grad eta| delta^4 (x^4/24) = C / dy
    assert np.allclose(inner, np.minimum(0.2 * phi4[3:-3], lad), rtol=1e-12, atol=1e-12)


def test_brute_force_matches_closed_forms(oracle):
    spec = G.ellipse(32, 12, axis_ratio=2.0, ratio=1.2, rout=2.0, dr1=2e-2)
    pts = G.cartesian_points(spec)
    t = np.linspace(0, 2 * np.pi, 200000, endpoint=False)
    wall = np.stack([0.5 * np.cos(t), 0.25 * np.sin(t)], axis=1)
    d = oracle.brute_force(pts, wall).reshape(spec.shape)
    assert np.abs(d - spec.exact).max() < 1e-4
    ch = G.channel(9, 9)
    pts = G.cartesian_points(ch)
    xs = np.arange(-9, 18) * (2.0 / 9.0)
    wall = np.concatenate([np.stack([xs, 0 * xs], 1), np.stack([xs, 0 * xs + 1], 1)])
    d = oracle.brute_force(pts, wall).reshape(ch.shape)
    assert np.abs(d - ch.exact).max() < 1e-12


def test_ogrid_distance_order(oracle):
    """Ellipse O-grids: error of the converged LAD + curvature solution
    against the exact normal offset falls under refinement."""
    errs = []
    for nt, nr in ((32, 16), (64, 32)):
        spec = G.ellipse(nt, nr, axis_ratio=1.5, ratio=1.25 if nr == 16 else 1.12,
                         rout=3.0, dr1=1e-2)
        m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LINEAR, curvature=1,
                               eps=0.2, scheme="E4", tol=1e-9, max_iter=20000)
        phi, st, it, h = oracle.solve(spec, m)
        assert st == 0
        errs.append(np.abs(phi - spec.exact).max())
    assert errs[1] < errs[0]


def _perturbation_growth(oracle, spec, n, **kw):
    rng = np.random.default_rng(0)
    p1, _, _, _ = oracle.solve(spec, oracle.make_method(fixed_iters=1, **kw))
    p1b = p1 * (1 + 1e-15 * rng.standard_normal(p1.shape))
    a, _, _, _ = oracle.solve(spec, oracle.make_method(fixed_iters=n - 1, **kw), phi0=p1)
    b, _, _, _ = oracle.solve(spec, oracle.make_method(fixed_iters=n - 1, **kw), phi0=p1b)
    return np.abs(a - b).max() / np.abs(a).max()


def test_lad_reading_keeps_rounding_at_rounding_level(oracle):
    """The LAD reading (diffusivity from phi^n once per iteration, smoothed
    with the truncated Gaussian filter) leaves a 1e-15 perturbation at
    rounding level over 20 iterations; the unsmoothed per-stage variant
    amplifies it by many orders of magnitude (fourth-difference
    anti-diffusion through the sensor), which is why it is not the reading."""
    spec = G.channel(37, 29)
    kw = dict(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, scheme="E6", eps=0.2)
    assert _perturbation_growth(oracle, spec, 20, lad_raw=0, **kw) < 1e-12
    assert _perturbation_growth(oracle, spec, 20, lad_raw=1, **kw) > 1e-8


# ---------------------------------------------------------------------------
# Upwind baseline (Sec. 3.2.1, Eqs. UW1-UW5)

def test_uw_eikonal_channel_is_exact(oracle):
    """First-order upwind Eikonal in the channel: d = min(y, 1-y) is
    piecewise linear, its one-sided differences are exactly +-h, and the
    switch picks the steeper side on the ridge, so the march stops on the
    exact distance."""
    for ny in (29, 30):
        spec = G.channel(37, ny)
        m = oracle.make_method(equation=oracle.EIKONAL, scheme="UW", filter=0, tol=1e-12,
                               max_iter=20000)
        phi, st, it, h = oracle.solve(spec, m)
        assert st == 0
        assert np.abs(phi - spec.exact).max() < 1e-10


def test_uw_switch_pairing_as_printed_fails(oracle):
    """Eq. UW3 pairs n_{i-1} with F as printed; with that pairing a rising
    line takes its downwind difference and the channel march does not
    settle, while the pairing n_{i-1} B + n_{i+1} F (Godunov's choice:
    B rising, F falling, 0 at a minimum, the steeper side on a ridge)
    reaches the exact distance (test above)."""
    spec = G.channel(37, 29)
    m = oracle.make_method(equation=oracle.EIKONAL, scheme="UW", filter=0, tol=1e-12,
                           max_iter=3000, uw_printed=1)
    phi, st, it, h = oracle.solve(spec, m)
    assert st != 0
    assert not (np.abs(phi - spec.exact).max() < 1e-2)


def test_uw_hj_channel_first_order(oracle):
    """Standard HJ (eps 0.1) with the upwind term and the 2nd-order central
    Laplacian converges to the 1-D ODE profile at first order."""
    sol = _hj_ode(0.1)
    errs = []
    for ny in (33, 65, 129):
        spec = G.channel(16, ny)
        m = oracle.make_method(equation=oracle.HJ, eps=0.1, scheme="UW", filter=0, tol=1e-12,
                               max_iter=200000)
        phi, st, it, h = oracle.solve(spec, m)
        assert st == 0
        y = np.arange(ny) / (ny - 1)
        yy = np.minimum(y, 1 - y)
        ref = np.array([sol.sol(v)[0] if v > sol.t_events[0][0] else 0.0 for v in yy])
        errs.append(np.abs(phi[:, 5] - ref).max())
        assert np.abs(phi - phi[:, :1]).max() == 0.0
        assert np.abs(phi - phi[::-1]).max() < 1e-14
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4


def test_uw_eikonal_box_first_order(oracle):
    """Upwind Eikonal in the 2-D box: error against min(x, 1-x, y, 1-y)
    halves with the spacing (the kinks on the diagonals limit it to first
    order) and the field keeps the box's x <-> y symmetry exactly."""
    errs = []
    for n in (33, 65):
        spec = G.box2d(n)
        m = oracle.make_method(equation=oracle.EIKONAL, scheme="UW", filter=0, tol=1e-12,
                               max_iter=200000)
        phi, st, it, h = oracle.solve(spec, m)
        assert st == 0
        errs.append(np.abs(phi - spec.exact).max())
        assert np.abs(phi - phi.T).max() == 0.0
    assert 1.7 < errs[0] / errs[1] < 2.3


# ---- level-set burnback (Sec. 5.5) ------------------------------------

def test_level_length_line_and_circle(oracle):
    """Iso-line lengths: a straight level of a linear field is the domain
    width exactly; the level 0 of r - R is 2 pi R up to the O(h^2) chords."""
    spec = G.square(101, 1.0)
    X, Y = G.square_xy(spec)
    width = 2.0
    for c in (0.013, -0.4):
        assert abs(oracle.level_length(spec, Y - c, 0.0) - width) < 1e-12
    spec = G.square(401, 1.0)
    X, Y = G.square_xy(spec)
    r = np.hypot(X, Y)
    for R in (0.3, 0.71):
        L = oracle.level_length(spec, r - R, 0.0)
        assert abs(L / (2 * np.pi * R) - 1) < 2e-4
    # a saddle cell (corners +, -, +, - counter-clockwise): the sign of the
    # cell mean decides which corners the two segments cut off
    one = G.square(2, 0.5)
    v = np.array([[0.9, -1.1], [-1.1, 0.9]])        # rows y, columns x
    assert abs(oracle.level_length(one, v, 0.0) - 0.9 * np.sqrt(2)) < 1e-14
    assert abs(oracle.level_length(one, v + 0.2, 0.0) - np.sqrt(2) * 2 * 0.45) < 1e-14


def test_levelset_planar_front_moves_at_speed(oracle):
    """phi = x - c with speed F: the upwind differences of a linear field
    are exact, RK4 integrates the constant rate exactly, so away from the
    two faces' zero-gradient rows (whose influence spreads from the upwind
    face) phi = x - c - F t to rounding."""
    spec = G.square(81, 1.0)
    X, Y = G.square_xy(spec)
    F, h = 0.3, spec.h[0]
    dt = 0.5 * h / F
    n = 40
    phi = oracle.levelset_advance(spec, X - 0.1, F, dt, n)
    t = n * dt
    far = (X > -1.0 + F * t + 1.0) & (X < 0.9)
    assert np.abs(phi - (X - 0.1 - F * t))[far].max() < 1e-12


def test_levelset_expanding_circle(oracle):
    """A port of radius R0 (phi = r - R0, positive in the solid) burns
    outward: after time t its boundary is the circle R0 + F t; the level-0
    length follows 2 pi (R0 + F t) and phi near the front is r - R0 - F t
    to first order in h."""
    errs = []
    for n in (81, 161):
        spec = G.square(n, 1.0)
        X, Y = G.square_xy(spec)
        r = np.hypot(X, Y)
        F, h, R0 = 0.3, spec.h[0], 0.25
        dt = 0.5 * h / F
        nsteps = int(round(0.5 / dt))
        t = nsteps * dt
        phi = oracle.levelset_advance(spec, r - R0, F, dt, nsteps)
        Rt = R0 + F * t
        L = oracle.level_length(spec, phi, 0.0)
        assert abs(L / (2 * np.pi * Rt) - 1) < 0.02
        band = np.abs(r - Rt) < 0.15
        errs.append(np.abs(phi - (r - Rt))[band].max())
    assert errs[1] < 0.7 * errs[0]


def test_signed_distance_combination(oracle):
    solid = np.array([[0, 1], [1, 0]], dtype=np.uint8)
    ds = np.array([[9.0, 2.0], [3.0, 9.0]])
    dg = np.array([[4.0, 9.0], [9.0, 5.0]])
    assert np.array_equal(oracle.signed_distance(solid, ds, dg), np.array([[-4.0, 2.0], [3.0, -5.0]]))


# ---------------------------------------------------------------------------
# Pins of the LAD smoothing weights, the local time step, nu and the 3x3
# metric inverse.

def _gauss_weights_from_moments():
    """The symmetric nine-point smoothing stencil (b0, b1..b4 at offsets 0,
    +-1..+-4) fixed by five conditions: unit sum; second, fourth and sixth
    moments those of a Gaussian of variance 4/3 (4/3, 16/3, 320/9); and no
    response to the odd-even mode (omega = pi)."""
    A = np.zeros((5, 5))
    rhs = np.array([1.0, 4 / 3, 16 / 3, 320 / 9, 0.0])
    A[0] = [1, 2, 2, 2, 2]
    for r, p in enumerate((2, 4, 6), start=1):
        A[r] = [0] + [2 * k ** p for k in range(1, 5)]
    A[4] = [1] + [2 * (-1) ** k for k in range(1, 5)]
    return np.linalg.solve(A, rhs)


def test_lad_smoothing_weights_from_moments(oracle):
    """The oracle's smoothing of the LAD diffusivity (reading of Kawai &
    Lele's filter, Eq. Gamma_form2) returns, for a unit impulse on a
    periodic line, the weights the moment conditions fix; a swapped or
    mistyped weight that keeps the sum breaks a moment."""
    b = _gauss_weights_from_moments()
    n = 32
    e = np.zeros(n)
    e[10] = 1.0
    out = oracle.gauss_line(e, periodic=True)
    want = np.zeros(n)
    for k in range(-4, 5):
        want[10 + k] = b[abs(k)]
    assert np.abs(out - want).max() < 1e-15


@pytest.mark.parametrize("mode", [1, 3, 7, 16])
def test_lad_smoothing_transfer_function(oracle, mode):
    """On a periodic line a cosine mode comes back scaled by the stencil's
    transfer function b0 + 2 sum_k b_k cos(k w); the pi mode vanishes."""
    b = _gauss_weights_from_moments()
    n = 32
    w = 2 * np.pi * mode / n
    j = np.arange(n)
    T = b[0] + 2 * sum(b[k] * np.cos(k * w) for k in range(1, 5))
    out = oracle.gauss_line(np.cos(w * j + 0.3), periodic=True)
    assert np.abs(out - T * np.cos(w * j + 0.3)).max() < 1e-14
    if mode == 16:
        assert np.abs(out).max() < 1e-14


def test_lad_smoothing_clamped_ends(oracle):
    """Non-periodic lines: constants stay constant, the interior keeps
    linear functions (symmetric weights), and the ends see the end value
    repeated beyond the line (a ramp's first point moves up by
    sum_k k b_k over the missing side)."""
    b = _gauss_weights_from_moments()
    n = 20
    assert np.abs(oracle.gauss_line(np.full(n, 2.5)) - 2.5).max() < 1e-15
    ramp = np.arange(n, dtype=float)
    out = oracle.gauss_line(ramp)
    assert np.abs(out[4:-4] - ramp[4:-4]).max() < 1e-13
    assert abs(out[0] - sum(k * b[k] for k in range(1, 5))) < 1e-14


def test_lad_field_is_smoothed_sensor(oracle):
    """LAD diffusivity (Eq. Gamma_form2 with the smoothing reading) on a
    channel (x periodic, walls in y): phi = s j^4/24 + A cos(w i) has index
    fourth differences s along y (copied inward at the walls) and
    16 A sin^4(w/2) cos(w i) along x, so the sensor
    |grad eta| s + |grad xi| 16 A sin^4(w/2) cos(w i) stays positive, the
    smoothing scales the cosine by the transfer function and leaves the
    y-constant part alone."""
    b = _gauss_weights_from_moments()
    nx, ny = 32, 17
    spec = G.channel(nx, ny)
    dx, dy = 2.0 / nx, 1.0 / (ny - 1)
    s, A, mode = 2.0, 0.05, 3
    w = 2 * np.pi * mode / nx
    i = np.arange(nx)
    j = np.arange(ny)
    phi = s * (j ** 4 / 24.0)[:, None] + A * np.cos(w * i)[None, :]
    m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, eps=0.2, C_lad=0.1)
    lad = oracle.lad_field(spec, m, phi)
    T = b[0] + 2 * sum(b[k] * np.cos(k * w) for k in range(1, 5))
    amp = 16 * A * np.sin(w / 2) ** 4
    want = 0.1 * (s / dy + amp * T * np.cos(w * i) / dx)
    assert s / dy > amp / dx
    assert np.abs(lad - want[None, :]).max() < 1e-10 * np.abs(want).max()


def _kprime(scheme):
    w = np.linspace(0, np.pi, 200001)
    return round(float(np.max(symbol(scheme, w))), 3)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_kprime_is_the_largest_modified_wavenumber(oracle, scheme):
    """The local step's k' (reading of Sec. 3.3's local time stepping) is
    the scheme's largest modified wavenumber to three decimals: Poisson on a
    doubly periodic grid without filter takes dt = 1/(k'^2 sum 1/h^2), so a
    Fourier mode is multiplied by the RK4 polynomial of
    z = -k'(w)^2 dt / h^2 and the mean grows by dt."""
    n0, n1, h = 16, 8, 0.1
    spec = G.GridSpec("periodic", 2, (n0, n1, 1),
                      ((G.PERIODIC, G.PERIODIC), (G.PERIODIC, G.PERIODIC), (0, 0)),
                      h=(h, h, 1.0))
    w = 2 * np.pi * 3 / n0
    x = np.arange(n0)
    phi0 = np.broadcast_to(0.5 + 0.1 * np.cos(w * x)[None, :], (n1, n0)).copy()
    m = oracle.make_method(equation=oracle.POISSON, scheme=scheme, filter=0, rk=oracle.RK4,
                           fixed_iters=1)
    out, st, it, hist = oracle.solve(spec, m, phi0=phi0)
    kp = _kprime(scheme)
    dt = 1.0 / (kp * kp * 2 / h ** 2)
    z = -symbol(scheme, w) ** 2 * dt / h ** 2
    P = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    want = 0.5 + dt + 0.1 * P * np.cos(w * x)
    assert np.abs(out - want[None, :]).max() < 1e-13


@pytest.mark.parametrize("scheme", SCHEMES + ["UW"])
@pytest.mark.parametrize("form", ["eikonal", "hj", "hj_lad", "hj_curv"])
def test_local_step_on_a_constant_field(oracle, scheme, form):
    """At a constant field c on a doubly periodic grid every residual is 1
    (|grad phi| = 0, no Laplacian, no curvature, LAD sensor 0), so one
    pseudo step adds exactly the local step
      dt = sigma / (2 k_adv S1 max(|grad phi|, 1) + k'^2 (Gamma + nu) S2),
    S1 = sum 1/h_l, S2 = sum 1/h_l^2, Gamma = eps c (0 for LAD: its sensor
    vanishes), nu = nu0 (1 - 0)^2 with curvature; the Eikonal drops the
    second term.  k' from the symbol; the upwind baseline uses k_adv = 2 and
    k' = 1.  The filter leaves constants alone."""
    if scheme == "UW" and form == "hj_curv":
        pytest.skip("curvature is not paired with the upwind scheme")
    hx, hy = 0.1, 0.05
    spec = G.GridSpec("periodic", 2, (12, 10, 1),
                      ((G.PERIODIC, G.PERIODIC), (G.PERIODIC, G.PERIODIC), (0, 0)),
                      h=(hx, hy, 1.0))
    c, eps, nu0, sigma = 0.8, 0.3, 0.02, 0.7
    eq = oracle.EIKONAL if form == "eikonal" else oracle.HJ
    gam = oracle.GAMMA_LAD if form == "hj_lad" else oracle.GAMMA_LINEAR
    m = oracle.make_method(equation=eq, gamma=gam, curvature=int(form == "hj_curv"),
                           eps=eps, nu0=nu0, sigma=sigma, scheme=scheme, rk=oracle.RK4,
                           alpha_f=0.48, fixed_iters=1)
    out, st, it, hist = oracle.solve(spec, m, phi0=np.full((10, 12), c))
    kp = 1.0 if scheme == "UW" else _kprime(scheme)
    kadv = 2.0 if scheme == "UW" else kp
    S1, S2 = 1 / hx + 1 / hy, 1 / hx ** 2 + 1 / hy ** 2
    diff = {"eikonal": 0.0, "hj": eps * c, "hj_lad": 0.0, "hj_curv": eps * c + nu0}[form]
    dt = sigma / (2 * kadv * S1 + kp * kp * diff * S2)
    assert np.abs(out - (c + dt)).max() < 1e-14


@pytest.mark.parametrize("c", [0.6, 1.7])
def test_nu_on_an_ogrid(oracle, c):
    """Curvature form with nu = nu0 (1 - |grad phi|)^2 (Sec. 5.4): on a
    uniform-theta O-grid phi = c (r_out - r) has discrete |grad phi| = c,
    Laplacian -c/r and |grad phi| kappa = -c^2/((c + eps0) r) < 0 exactly
    (the O-grid identities), so with eps = 0
      R = 1 - nu0 (1 - c)^2 c / r - c^2."""
    spec = G.cylinder(48, 20, rout=6.0, dr1=2e-2, ratio=1.15)
    r = spec.exact + 0.5
    nu0 = 0.05
    m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LINEAR, curvature=1,
                           eps=0.0, nu0=nu0, eps0=1e-6, scheme="C6")
    ev = oracle.evaluate(spec, m, c * (6.0 - r))
    want = 1 - nu0 * (1 - c) ** 2 * c / r - c * c
    assert np.abs(ev["g"] - c).max() < 1e-11
    assert np.abs(ev["R"] - want).max() < 1e-9


def _affine3d(n=(9, 10, 11), periodic0=False):
    M = np.array([[0.11, 0.03, -0.02],
                  [-0.04, 0.09, 0.025],
                  [0.015, -0.035, 0.13]])
    x0 = np.array([0.3, -0.2, 0.5])
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    X = [x0[m] + M[m, 0] * i + M[m, 1] * j + M[m, 2] * k for m in range(3)]
    bc0 = (G.PERIODIC, G.PERIODIC) if periodic0 else (G.WALL, G.NEUMANN)
    period = None
    if periodic0:
        period = tuple(tuple((n[0] * M[m, 0]) if l == 0 else 0.0 for m in range(3))
                       for l in range(3))
    spec = G.GridSpec("affine3d", 3, n, (bc0, (G.WALL, G.OUTFLOW), (G.NEUMANN, G.WALL)),
                      coords=np.stack(X), period=period)
    return spec, M


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("periodic0", [False, True])
def test_metrics_3d_affine_grid(oracle, scheme, periodic0):
    """An affine 3D grid x = x0 + M (i, j, k) with a full matrix M: every
    scheme and closure differentiates linear functions exactly, so the
    coordinate derivatives are M at every point and the metrics
    d xi_l / d x_m are the entries of M^-1 -- every cofactor of the 3x3
    inverse, off-block terms included.  With direction 0 periodic the seam
    jump n0 M[:, 0] must be added across the seam."""
    spec, M = _affine3d(periodic0=periodic0)
    met = oracle.metrics(spec, scheme)
    inv = np.linalg.inv(M)
    for l in range(3):
        for mm in range(3):
            assert np.abs(met[3 * l + mm] - inv[l, mm]).max() < 1e-11 * np.abs(inv).max()


@pytest.mark.parametrize("case", ["duct_lad", "ogrid_curv", "star_uw", "affine_poisson"])
def test_thread_count_does_not_change_results(oracle, case):
    """The oracle's grid-wide loops are shared among threads line by line
    and point by point; every value must come out bit-identical with one
    thread and with several (fields and the FP64 change history)."""
    if case == "duct_lad":
        spec = G.duct(17, nx=12)
        m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, eps=0.2,
                               scheme="C6", alpha_f=0.48, fixed_iters=6)
    elif case == "ogrid_curv":
        spec = G.cylinder(32, 24, rout=5.0, dr1=1e-2, ratio=1.1)
        m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, curvature=1,
                               eps=0.2, scheme="E6", rk=oracle.RK3, fixed_iters=6)
    elif case == "star_uw":
        spec = G.star_grain(40)
        m = oracle.make_method(equation=oracle.EIKONAL, scheme="UW", fixed_iters=6)
    else:
        spec, _ = _affine3d()
        m = oracle.make_method(equation=oracle.POISSON, scheme="C4", fixed_iters=6)
    before = oracle.set_threads(0)
    try:
        oracle.set_threads(1)
        ref, st1, it1, h1 = oracle.solve(spec, m)
        oracle.set_threads(4)
        par, st4, it4, h4 = oracle.solve(spec, m)
    finally:
        oracle.set_threads(before)
    assert (st1, it1) == (st4, it4)
    assert np.array_equal(ref, par)
    assert np.array_equal(h1, h4)


def _warped_jacobian(spec, amp=0.05):
    """Analytic d x_m / d xi_l (index space) of grids.warped_box."""
    nx, ny, nz = spec.n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = [i / (nx - 1.0), j / (ny - 1.0), k / (nz - 1.0)]
    h = [1.0 / (nx - 1.0), 1.0 / (ny - 1.0), 1.0 / (nz - 1.0)]
    pi = np.pi
    A = np.zeros((3, 3) + spec.shape)
    for m in range(3):
        a, b = (m + 1) % 3, (m + 2) % 3
        # x_m = s_m + amp sin(pi s_m) sin(2 pi s_a) cos(pi s_b)
        f1, f2, f3 = np.sin(pi * s[m]), np.sin(2 * pi * s[a]), np.cos(pi * s[b])
        A[m, m] = (1 + amp * pi * np.cos(pi * s[m]) * f2 * f3) * h[m]
        A[m, a] = amp * f1 * 2 * pi * np.cos(2 * pi * s[a]) * f3 * h[a]
        A[m, b] = -amp * f1 * f2 * pi * np.sin(pi * s[b]) * h[b]
    return A


def _inverse_metrics(A):
    Am = np.moveaxis(A, (0, 1), (-2, -1))
    inv = np.linalg.inv(Am)                  # inv[..., l, m] = d xi_l / d x_m
    return np.moveaxis(inv, (-2, -1), (0, 1))


def _dline(oracle, f, axis, scheme):
    """Derivative along one array axis (no periodic directions)."""
    g = np.moveaxis(f, axis, -1)
    out = np.empty_like(g)
    for idx in np.ndindex(g.shape[:-1]):
        out[idx] = oracle.deriv_line(np.ascontiguousarray(g[idx]), scheme)
    return np.moveaxis(out, -1, axis)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_metrics_3d_conservative_form_affine(oracle, scheme):
    """The conservative metric form (J xi_{l,m} written as a divergence of
    coordinate products) equals M^-1 on an affine grid, as the inverse form
    does: the products are linear there and every scheme is exact."""
    spec, M = _affine3d()
    spec.metric_form = 1
    met = oracle.metrics(spec, scheme)
    inv = np.linalg.inv(M)
    for l in range(3):
        for mm in range(3):
            assert np.abs(met[3 * l + mm] - inv[l, mm]).max() < 1e-11 * np.abs(inv).max()


def test_metric_identity_of_the_conservative_form(oracle):
    """On the warped box (a full, varying Jacobian) the conservative form
    satisfies the discrete metric identities sum_l D_l (J xi_{l,m}) = 0 to
    rounding, with J the determinant of the coordinate derivatives; the
    inverse form leaves a truncation-size residual."""
    spec = G.warped_box(13)
    res = {}
    # array axes of a (z, y, x) field: direction l runs along axis 2 - l
    D = [[_dline(oracle, spec.coords[m], 2 - l, "E4") for l in range(3)] for m in range(3)]
    Am = np.moveaxis(np.array(D), (0, 1), (-2, -1))
    det = np.linalg.det(Am)
    for form in (0, 1):
        spec.metric_form = form
        met = oracle.metrics(spec, "E4").reshape((3, 3) + spec.shape)
        worst = 0.0
        for mm in range(3):
            s = sum(_dline(oracle, det * met[l, mm], 2 - l, "E4") for l in range(3))
            worst = max(worst, float(np.abs(s).max()))
        res[form] = worst
    scale = float(np.abs(det).max())
    assert res[1] < 1e-13 * scale * 13
    assert res[0] > 1e3 * res[1]


@pytest.mark.parametrize("form", [0, 1])
def test_warped_metrics_converge_at_the_scheme_order(oracle, form):
    """Both metric forms approach the analytic metrics of the warped box at
    the scheme's order under refinement (E4: about 16x per halving of the
    spacing; a sign or index slip in either form would not converge)."""
    errs = []
    for n in (17, 33):
        spec = G.warped_box(n, metric_form=form)
        met = oracle.metrics(spec, "E4").reshape((3, 3) + spec.shape)
        ex = _inverse_metrics(_warped_jacobian(spec))
        errs.append(float(np.abs(met - ex).max() / np.abs(ex).max()))
    assert errs[1] < errs[0] / 10.0
    assert errs[1] < 1e-3


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("scheme,sigma", [("C6", 1.0), ("E4", 0.5)])
def test_warped_box_distance(oracle, form, scheme, sigma):
    """The LAD pseudo-HJ march on the 17^3 warped box (both metric forms)
    converges to within about a cell of min(x, 1-x, y, 1-y, z, 1-z) (the
    kinks where the nearest wall changes); E4 needs the halved pseudo-step
    here (with sigma = 1 it settles to 5e-8 and then grows)."""
    spec = G.warped_box(17, metric_form=form)
    m = oracle.make_method(equation=oracle.HJ, gamma=oracle.GAMMA_LAD, eps=0.2, scheme=scheme,
                           alpha_f=0.48, sigma=sigma, tol=1e-8, max_iter=3000)
    phi, st, it, _ = oracle.solve(spec, m)
    assert st == 0
    assert np.abs(phi - spec.exact).max() < 1.0 / 16
