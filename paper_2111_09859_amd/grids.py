"""Seeded synthetic grids for wall-distance solves.

Geometry only: coordinates, boundary-condition codes, solid masks and the
closed-form distance where the geometry has one.  Nothing here computes any
part of the wall-distance method; both the GPU path and the test oracle take
their inputs from this module.

Layout: a 2D field has numpy shape ``(n1, n0)``, a 3D field ``(n2, n1, n0)``;
x (index 0) is fastest.  Coordinates are stacked SoA: ``(ndim,) + shape``.

The paper's own case table is an image that did not survive, so these
generators stand in for its canonical cases (channel, cylinder/circular
bump, 3D box/duct, star-shaped propellant grain) with the sizes of the
workloads this library is measured on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

WALL, NEUMANN, OUTFLOW, PERIODIC = 0, 1, 2, 3
SEED = 211109859


@dataclass
class GridSpec:
    name: str
    ndim: int
    n: tuple                         # (n0, n1, n2); n2 = 1 in 2D
    bc: tuple                        # ((lo, hi), (lo, hi), (lo, hi))
    h: Optional[tuple] = None        # uniform spacing (Cartesian grids)
    coords: Optional[np.ndarray] = None
    period: Optional[tuple] = None   # coordinate jump across periodic seams
    mask: Optional[np.ndarray] = None
    exact: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    metric_form: int = 0                 # 0 inverse of the coordinate Jacobian,
                                         # 1 conservative form (3D)

    @property
    def shape(self):
        return tuple(reversed(self.n[: self.ndim]))

    @property
    def npoints(self):
        return int(np.prod(self.n[: self.ndim]))


def capped_geometric(nr: int, dr1: float, ratio: float, total: float):
    """Radial offsets rho_0 = 0 < rho_1 < ... < rho_{nr-1} = total.

    Spacing dr_j = min(dr1 * ratio**j, cap) with the cap found by bisection
    so that the offsets end exactly at ``total``.  If even the uncapped
    series falls short, the ratio is raised (bisection) instead and no cap
    applies.
    """
    j = np.arange(nr - 1, dtype=np.float64)

    def span(r, cap):
        return float(np.minimum(dr1 * r ** j, cap).sum())

    if span(ratio, np.inf) < total:
        lo, hi = ratio, 4.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if span(mid, np.inf) < total:
                lo = mid
            else:
                hi = mid
        ratio, cap = 0.5 * (lo + hi), np.inf
        dr = dr1 * ratio ** j
    else:
        lo, hi = dr1, total
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if span(ratio, mid) < total:
                lo = mid
            else:
                hi = mid
        cap = 0.5 * (lo + hi)
        dr = np.minimum(dr1 * ratio ** j, cap)
    dr *= total / dr.sum()
    rho = np.concatenate([[0.0], np.cumsum(dr)])
    rho[-1] = total
    return rho, ratio, cap


def channel(nx: int = 129, ny: int = 65, lx: float = 2.0) -> GridSpec:
    """Uniform Cartesian channel: x periodic on [0, lx) with nx distinct
    points, walls y = 0 and y = 1 (ny points).  Exact d = min(y, 1 - y)."""
    dx, dy = lx / nx, 1.0 / (ny - 1)
    y = np.arange(ny) * dy
    exact = np.broadcast_to(np.minimum(y, 1.0 - y)[:, None], (ny, nx)).copy()
    return GridSpec("channel", 2, (nx, ny, 1),
                    ((PERIODIC, PERIODIC), (WALL, WALL), (WALL, WALL)),
                    h=(dx, dy, 1.0), exact=exact,
                    meta={"lx": lx})


def channel_curvilinear(nx: int = 65, ny: int = 33, lx: float = 2.0) -> GridSpec:
    """The channel given by coordinates (periodic x seam jump lx)."""
    g = channel(nx, ny, lx)
    dx, dy = g.h[0], g.h[1]
    X, Y = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dy)
    g.coords = np.stack([X, Y])
    g.period = ((lx, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    g.h = None
    g.name = "channel_curvilinear"
    return g


def o_grid(ntheta: int, nr: int, a: float = 0.5, b: float = 0.5,
           rout: float = 20.0, dr1: float = 1e-3, ratio: float = 1.03,
           far: int = OUTFLOW) -> GridSpec:
    """O-grid around an ellipse with semi-axes (a, b), built by offsets
    along the wall's outward normals, so the exact wall distance of node
    (i, j) is the offset rho_j.  Wall at j = 0; far field at j = nr - 1.
    theta is periodic with ntheta distinct points.  A circle (a == b) gives
    the cylinder O-grid with the far boundary at radius rout."""
    total = rout - a if a == b else rout - max(a, b)
    rho, ratio_used, cap = capped_geometric(nr, dr1, ratio, total)
    t = 2.0 * np.pi * np.arange(ntheta) / ntheta
    wx, wy = a * np.cos(t), b * np.sin(t)
    nx_, ny_ = b * np.cos(t), a * np.sin(t)
    nn = np.hypot(nx_, ny_)
    nx_, ny_ = nx_ / nn, ny_ / nn
    X = wx[None, :] + rho[:, None] * nx_[None, :]
    Y = wy[None, :] + rho[:, None] * ny_[None, :]
    exact = np.broadcast_to(rho[:, None], (nr, ntheta)).copy()
    name = "cylinder" if a == b else "ellipse"
    return GridSpec(name, 2, (ntheta, nr, 1),
                    ((PERIODIC, PERIODIC), (WALL, far), (WALL, WALL)),
                    coords=np.stack([X, Y]), exact=exact,
                    meta={"a": a, "b": b, "ratio": ratio_used, "cap": cap,
                          "rho": rho, "theta": t})


def cylinder3d(ntheta: int, nr: int, nz: int, R: float = 0.5, rout: float = 6.0,
               dr1: float = 1e-2, ratio: float = 1.12, far: int = OUTFLOW,
               length: float = 1.0) -> GridSpec:
    """The cylinder O-grid extruded along z (nz points on [0, length], faces
    with zero normal gradient): a 3D curvilinear grid whose metrics mix the
    two in-plane directions.  Exact d = r - R."""
    g = cylinder(ntheta, nr, R, rout, dr1, ratio, far)
    z = np.linspace(0.0, length, nz)
    X = np.broadcast_to(g.coords[0][None], (nz, nr, ntheta)).copy()
    Y = np.broadcast_to(g.coords[1][None], (nz, nr, ntheta)).copy()
    Z = np.broadcast_to(z[:, None, None], (nz, nr, ntheta)).copy()
    exact = np.broadcast_to(g.exact[None], (nz, nr, ntheta)).copy()
    return GridSpec("cylinder3d", 3, (ntheta, nr, nz),
                    ((PERIODIC, PERIODIC), (WALL, far), (NEUMANN, NEUMANN)),
                    coords=np.stack([X, Y, Z]), exact=exact, meta=dict(g.meta))


def cylinder(ntheta: int = 512, nr: int = 256, R: float = 0.5,
             rout: float = 20.0, dr1: float = 1e-3, ratio: float = 1.03,
             far: int = OUTFLOW) -> GridSpec:
    """Cylinder O-grid: wall r = R, far field r = rout, radial spacing
    dr_j = min(dr1 ratio^j, cap).  Exact d = r - R."""
    return o_grid(ntheta, nr, R, R, rout, dr1, ratio, far)


def ellipse(ntheta: int, nr: int, axis_ratio: float, ratio: float,
            a: float = 0.5, rout: float = 20.0, dr1: float = 1e-3,
            far: int = OUTFLOW) -> GridSpec:
    """Ellipse O-grid (semi-axes a, a/axis_ratio), normal offsets to
    rho = rout - a.  Exact d = rho_j."""
    return o_grid(ntheta, nr, a, a / axis_ratio, rout, dr1, ratio, far)


def duct(n: int = 256, nx: Optional[int] = None) -> GridSpec:
    """3D square duct on [0,1]^3: x periodic (nx distinct points, dx = 1/nx),
    walls y = 0, 1 and z = 0, 1 (n points each).  Exact
    d = min(y, 1-y, z, 1-z)."""
    nx = n if nx is None else nx
    dx, dy = 1.0 / nx, 1.0 / (n - 1)
    y = np.arange(n) * dy
    dy_ = np.minimum(y, 1.0 - y)
    ex = np.minimum(dy_[None, :, None], dy_[:, None, None])
    exact = np.broadcast_to(ex, (n, n, nx)).copy()
    return GridSpec("duct", 3, (nx, n, n),
                    ((PERIODIC, PERIODIC), (WALL, WALL), (WALL, WALL)),
                    h=(dx, dy, dy), exact=exact)


def warped_box(n: int = 33, amp: float = 0.05, nx: Optional[int] = None,
               ny: Optional[int] = None, metric_form: int = 0) -> GridSpec:
    """Curvilinear 3D grid of the unit cube [0,1]^3 with walls on all six
    faces, its interior nodes displaced smoothly so that every coordinate
    depends on every index (a full, varying 3x3 Jacobian, not an
    extrusion): with s = (i, j, k) / (n - 1),
      x = s_x + amp sin(pi s_x) sin(2 pi s_y) cos(pi s_z),
      y = s_y + amp sin(pi s_y) sin(2 pi s_z) cos(pi s_x),
      z = s_z + amp sin(pi s_z) sin(2 pi s_x) cos(pi s_y).
    Each face keeps its plane (x = 0 on s_x = 0, ...), so the exact
    distance is min(x, 1-x, y, 1-y, z, 1-z) at every node."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sx, sy, sz = i / (nx - 1.0), j / (ny - 1.0), k / (nz - 1.0)
    pi = np.pi
    x = sx + amp * np.sin(pi * sx) * np.sin(2 * pi * sy) * np.cos(pi * sz)
    y = sy + amp * np.sin(pi * sy) * np.sin(2 * pi * sz) * np.cos(pi * sx)
    z = sz + amp * np.sin(pi * sz) * np.sin(2 * pi * sx) * np.cos(pi * sy)
    exact = np.minimum.reduce([x, 1 - x, y, 1 - y, z, 1 - z])
    return GridSpec("warped_box", 3, (nx, ny, nz),
                    ((WALL, WALL), (WALL, WALL), (WALL, WALL)),
                    coords=np.stack([x, y, z]), exact=exact, metric_form=metric_form)


def box2d(n: int = 65) -> GridSpec:
    """2D box [0,1]^2 with four walls.  Exact d = min(x, 1-x, y, 1-y)."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    dx = np.minimum(x, 1.0 - x)
    exact = np.minimum(dx[None, :], dx[:, None])
    return GridSpec("box2d", 2, (n, n, 1),
                    ((WALL, WALL), (WALL, WALL), (WALL, WALL)),
                    h=(h, h, 1.0), exact=exact)


def star_port_radius(theta, step: int = 0, r0: float = 0.2, amp: float = 0.3,
                     lobes: int = 6, recession: float = 0.002):
    """Port boundary r_k(theta) = r0 (1 + amp cos(lobes theta)) + k recession."""
    return r0 * (1.0 + amp * np.cos(lobes * theta)) + step * recession


def square(n: int = 65, half: float = 1.0, bc: int = NEUMANN) -> GridSpec:
    """Cartesian n x n grid on [-half, half]^2 with the same kind on every
    face (a field's domain for the level-set march and the iso-lines)."""
    h = 2.0 * half / (n - 1)
    return GridSpec("square", 2, (n, n, 1), ((bc, bc), (bc, bc), (WALL, WALL)),
                    h=(h, h, 1.0), meta={"half": half})


def square_xy(spec: GridSpec):
    """Node coordinates (X, Y) of a `square` grid, arrays of spec.shape."""
    half = spec.meta["half"]
    x = -half + np.arange(spec.n[0]) * spec.h[0]
    y = -half + np.arange(spec.n[1]) * spec.h[1]
    return np.meshgrid(x, y)


def star_grain_solid(n: int = 512, step: int = 0, **kw) -> GridSpec:
    """The star grain's propellant side: the port (r < r_k(theta)) is masked,
    so its boundary is the wall, and the outer faces have zero normal
    gradient; the distance solved here is the solid-side half of the signed
    distance of the burnback (Sec. 5.5)."""
    g = star_grain(n, step, **kw)
    port = (1 - g.mask).astype(np.uint8)
    return GridSpec("star_grain_solid", 2, g.n,
                    ((NEUMANN, NEUMANN), (NEUMANN, NEUMANN), (WALL, WALL)),
                    h=g.h, mask=port, meta=dict(g.meta))


def star_grain(n: int = 512, step: int = 0, **kw) -> GridSpec:
    """Cartesian n x n grid on [-0.5, 0.5]^2; the star-shaped port
    r < r_k(theta) is fluid, everything else is solid propellant (mask 1).
    All four faces lie in the solid and are walls."""
    h = 1.0 / (n - 1)
    x = -0.5 + np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X, Y)
    th = np.arctan2(Y, X)
    mask = (r >= star_port_radius(th, step, **kw)).astype(np.uint8)
    return GridSpec("star_grain", 2, (n, n, 1),
                    ((WALL, WALL), (WALL, WALL), (WALL, WALL)),
                    h=(h, h, 1.0), mask=mask, meta={"step": step})


# ---------------------------------------------------------------------------
# Moving walls (the unsteady canonical cases of Sec. 5.5): one grid per
# physical time step, the same index dimensions at every step.
def piston(ntheta: int = 64, nr: int = 25, nz: int = 33, h: float = 1.0,
           R: float = 0.25, Rb: float = 1.0) -> GridSpec:
    """Piston-cylinder stand-in: the annular bore R <= r <= Rb (a rod on the
    axis keeps the O-grid free of a singular line), closed by the cylinder
    head at z = 0 and the piston face at z = h.  Walls on the four r and z
    faces, theta periodic; uniform spacing in r and z, so moving the piston
    only rescales z.  Exact d = min(r - R, Rb - r, z, h - z)."""
    t = 2.0 * np.pi * np.arange(ntheta) / ntheta
    r = R + (Rb - R) * np.arange(nr) / (nr - 1)
    z = h * np.arange(nz) / (nz - 1)
    Z, Rr, T = np.meshgrid(z, r, t, indexing="ij")
    exact = np.minimum(np.minimum(Rr - R, Rb - Rr), np.minimum(Z, h - Z))
    return GridSpec("piston", 3, (ntheta, nr, nz),
                    ((PERIODIC, PERIODIC), (WALL, WALL), (WALL, WALL)),
                    coords=np.stack([Rr * np.cos(T), Rr * np.sin(T), Z]),
                    exact=exact, meta={"h": h, "R": R, "Rb": Rb})


def piston_stroke(steps: int, h0: float = 1.0, amp: float = 0.4) -> np.ndarray:
    """Piston positions h_k = h0 + amp cos(2 pi k / steps), k = 0..steps:
    one full stroke (top dead centre, bottom, back)."""
    k = np.arange(steps + 1)
    return h0 + amp * np.cos(2.0 * np.pi * k / steps)


def bouncing_cube(n: int = 65, zb: float = 0.5, side: float = 0.25,
                  cx: float = 0.5, cy: float = 0.5) -> GridSpec:
    """Cube-between-walls stand-in: Cartesian n^3 grid on [0, 1]^3, walls at
    the floor z = 0 and the ceiling z = 1, zero normal gradient on the four
    sides, and a solid cube (mask 1, surface included) whose faces lie on
    grid planes: its extents are snapped to the nearest nodes, its bottom
    at zb.  Exact d = min(z, 1 - z, distance to the snapped cube)."""
    h = 1.0 / (n - 1)
    w = int(round(side / h))
    i0 = int(round(cx / h - 0.5 * w))
    j0 = int(round(cy / h - 0.5 * w))
    k0 = min(max(int(round(zb / h)), 0), n - 1 - w)
    x = np.arange(n) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    lo = (i0 * h, j0 * h, k0 * h)
    hi = ((i0 + w) * h, (j0 + w) * h, (k0 + w) * h)

    def gap(c, a, b):
        return np.maximum(np.maximum(a - c, c - b), 0.0)

    box = np.sqrt(gap(X, lo[0], hi[0]) ** 2 + gap(Y, lo[1], hi[1]) ** 2
                  + gap(Z, lo[2], hi[2]) ** 2)
    exact = np.minimum(np.minimum(Z, 1.0 - Z), box)
    inside = ((X >= lo[0] - 1e-12) & (X <= hi[0] + 1e-12) & (Y >= lo[1] - 1e-12)
              & (Y <= hi[1] + 1e-12) & (Z >= lo[2] - 1e-12) & (Z <= hi[2] + 1e-12))
    return GridSpec("bouncing_cube", 3, (n, n, n),
                    ((NEUMANN, NEUMANN), (NEUMANN, NEUMANN), (WALL, WALL)),
                    h=(h, h, h), mask=inside.astype(np.uint8), exact=exact,
                    meta={"lo": lo, "hi": hi, "zb": k0 * h})


def bounce_heights(steps: int, t_end: float, z0: float = 0.6, g: float = 1.0,
                   kept: float = 0.8) -> np.ndarray:
    """Bottom height of a cube dropped from rest at z0 under gravity g onto
    the floor, keeping the fraction `kept` of its energy at every bounce
    (the rebound speed scales by sqrt(kept)); sampled at t_k = k t_end /
    steps, k = 0..steps.  Closed form per flight."""
    out = np.empty(steps + 1)
    for k in range(steps + 1):
        t = k * t_end / steps
        # first flight: the drop
        t_hit = math.sqrt(2.0 * z0 / g)
        if t < t_hit:
            out[k] = z0 - 0.5 * g * t * t
            continue
        t -= t_hit
        v = g * t_hit
        z = 0.0
        while True:
            v *= math.sqrt(kept)
            flight = 2.0 * v / g
            if flight < 1e-9 or t < flight:
                z = max(v * t - 0.5 * g * t * t, 0.0) if flight >= 1e-9 else 0.0
                break
            t -= flight
        out[k] = z
    return out


def cartesian_points(spec: GridSpec) -> np.ndarray:
    """(npoints, ndim) physical coordinates of a grid, x fastest."""
    if spec.coords is not None:
        return np.stack([c.ravel() for c in spec.coords], axis=1)
    axes = [np.arange(spec.n[l]) * spec.h[l] for l in range(spec.ndim)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.transpose().ravel() for m in mesh], axis=1)


# ---------------------------------------------------------------------------
# Workload mixes
def batch_mix(count: int = 64, seed: int = SEED, max_u: float = 10.0,
              min_u: float = 6.0):
    """Seeded mix of 2D grids: m = 2 round(2^u / 2), u ~ U[min_u, max_u],
    shape (m+1) x (m/2+1); geometry uniform over {channel, cylinder,
    ellipse}; ellipse axis ratio U[1, 4]; radial ratio U[1.01, 1.08];
    O-grids with the zero-gradient (Neumann) far field of Sec. 3.5;
    scheme uniform over {E6, C6}.  Returns a list of (GridSpec, scheme)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        u = rng.uniform(min_u, max_u)
        m = 2 * int(round(2.0 ** u / 2.0))
        geo = rng.integers(0, 3)
        scheme = "E6" if rng.integers(0, 2) == 0 else "C6"
        ar = rng.uniform(1.0, 4.0)
        s = rng.uniform(1.01, 1.08)
        if geo == 0:
            spec = channel(m + 1, m // 2 + 1)
        elif geo == 1:
            spec = cylinder(m + 1, m // 2 + 1, ratio=s, far=NEUMANN)
        else:
            spec = ellipse(m + 1, m // 2 + 1, axis_ratio=ar, ratio=s, far=NEUMANN)
        out.append((spec, scheme))
    return out


def serving_stream(count: int = 2000, rate: float = 200.0, seed: int = SEED,
                   frac_2d: float = 0.75, max_u2: float = 11.0,
                   max_n3: int = 192):
    """Open-loop request stream: Poisson arrivals (mean ``rate`` per s);
    0.75 2D / 0.25 3D.  2D: n = 2^u + 1, u ~ U[7, max_u2], geometry as in
    ``batch_mix`` on an n x n grid; 3D: duct with n = round(2^u),
    u ~ U[6, log2(max_n3)].  Returns a list of dicts (arrival time, kind,
    parameters) -- grids are built lazily by ``build_request``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < frac_2d:
            u = rng.uniform(7.0, max_u2)
            n = int(round(2.0 ** u)) + 1
            geo = int(rng.integers(0, 3))
            req = {"t": t, "kind": "2d", "n": n, "geo": geo,
                   "ar": float(rng.uniform(1.0, 4.0)),
                   "ratio": float(rng.uniform(1.01, 1.08))}
        else:
            u = rng.uniform(6.0, math.log2(max_n3))
            req = {"t": t, "kind": "3d", "n": int(round(2.0 ** u))}
        req["scheme"] = "E6" if rng.integers(0, 2) == 0 else "C6"
        req["id"] = k
        out.append(req)
    return out


def build_request(req) -> GridSpec:
    if req["kind"] == "3d":
        return duct(req["n"])
    n = req["n"]
    if req["geo"] == 0:
        return channel(n, n)
    if req["geo"] == 1:
        return cylinder(n, n, ratio=req["ratio"], far=NEUMANN)
    return ellipse(n, n, axis_ratio=req["ar"], ratio=req["ratio"], far=NEUMANN)


def scored(spec: GridSpec, band: float = 0.1) -> np.ndarray:
    """Points where the exact distance is the solution of the discrete
    problem: all of them, except on O-grids with a zero-gradient far field,
    where the outer ``band`` fraction of radial lines is left out (there the
    boundary condition, not the method, sets the field)."""
    keep = np.ones(spec.shape, dtype=bool)
    if spec.ndim == 2 and spec.coords is not None and spec.bc[1][1] == NEUMANN:
        nr = spec.n[1]
        cut = int(np.ceil((1.0 - band) * (nr - 1)))
        keep[cut:, :] = False
    return keep


def linf_error(spec: GridSpec, phi) -> float:
    """L-inf distance error against the exact field over ``scored`` points."""
    phi = np.asarray(phi, dtype=np.float64)
    return float(np.abs(phi - spec.exact)[scored(spec)].max())
