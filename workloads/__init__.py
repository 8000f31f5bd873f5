"""Seeded synthetic inputs for the semi-implicit PHS-RBF solver.

This module produces point clouds (coordinates, point kinds, outward boundary
normals, the pressure-pin point), the closed-form flows that supply Dirichlet
data and accuracy references, and nothing else: it holds none of the method's
arithmetic (no neighbour search, no collocation, no operators, no solver).
Both the HIP library's callers and the FP64 oracle read the clouds made here.

Every generator is deterministic for a given seed (numpy ``default_rng``).
Points are returned Morton-sorted (21 bits per dimension over the bounding box),
which keeps stencil neighbours close in memory for the device kernels.

Point kinds: 0 = interior, 1 = Dirichlet-velocity boundary (wall or inlet,
where the pressure correction obeys a homogeneous Neumann condition and the
boundary pressure follows the normal momentum equation), 2 = Dirichlet-velocity
boundary with prescribed pressure (pressure correction zero there).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INTERIOR = 0
DIRICHLET = 1
PRESCRIBED_PRESSURE = 2
OUTLET = 3          # prescribed pressure, zero normal derivative of the velocity
SYMMETRY = 4        # symmetry plane normal to a coordinate axis


@dataclass
class Cloud:
    dim: int
    xyz: np.ndarray          # (n, dim) float64
    kind: np.ndarray         # (n,) uint8
    normal: np.ndarray       # (n, dim) float64; unit outward normal on boundary points, 0 inside
    pin: int                 # interior point whose pressure correction is held at zero
    name: str = ""
    h: float = 0.0           # nominal point spacing of the generator
    meta: dict = field(default_factory=dict)
    period: tuple = (0.0, 0.0, 0.0)   # > 0: the cloud wraps along that axis

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    def boundary(self) -> np.ndarray:
        return self.kind != INTERIOR


# --------------------------------------------------------------------------
# closed-form incompressible flows (rho = 1)
# --------------------------------------------------------------------------

def kovasznay(x, y, Re=40.0):
    """Kovasznay's steady laminar wake behind a grid (Re = 1/nu)."""
    lam = Re / 2.0 - np.sqrt(Re * Re / 4.0 + 4.0 * np.pi * np.pi)
    e = np.exp(lam * x)
    u = 1.0 - e * np.cos(2.0 * np.pi * y)
    v = lam / (2.0 * np.pi) * e * np.sin(2.0 * np.pi * y)
    p = 0.5 * (1.0 - np.exp(2.0 * lam * x))
    return u, v, p


def taylor_green(x, y, t, nu=0.01):
    """Decaying Taylor-Green vortex on a periodic 2*pi square."""
    F = np.exp(-2.0 * nu * t)
    u = np.cos(x) * np.sin(y) * F
    v = -np.sin(x) * np.cos(y) * F
    p = -0.25 * (np.cos(2.0 * x) + np.cos(2.0 * y)) * F * F
    return u, v, p


def beltrami(x, y, z, t, a=np.pi / 4, d=np.pi / 2, nu=0.01):
    """Ethier-Steinman three-dimensional Beltrami flow."""
    G = np.exp(-nu * d * d * t)
    u = -a * (np.exp(a * x) * np.sin(a * y + d * z) + np.exp(a * z) * np.cos(a * x + d * y)) * G
    v = -a * (np.exp(a * y) * np.sin(a * z + d * x) + np.exp(a * x) * np.cos(a * y + d * z)) * G
    w = -a * (np.exp(a * z) * np.sin(a * x + d * y) + np.exp(a * y) * np.cos(a * z + d * x)) * G
    p = -0.5 * a * a * (
        np.exp(2 * a * x) + np.exp(2 * a * y) + np.exp(2 * a * z)
        + 2 * np.sin(a * x + d * y) * np.cos(a * z + d * x) * np.exp(a * (y + z))
        + 2 * np.sin(a * y + d * z) * np.cos(a * x + d * y) * np.exp(a * (z + x))
        + 2 * np.sin(a * z + d * x) * np.cos(a * y + d * z) * np.exp(a * (x + y))
    ) * G * G
    return u, v, w, p


def couette(x, y, r1=0.5, r2=1.0, omega=2.0):
    """Steady cylindrical Couette flow between an inner cylinder of radius r1
    turning at angular speed omega and a fixed outer cylinder of radius r2
    (Sec. 4.1, Eq. couette v_theta): v_theta(r) = a/r + b r with
    a = omega r1^2 r2^2 / (r2^2 - r1^2) and b = -omega r1^2 / (r2^2 - r1^2).
    The radial momentum balance dp/dr = v_theta^2 / r (rho = 1) gives
    p = -a^2/(2 r^2) + 2 a b ln r + b^2 r^2 / 2, shifted to zero mean over
    [r1, r2] in r (the level is arbitrary)."""
    a = omega * r1 * r1 * r2 * r2 / (r2 * r2 - r1 * r1)
    b = -omega * r1 * r1 / (r2 * r2 - r1 * r1)
    r = np.sqrt(x * x + y * y)
    vt = a / r + b * r
    u = -vt * y / r
    v = vt * x / r

    def prim(rr):
        return -a * a / (2 * rr * rr) + 2 * a * b * np.log(rr) + b * b * rr * rr / 2

    # mean of prim over r in [r1, r2] (closed form of its integral / (r2 - r1))
    def integ(rr):
        return a * a / (2 * rr) + 2 * a * b * (rr * np.log(rr) - rr) + b * b * rr ** 3 / 6

    mean = (integ(r2) - integ(r1)) / (r2 - r1)
    p = prim(r) - mean
    return u, v, p


def poiseuille(x, y, U=1.0, mu=0.01):
    """Plane Poiseuille flow in the channel 0 <= y <= 1 (rho = 1): u = 4U y(1-y),
    v = 0, p = -8 mu U x. Fully developed, so every outlet x = const has a zero
    normal velocity gradient."""
    u = 4.0 * U * y * (1.0 - y)
    v = np.zeros_like(u)
    p = -8.0 * mu * U * x
    return u, v, p


def flow_fields(cloud: Cloud, t: float = 0.0):
    """Exact (velocity[dim, n], pressure[n]) of the cloud's flow at time t. A
    rotated cloud (rotated()) carries the rotated flow: R u(R^T x), p(R^T x)."""
    if cloud.meta.get("rotation") is not None:
        rot = np.asarray(cloud.meta["rotation"], dtype=np.float64)
        meta = {k: v for k, v in cloud.meta.items() if k != "rotation"}
        base = Cloud(dim=cloud.dim, xyz=cloud.xyz @ rot, kind=cloud.kind, normal=cloud.normal @ rot, pin=cloud.pin,
                     name=cloud.name, h=cloud.h, meta=meta, period=cloud.period)
        vel, p = flow_fields(base, t)
        return np.ascontiguousarray(rot @ vel), p
    x = cloud.xyz
    flow = cloud.meta.get("flow")
    if flow == "kovasznay":
        u, v, p = kovasznay(x[:, 0], x[:, 1], cloud.meta.get("Re", 40.0))
        vel = np.stack([u, v])
    elif flow == "taylor_green":
        u, v, p = taylor_green(x[:, 0], x[:, 1], t, cloud.meta.get("nu", 0.01))
        vel = np.stack([u, v])
    elif flow == "beltrami":
        u, v, w, p = beltrami(x[:, 0], x[:, 1], x[:, 2], t, nu=cloud.meta.get("nu", 0.01))
        vel = np.stack([u, v, w])
    elif flow == "poiseuille_forced":
        u, v, _ = poiseuille(x[:, 0], x[:, 1], cloud.meta.get("U", 1.0), cloud.meta["nu"])
        p = np.zeros_like(u)
        vel = np.stack([u, v])
    elif flow == "poiseuille":
        u, v, p = poiseuille(x[:, 0], x[:, 1], cloud.meta.get("U", 1.0), cloud.meta["nu"])
        vel = np.stack([u, v])
    elif flow == "stagnation":
        vel, p = polynomial_flow(x, t, "stagnation", 1.0)
    elif flow == "couette":
        u, v, p = couette(x[:, 0], x[:, 1], cloud.meta["r1"], cloud.meta["r2"], cloud.meta["omega"])
        vel = np.stack([u, v])
    elif flow == "kovasznay_holes":
        u, v, p = kovasznay(x[:, 0], x[:, 1], cloud.meta.get("Re", 40.0))
        vel = np.stack([u, v])
        on_hole = cloud.meta["on_hole"]
        vel[:, on_hole] = 0.0          # no-slip on the holes
    else:
        raise ValueError(f"cloud has no closed-form flow: {flow!r}")
    return np.ascontiguousarray(vel), np.ascontiguousarray(p)


def polynomial_flow(xyz, t: float, which: str, rho: float = 1.0):
    """Exact Navier-Stokes solutions whose fields are polynomials of degree <= 2
    in space and <= 1 in time, so that PHS-RBF operators with degree >= 2
    polynomials and BDF2 reproduce them without discretization error.

    "stagnation": steady u = (x, -y) [3D: (x, y, -2z)], p = -rho |grad phi|^2 / 2.
    "uniform": spatially uniform u(t) that grows linearly in t, driven by a
    constant pressure gradient p = -rho u'(t) . x.
    Both are divergence free for any viscosity. Returns (vel[dim, n], p[n]).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    dim = xyz.shape[1]
    if which == "stagnation":
        if dim == 2:
            x, y = xyz[:, 0], xyz[:, 1]
            vel = np.stack([x, -y])
            p = -rho * (x * x + y * y) / 2
        else:
            x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
            vel = np.stack([x, y, -2.0 * z])
            p = -rho * (x * x + y * y + 4.0 * z * z) / 2
    elif which == "uniform":
        a0 = np.array([0.7, -0.2, 0.1])[:dim]
        a1 = np.array([0.5, 0.3, -0.4])[:dim]
        vel = np.repeat((a0 + a1 * t)[:, None], len(xyz), axis=1)
        p = -rho * (xyz @ a1)
    else:
        raise ValueError(which)
    return np.ascontiguousarray(vel), np.ascontiguousarray(p)


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def _part1by1(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * 2)
    return out


def _part1by2(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * 3)
    return out


def morton_order(xyz: np.ndarray) -> np.ndarray:
    """Stable permutation sorting points by a 21-bit-per-axis Morton code."""
    lo = xyz.min(axis=0)
    span = np.maximum(xyz.max(axis=0) - lo, 1e-300)
    qv = np.floor((xyz - lo) / span * ((1 << 21) - 1)).astype(np.int64)
    qv = np.clip(qv, 0, (1 << 21) - 1)
    if xyz.shape[1] == 2:
        code = _part1by1(qv[:, 0]) | (_part1by1(qv[:, 1]) << np.uint64(1))
    else:
        code = (_part1by2(qv[:, 0]) | (_part1by2(qv[:, 1]) << np.uint64(1))
                | (_part1by2(qv[:, 2]) << np.uint64(2)))
    return np.argsort(code, kind="stable")


def _finish(dim, xyz, kind, normal, name, h, meta, centre, boundary_kind=DIRICHLET, period=(0.0, 0.0, 0.0)):
    if boundary_kind is not None:   # None: keep the kinds given per point
        kind = np.where(kind != INTERIOR, boundary_kind, INTERIOR)
    kind = kind.astype(np.uint8)
    order = morton_order(xyz)
    xyz = np.ascontiguousarray(xyz[order], dtype=np.float64)
    kind = np.ascontiguousarray(kind[order], dtype=np.uint8)
    normal = np.ascontiguousarray(normal[order], dtype=np.float64)
    for key in ("on_hole",):
        if key in meta:
            meta[key] = np.ascontiguousarray(meta[key][order])
    # pressure pin: the interior point nearest the domain centre, ties -> lowest index
    d2 = ((xyz - np.asarray(centre)) ** 2).sum(axis=1)
    d2 = np.where(kind == INTERIOR, d2, np.inf)
    pin = int(np.lexsort((np.arange(len(d2)), d2))[0])
    if ((kind == PRESCRIBED_PRESSURE) | (kind == OUTLET)).any():
        pin = -1   # the prescribed boundary pressure fixes the pressure level
    return Cloud(dim=dim, xyz=xyz, kind=kind, normal=normal, pin=pin, name=name, h=h, meta=meta,
                 period=tuple(period))


def _square_perimeter(lo, hi, per_edge):
    """Evenly spaced points on the square's edges, each edge starting at a corner
    (all four corners included once), counter-clockwise, with outward normals;
    a corner's normal is the normalised sum of its two edge normals."""
    L = hi - lo
    s = np.arange(per_edge) * (L / per_edge)
    pts, nrm = [], []
    edges = [((lo, lo), (1, 0), (0, -1)), ((hi, lo), (0, 1), (1, 0)),
             ((hi, hi), (-1, 0), (0, 1)), ((lo, hi), (0, -1), (-1, 0))]
    for (cx, cy), (tx, ty), (nx, ny) in edges:
        px = cx + tx * s
        py = cy + ty * s
        pts.append(np.stack([px, py], axis=1))
        nrm.append(np.tile(np.array([nx, ny], dtype=np.float64), (per_edge, 1)))
    pts = np.concatenate(pts)
    nrm = np.concatenate(nrm)
    # corners: the first point of each edge
    c = 1.0 / np.sqrt(2.0)
    corner_n = [(-c, -c), (c, -c), (c, c), (-c, c)]
    for e in range(4):
        nrm[e * per_edge] = corner_n[e]
    return pts, nrm


# --------------------------------------------------------------------------
# clouds
# --------------------------------------------------------------------------

def kovasznay_square(nx: int = 40, seed: int = 1, jitter: float = 0.2, Re: float = 40.0,
                     lo: float = -0.5, hi: float = 1.5, boundary_kind: int = DIRICHLET) -> Cloud:
    """Kovasznay flow on [lo, hi]^2: a cell-centred nx-by-nx interior lattice with each
    coordinate jittered by U(-jitter*h, jitter*h), plus 4*nx boundary points at spacing h."""
    rng = np.random.default_rng(seed)
    h = (hi - lo) / nx
    g = lo + (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1)
    inter = inter + rng.uniform(-jitter * h, jitter * h, size=inter.shape)
    bpts, bnrm = _square_perimeter(lo, hi, nx)
    xyz = np.concatenate([inter, bpts])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.ones(len(bpts), np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), bnrm])
    return _finish(2, xyz, kind, normal, f"kovasznay_{nx}", h,
                   {"flow": "kovasznay", "Re": Re, "nu": 1.0 / Re, "seed": seed},
                   centre=((lo + hi) / 2, (lo + hi) / 2), boundary_kind=boundary_kind)


def poisson_disk(rng, lo, hi, r, rounds=24):
    """Dart throwing on a background grid of cell size r/sqrt(2) (at most one point
    per cell). Cells are visited in 9 interleaved classes so that proposals made
    together are never closer than r to each other; each round offers every empty
    cell one uniform proposal, accepted when no existing point lies within r."""
    a = r / np.sqrt(2.0)
    G = int(np.ceil((hi - lo) / a))
    ox = np.full((G + 4, G + 4), np.nan)
    oy = np.full((G + 4, G + 4), np.nan)
    r2 = r * r
    offs = [(di, dj) for di in range(-2, 3) for dj in range(-2, 3) if (di, dj) != (0, 0)]
    cls = []
    for ci in range(3):
        for cj in range(3):
            I, J = np.meshgrid(np.arange(ci, G, 3), np.arange(cj, G, 3), indexing="ij")
            cls.append((I.ravel(), J.ravel()))
    for _ in range(rounds):
        for I0, J0 in cls:
            m = np.isnan(ox[I0 + 2, J0 + 2])
            I, J = I0[m], J0[m]
            px = lo + (I + rng.random(I.size)) * a
            py = lo + (J + rng.random(J.size)) * a
            ok = (px < hi) & (py < hi)
            for di, dj in offs:
                nx_ = ox[I + 2 + di, J + 2 + dj]
                ny_ = oy[I + 2 + di, J + 2 + dj]
                with np.errstate(invalid="ignore"):
                    ok &= ~(((px - nx_) ** 2 + (py - ny_) ** 2) < r2)
            ox[I[ok] + 2, J[ok] + 2] = px[ok]
            oy[I[ok] + 2, J[ok] + 2] = py[ok]
    m = ~np.isnan(ox)
    return np.stack([ox[m], oy[m]], axis=1)


# Radius giving 250,000 +- 0.5% points in [0, 2*pi]^2 with seed 2 and 24 rounds
# (found by bisection on the point count).
TG_RADIUS_250K = 0.01025


def taylor_green_disk(r: float = TG_RADIUS_250K, seed: int = 2, nu: float = 0.01,
                      rounds: int = 24, boundary_kind: int = PRESCRIBED_PRESSURE) -> Cloud:
    """Taylor-Green vortex on [0, 2*pi]^2: Poisson-disk interior of radius r (interior
    points closer than r/2 to the boundary dropped) and boundary points at spacing ~r."""
    rng = np.random.default_rng(seed)
    lo, hi = 0.0, 2.0 * np.pi
    inter = poisson_disk(rng, lo, hi, r, rounds)
    keep = ((inter[:, 0] > lo + r / 2) & (inter[:, 0] < hi - r / 2)
            & (inter[:, 1] > lo + r / 2) & (inter[:, 1] < hi - r / 2))
    inter = inter[keep]
    per_edge = int(round((hi - lo) / r))
    bpts, bnrm = _square_perimeter(lo, hi, per_edge)
    xyz = np.concatenate([inter, bpts])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.ones(len(bpts), np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), bnrm])
    return _finish(2, xyz, kind, normal, f"taylor_green_{len(xyz)}", r,
                   {"flow": "taylor_green", "nu": nu, "seed": seed},
                   centre=(np.pi, np.pi), boundary_kind=boundary_kind)


def _edge_points(x0, y0, x1, y1, count, nrm, include_end=False):
    """count evenly spaced points from (x0, y0) towards (x1, y1) (the end point
    only with include_end), all with normal nrm."""
    s = np.arange(count + (1 if include_end else 0)) / count
    pts = np.stack([x0 + (x1 - x0) * s, y0 + (y1 - y0) * s], axis=1)
    return pts, np.tile(np.asarray(nrm, dtype=np.float64), (len(pts), 1))


def symmetric_square(nx: int = 16, seed: int = 17, jitter: float = 0.2) -> Cloud:
    """Unit square for the stagnation flow u = (x, -y): a symmetry plane on
    y = 0 (normal (0, -1), corners excluded) and velocity-Dirichlet points on the
    other three edges (corners included)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / nx
    g = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1) + rng.uniform(-jitter * h, jitter * h, size=(nx * nx, 2))
    sym, sym_n = _edge_points(h, 0.0, 1.0, 0.0, nx - 1, (0.0, -1.0))     # x = h .. 1-h
    sym = sym[: nx - 1]
    sym_n = sym_n[: nx - 1]
    right, rn = _edge_points(1.0, 0.0, 1.0, 1.0, nx, (1.0, 0.0))
    top, tn = _edge_points(1.0, 1.0, 0.0, 1.0, nx, (0.0, 1.0))
    left, ln = _edge_points(0.0, 1.0, 0.0, 0.0, nx, (-1.0, 0.0))
    xyz = np.concatenate([inter, sym, right, top, left])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(len(sym), SYMMETRY, np.uint8),
                           np.full(len(right) + len(top) + len(left), DIRICHLET, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), sym_n, rn, tn, ln])
    return _finish(2, xyz, kind, normal, f"symmetric_square_{len(xyz)}", h, {"flow": "stagnation", "nu": 0.05},
                   centre=(0.5, 0.5), boundary_kind=None)


def kovasznay_strip(nx: int = 40, ny: int = 10, seed: int = 19, jitter: float = 0.2, Re: float = 40.0) -> Cloud:
    """Kovasznay flow on [-0.5, 1.5] x [0, 0.5]: both y = 0 and y = 0.5 are
    symmetry lines of the flow (v = 0, du/dy = 0), so they carry symmetry
    points (corners excluded); inlet and outlet edges are velocity-Dirichlet."""
    rng = np.random.default_rng(seed)
    hx, hy = 2.0 / nx, 0.5 / ny
    gx = -0.5 + (np.arange(nx) + 0.5) * hx
    gy = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1)
    inter = inter + np.stack([rng.uniform(-jitter * hx, jitter * hx, len(inter)),
                              rng.uniform(-jitter * hy, jitter * hy, len(inter))], axis=1)
    bot, bn = _edge_points(-0.5 + hx, 0.0, 1.5, 0.0, nx - 1, (0.0, -1.0))
    top, tn = _edge_points(1.5 - hx, 0.5, -0.5, 0.5, nx - 1, (0.0, 1.0))
    bot, bn, top, tn = bot[: nx - 1], bn[: nx - 1], top[: nx - 1], tn[: nx - 1]
    inl, iln = _edge_points(-0.5, 0.5, -0.5, 0.0, ny, (-1.0, 0.0), include_end=True)
    outl, oln = _edge_points(1.5, 0.0, 1.5, 0.5, ny, (1.0, 0.0), include_end=True)
    xyz = np.concatenate([inter, bot, top, inl, outl])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(len(bot) + len(top), SYMMETRY, np.uint8),
                           np.full(len(inl) + len(outl), DIRICHLET, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), bn, tn, iln, oln])
    return _finish(2, xyz, kind, normal, f"kovasznay_strip_{len(xyz)}", min(hx, hy),
                   {"flow": "kovasznay", "Re": Re, "nu": 1.0 / Re, "seed": seed},
                   centre=(0.5, 0.25), boundary_kind=None)


def periodic_channel(nx: int = 32, ny: int = 16, length: float = 2.0, seed: int = 29, jitter: float = 0.2,
                     nu: float = 0.01, U: float = 1.0) -> Cloud:
    """Channel periodic in x (period `length`) between walls y = 0 and y = 1,
    for Poiseuille flow driven by the body force 8 nu U e_x instead of a
    pressure gradient (meta["force"]); the pressure is then constant. A
    jittered cell-centred lattice and wall points at the cell centres of x."""
    rng = np.random.default_rng(seed)
    hx, hy = length / nx, 1.0 / ny
    gx = (np.arange(nx) + 0.5) * hx
    gy = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1)
    inter = inter + np.stack([rng.uniform(-jitter * hx, jitter * hx, len(inter)),
                              rng.uniform(-jitter * hy, jitter * hy, len(inter))], axis=1)
    walls = np.concatenate([np.stack([gx, np.zeros_like(gx)], 1), np.stack([gx, np.ones_like(gx)], 1)])
    wn = np.concatenate([np.tile([0.0, -1.0], (nx, 1)), np.tile([0.0, 1.0], (nx, 1))])
    xyz = np.concatenate([inter, walls])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(len(walls), DIRICHLET, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), wn])
    return _finish(2, xyz, kind, normal, f"periodic_channel_{len(xyz)}", min(hx, hy),
                   {"flow": "poiseuille_forced", "U": U, "nu": nu, "seed": seed, "force": (8.0 * nu * U, 0.0, 0.0)},
                   centre=(length / 2, 0.5), boundary_kind=None, period=(length, 0.0, 0.0))


def taylor_green_periodic(nx: int = 48, seed: int = 23, jitter: float = 0.2, nu: float = 0.01) -> Cloud:
    """The Taylor-Green vortex on the periodic square [0, 2 pi)^2 (period 2 pi
    in x and y, no boundary points): a cell-centred nx-by-nx lattice, each
    coordinate jittered by U(-jitter h, jitter h)."""
    rng = np.random.default_rng(seed)
    L = 2.0 * np.pi
    h = L / nx
    g = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel()], axis=1) + rng.uniform(-jitter * h, jitter * h, size=(nx * nx, 2))
    kind = np.zeros(len(xyz), np.uint8)
    return _finish(2, xyz, kind, np.zeros_like(xyz), f"taylor_green_periodic_{len(xyz)}", h,
                   {"flow": "taylor_green", "nu": nu, "seed": seed}, centre=(np.pi, np.pi), boundary_kind=None,
                   period=(L, L, 0.0))


def poiseuille_channel(nx: int = 48, ny: int = 16, length: float = 3.0, seed: int = 13, jitter: float = 0.2,
                       nu: float = 0.01) -> Cloud:
    """Channel [0, length] x [0, 1] for plane Poiseuille flow: a jittered
    cell-centred nx-by-ny lattice, Dirichlet velocity on the inlet x = 0 and the
    walls y = 0, 1 (corners included, with their wall normals), and an outlet
    (kind OUTLET, outward normal +x) on x = length between the walls."""
    rng = np.random.default_rng(seed)
    hx, hy = length / nx, 1.0 / ny
    gx = (np.arange(nx) + 0.5) * hx
    gy = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1)
    inter = inter + np.stack([rng.uniform(-jitter * hx, jitter * hx, len(inter)),
                              rng.uniform(-jitter * hy, jitter * hy, len(inter))], axis=1)
    wx = np.arange(nx + 1) * hx                      # wall points, corners included
    walls = np.concatenate([np.stack([wx, np.zeros_like(wx)], 1), np.stack([wx, np.ones_like(wx)], 1)])
    wn = np.concatenate([np.tile([0.0, -1.0], (nx + 1, 1)), np.tile([0.0, 1.0], (nx + 1, 1))])
    ey = gy                                           # inlet and outlet points between the walls
    inlet = np.stack([np.zeros_like(ey), ey], 1)
    outlet = np.stack([np.full_like(ey, length), ey], 1)
    xyz = np.concatenate([inter, walls, inlet, outlet])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(len(walls), DIRICHLET, np.uint8),
                           np.full(len(inlet), DIRICHLET, np.uint8), np.full(len(outlet), OUTLET, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), wn, np.tile([-1.0, 0.0], (len(inlet), 1)),
                             np.tile([1.0, 0.0], (len(outlet), 1))])
    return _finish(2, xyz, kind, normal, f"poiseuille_{len(xyz)}", min(hx, hy),
                   {"flow": "poiseuille", "U": 1.0, "nu": nu, "seed": seed},
                   centre=(length / 2, 0.5), boundary_kind=None)


# Poisson-disk radii giving the three point counts of the Couette study (2080,
# 4033 and 8078 points in total, within 1%, seed 11; found by bisection): 2086,
# 4046 and 8069 points.
COUETTE_RADII = {2080: 0.028959, 4033: 0.020455, 8078: 0.014289}


def couette_annulus(r: float, seed: int = 11, r1: float = 0.5, r2: float = 1.0, omega: float = 2.0,
                    Re: float = 100.0, rounds: int = 24, boundary_kind: int = DIRICHLET) -> Cloud:
    """Annulus r1 <= |x| <= r2 for cylindrical Couette flow: a Poisson-disk
    interior of radius r (points closer than r/2 to either circle dropped) and
    evenly spaced points at spacing ~r on both circles, with outward normals
    (into the inner cylinder on the inner circle). Re = (2 r1)(omega r1) / nu."""
    rng = np.random.default_rng(seed)
    pts = poisson_disk(rng, -r2, r2, r, rounds)
    rad = np.sqrt((pts ** 2).sum(axis=1))
    inter = pts[(rad > r1 + r / 2) & (rad < r2 - r / 2)]
    bp, bn = [], []
    for rc, sgn in ((r1, -1.0), (r2, 1.0)):
        m = int(round(2 * np.pi * rc / r))
        th = 2 * np.pi * np.arange(m) / m
        c, s_ = np.cos(th), np.sin(th)
        bp.append(np.stack([rc * c, rc * s_], axis=1))
        bn.append(sgn * np.stack([c, s_], axis=1))
    bpts = np.concatenate(bp)
    bnrm = np.concatenate(bn)
    xyz = np.concatenate([inter, bpts])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.ones(len(bpts), np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), bnrm])
    nu = (2 * r1) * (omega * r1) / Re
    return _finish(2, xyz, kind, normal, f"couette_{len(xyz)}", r,
                   {"flow": "couette", "r1": r1, "r2": r2, "omega": omega, "Re": Re, "nu": nu, "seed": seed},
                   centre=(0.5 * (r1 + r2), 0.0), boundary_kind=boundary_kind)


def beltrami_cube(n: int = 100, seed: int = 4, jitter: float = 0.2, nu: float = 0.01,
                  boundary_kind: int = PRESCRIBED_PRESSURE) -> Cloud:
    """Ethier-Steinman flow on [0,1]^3: a cell-centred n^3 lattice jittered by
    U(-jitter*h, jitter*h) per coordinate, plus the cell-centred n^2 lattice of each
    of the six faces (no edge or corner points)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    inter = inter + rng.uniform(-jitter * h, jitter * h, size=inter.shape)
    A, B = np.meshgrid(g, g, indexing="ij")
    A = A.ravel()
    B = B.ravel()
    zero = np.zeros_like(A)
    one = np.ones_like(A)
    faces, fn = [], []
    for axis in range(3):
        for side, val in ((-1.0, zero), (1.0, one)):
            cols = [A, B]
            cols.insert(axis, val)
            faces.append(np.stack(cols, axis=1))
            nn = np.zeros((len(A), 3))
            nn[:, axis] = side
            fn.append(nn)
    bpts = np.concatenate(faces)
    bnrm = np.concatenate(fn)
    xyz = np.concatenate([inter, bpts])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.ones(len(bpts), np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), bnrm])
    return _finish(3, xyz, kind, normal, f"beltrami_{n}", h,
                   {"flow": "beltrami", "nu": nu, "seed": seed}, centre=(0.5, 0.5, 0.5),
                   boundary_kind=boundary_kind)


def holed_square(n_target: int, seed: int, n_holes: int | None = None, Re: float = 40.0,
                 jitter: float = 0.2, edge_kind: int = DIRICHLET, hole_kind: int = DIRICHLET) -> Cloud:
    """Unit square minus 0-4 circular holes (radius U(0.05, 0.15), centre in
    [r+0.05, 1-r-0.05]^2, kept 0.05 apart). Jittered lattice interior with spacing h
    chosen to approach n_target points; points inside a hole or within h/2 of it are
    removed; hole boundaries carry points at spacing ~h with normals pointing into
    the hole (outward from the fluid). Kovasznay data on the square's edges and
    no-slip on the holes."""
    rng = np.random.default_rng(seed)
    nh = int(rng.integers(0, 5)) if n_holes is None else n_holes
    holes = []
    tries = 0
    while len(holes) < nh and tries < 1000:
        tries += 1
        r = rng.uniform(0.05, 0.15)
        c = rng.uniform(r + 0.05, 1 - r - 0.05, size=2)
        if all(np.hypot(*(c - c2)) > r + r2 + 0.05 for c2, r2 in holes):
            holes.append((c, r))
    area = 1.0 - sum(np.pi * r * r for _, r in holes)
    h = np.sqrt(area / n_target)
    nx = max(4, int(round(1.0 / h)))
    h = 1.0 / nx
    g = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1)
    inter = inter + rng.uniform(-jitter * h, jitter * h, size=inter.shape)
    keep = np.ones(len(inter), bool)
    hp, hn = [], []
    for c, r in holes:
        keep &= np.hypot(inter[:, 0] - c[0], inter[:, 1] - c[1]) > r + h / 2
        m = max(8, int(round(2 * np.pi * r / h)))
        th = np.arange(m) * (2 * np.pi / m)
        hp.append(np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], axis=1))
        hn.append(np.stack([-np.cos(th), -np.sin(th)], axis=1))
    inter = inter[keep]
    bpts, bnrm = _square_perimeter(0.0, 1.0, nx)
    parts = [inter, bpts] + hp
    xyz = np.concatenate(parts)
    n_hole_pts = sum(len(p) for p in hp)
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(len(bpts), edge_kind, np.uint8),
                           np.full(n_hole_pts, hole_kind, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), bnrm] + hn)
    on_hole = np.concatenate([np.zeros(len(inter) + len(bpts), bool), np.ones(n_hole_pts, bool)])
    return _finish(2, xyz, kind, normal, f"holed_{len(xyz)}_{seed}", h,
                   {"flow": "kovasznay_holes", "Re": Re, "nu": 1.0 / Re, "seed": seed,
                    "holes": [(float(c[0]), float(c[1]), float(r)) for c, r in holes],
                    "on_hole": on_hole},
                   centre=(0.5, 0.5), boundary_kind=None)


def periodic_cylinder_cell(nx: int = 48, radius: float = 0.2, seed: int = 31, jitter: float = 0.2) -> Cloud:
    """One cell of a periodic array of cylinders: the unit square, periodic in
    x and y, minus a circle of the given radius at (0.5, 0.5). A cell-centred
    nx-by-nx lattice jittered by U(-jitter h, jitter h), points within h/2 of
    the circle removed, the circle carrying points at spacing ~h with normals
    pointing into it (out of the fluid), no-slip there."""
    rng = np.random.default_rng(seed)
    h = 1.0 / nx
    g = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel()], axis=1) + rng.uniform(-jitter * h, jitter * h, size=(nx * nx, 2))
    inter = inter[np.hypot(inter[:, 0] - 0.5, inter[:, 1] - 0.5) > radius + h / 2]
    m = max(8, int(round(2 * np.pi * radius / h)))
    th = np.arange(m) * (2 * np.pi / m)
    circ = np.stack([0.5 + radius * np.cos(th), 0.5 + radius * np.sin(th)], axis=1)
    xyz = np.concatenate([inter, circ])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(m, DIRICHLET, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), -np.stack([np.cos(th), np.sin(th)], axis=1)])
    return _finish(2, xyz, kind, normal, f"periodic_cylinder_{len(xyz)}", h,
                   {"seed": seed, "holes": [(0.5, 0.5, float(radius))]}, centre=(0.0, 0.0), boundary_kind=None,
                   period=(1.0, 1.0, 0.0))


def rotated(cloud: Cloud, angle: float, axis=(0.0, 0.0, 1.0)) -> Cloud:
    """A cloud turned by `angle` (radians) about the origin (2D) or about
    `axis` through the origin (3D, Rodrigues' formula): coordinates and
    normals rotated, kinds kept, the pressure pin moved with its point. Its
    symmetry planes then lie off the coordinate axes, and flow_fields gives
    the rotated flow."""
    c, s = np.cos(angle), np.sin(angle)
    if cloud.dim == 2:
        rot = np.array([[c, -s], [s, c]])
    else:
        k = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
        K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
        rot = np.eye(3) + s * K + (1.0 - c) * (K @ K)
    xyz = cloud.xyz @ rot.T
    normal = cloud.normal @ rot.T
    centre = tuple(xyz[cloud.pin]) if cloud.pin >= 0 else (0.0,) * cloud.dim
    meta = dict(cloud.meta)
    meta["rotation"] = rot.tolist()
    return _finish(cloud.dim, xyz, cloud.kind, normal, f"{cloud.name}_rot", cloud.h, meta, centre=centre,
                   boundary_kind=None)


def symmetric_cube(n: int = 7, seed: int = 37, jitter: float = 0.2, face_kind: int = PRESCRIBED_PRESSURE) -> Cloud:
    """Unit cube for the 3D stagnation flow u = (x, y, -2z): a symmetry plane on
    z = 0 (normal (0, 0, -1), its edges excluded) and points of `face_kind` on
    the other five faces (edges included): by default prescribed pressure, so
    that p' is fixed there and the step's pressure system stays well posed
    when its right-hand side is rounding noise."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    inter = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + rng.uniform(-jitter * h, jitter * h,
                                                                              size=(n ** 3, 3))
    f = np.linspace(0.0, 1.0, n + 1)
    A, B = np.meshgrid(f, f, indexing="ij")
    A, B = A.ravel(), B.ravel()
    inner = (A > 0) & (A < 1) & (B > 0) & (B < 1)
    sym = np.stack([A[inner], B[inner], np.zeros(inner.sum())], axis=1)
    faces, fn = [], []
    seen = set()
    for ax in range(3):
        for val in (0.0, 1.0):
            if ax == 2 and val == 0.0:
                continue
            for a, b in zip(A, B):
                pt = [a, b]
                pt.insert(ax, val)
                key = tuple(np.round(pt, 12))
                if key in seen:   # edges and corners shared by two or three faces
                    continue
                seen.add(key)
                faces.append(pt)
                nv = [0.0, 0.0, 0.0]
                nv[ax] = 1.0 if val == 1.0 else -1.0
                fn.append(nv)
    faces, fn = np.array(faces), np.array(fn)
    xyz = np.concatenate([inter, sym, faces])
    kind = np.concatenate([np.zeros(len(inter), np.uint8), np.full(len(sym), SYMMETRY, np.uint8),
                           np.full(len(faces), face_kind, np.uint8)])
    normal = np.concatenate([np.zeros_like(inter), np.tile([0.0, 0.0, -1.0], (len(sym), 1)), fn])
    return _finish(3, xyz, kind, normal, f"symmetric_cube_{len(xyz)}", h, {"flow": "stagnation", "nu": 0.05},
                   centre=(0.5, 0.5, 0.5), boundary_kind=None)


def scattered_square(nx: int, seed: int = 7, jitter: float = 0.2, lo: float = 0.0,
                     hi: float = 1.0) -> Cloud:
    """A jittered nx-by-nx lattice on [lo, hi]^2 with boundary points (no flow attached);
    used for operator-accuracy studies."""
    c = kovasznay_square(nx=nx, seed=seed, jitter=jitter, lo=lo, hi=hi)
    c.meta = {"seed": seed}
    c.name = f"square_{nx}"
    return c


def scattered_cube(n: int, seed: int = 9, jitter: float = 0.2, boundary_kind: int = DIRICHLET) -> Cloud:
    c = beltrami_cube(n=n, seed=seed, jitter=jitter, boundary_kind=boundary_kind)
    c.meta = {"flow": "beltrami", "nu": 0.01, "seed": seed}
    c.name = f"cube_{n}"
    return c


def config_c3_sizes(count: int = 256, seed: int = 1000):
    """Per-instance (n_target, seed, poly_degree) of the 256-instance batch: sizes
    log-uniform over 500-50k, degree uniform over 2..5."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n = int(round(np.exp(rng.uniform(np.log(500), np.log(50_000)))))
        k = int(rng.integers(2, 6))
        out.append((n, seed + i, k))
    return out
