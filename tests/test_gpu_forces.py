"""Drag and lift on a circular cylinder through the C ABI
(rbffd_cylinder_forces) against the FP64 oracle: force, coefficients and the
traction at every surface point, also in a periodic cylinder array. At any size, cubic velocity and quadratic
pressure fields give the divergence-theorem force pi R^2 (div sigma)(centre)."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2106_07616_amd as R  # noqa: E402

_CUBIC = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]


def _poly(coef, ex, X, Y, dx=0, dy=0):
    t = 0.0
    for cf, (i, j) in zip(coef, ex):
        if i < dx or j < dy:
            continue
        f = (math.factorial(i) // math.factorial(i - dx)) * (math.factorial(j) // math.factorial(j - dy))
        t = t + cf * f * X ** (i - dx) * Y ** (j - dy)
    return t


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


def _kovasznay(c):
    u, v, p = W.kovasznay(c.xyz[:, 0], c.xyz[:, 1], 40.0)
    return np.stack([u, v]), p


@pytest.mark.parametrize("k,nsurf", [(3, 360), (4, 360), (3, 6), (5, 98)])
def test_cylinder_forces_match_oracle(ctx, orc, k, nsurf):
    """Kovasznay flow past one hole of a 3000-point square: the force, C_D and
    C_L within 1e-10 of the oracle's (relative to the traction scale), the
    traction within 1e-9."""
    c = W.holed_square(3000, seed=5, n_holes=1)
    cx, cy, r = c.meta["holes"][0]
    vel, p = _kovasznay(c)
    mu, rho, U = 1.0 / 40.0, 1.0, 1.0
    print(f"[forces] n={c.n} k={k} nsurf={nsurf}", flush=True)
    ops_o = orc.build_operators(c, k)
    Fo, tro, co = orc.cylinder_forces(ops_o, vel, p, (cx, cy), 2 * r, mu, nsurf, rho=rho, u_ref=U)
    s = R.Solver(ctx, c, k)
    F, cf, tr = s.cylinder_forces(torch.tensor(vel, device="cuda"), torch.tensor(p, device="cuda"), (cx, cy), 2 * r,
                                  mu, nsurf, rho=rho, u_ref=U, return_traction=True)
    tr = tr.cpu().numpy()
    scale = np.abs(tro).max()
    print(f"[forces] F gpu {F} oracle {Fo}; traction diff {np.abs(tr - tro).max() / scale:.1e}", flush=True)
    assert np.abs(tr - tro).max() <= 1e-9 * scale
    assert np.abs(np.array(F) - Fo).max() <= 1e-10 * scale * 2 * math.pi * r
    assert np.abs(np.array(cf) - co).max() <= 1e-10 * scale * 2 * math.pi * r / (0.5 * rho * U * U * 2 * r)
    F2 = s.cylinder_forces(torch.tensor(vel, device="cuda"), torch.tensor(p, device="cuda"), (cx, cy), 2 * r, mu,
                           nsurf)
    assert F2 == F     # same bits run to run


@pytest.mark.parametrize("n_target", [3000, 250000])
def test_cylinder_forces_divergence_theorem(ctx, n_target):
    """Cubic velocity, quadratic pressure (reproduced exactly for k >= 3): the
    force is pi R^2 (div sigma)(centre) at any cloud size, here up to a
    250k-point square with one hole."""
    c = W.holed_square(n_target, seed=5, n_holes=1)
    cx, cy, r = c.meta["holes"][0]
    rng = np.random.default_rng(3)
    a, b, g = rng.standard_normal(10), rng.standard_normal(10), rng.standard_normal(6)
    X, Y = c.xyz[:, 0] - 0.5, c.xyz[:, 1] - 0.5
    u = np.stack([_poly(a, _CUBIC, X, Y), _poly(b, _CUBIC, X, Y)])
    p = _poly(g, _CUBIC[:6], X, Y)
    mu = 0.7
    print(f"[forces] divergence theorem n={c.n}", flush=True)
    s = R.Solver(ctx, c, 3)
    F = s.cylinder_forces(torch.tensor(u, device="cuda"), torch.tensor(p, device="cuda"), (cx, cy), 2 * r, mu)
    X0, Y0 = cx - 0.5, cy - 0.5
    div = np.array([
        -_poly(g, _CUBIC[:6], X0, Y0, 1, 0) + 2 * mu * _poly(a, _CUBIC, X0, Y0, 2, 0)
        + mu * (_poly(a, _CUBIC, X0, Y0, 0, 2) + _poly(b, _CUBIC, X0, Y0, 1, 1)),
        -_poly(g, _CUBIC[:6], X0, Y0, 0, 1) + 2 * mu * _poly(b, _CUBIC, X0, Y0, 0, 2)
        + mu * (_poly(a, _CUBIC, X0, Y0, 1, 1) + _poly(b, _CUBIC, X0, Y0, 2, 0))])
    Fcf = math.pi * r * r * div
    print(f"[forces] F {F} closed form {Fcf}", flush=True)
    # derivative weights on fine clouds lose digits as 1/h: a looser bar at 250k
    tol = 1e-10 if c.n < 10000 else 1e-8
    assert np.abs(np.array(F) - Fcf).max() <= tol * max(1.0, np.abs(Fcf).max())


def test_cylinder_forces_reject_bad_arguments(ctx):
    c = W.holed_square(3000, seed=5, n_holes=1)
    cx, cy, r = c.meta["holes"][0]
    s = R.Solver(ctx, c, 3)
    vel, p = _kovasznay(c)
    u = torch.tensor(vel, device="cuda")
    pt = torch.tensor(p, device="cuda")
    for kw in (dict(nsurf=7), dict(nsurf=2), dict(diameter=0.0), dict(diameter=float("nan")),
               dict(rho=0.0, u_ref=1.0), dict(rho=1.0, u_ref=0.0)):
        args = dict(centre=(cx, cy), diameter=2 * r, mu=0.025, nsurf=360)
        args.update(kw)
        with pytest.raises(R.RbffdError):
            s.cylinder_forces(u, pt, **args)
    cube = W.beltrami_cube(n=6)
    s3 = R.Solver(ctx, cube, 2)
    with pytest.raises(R.RbffdError):
        s3.cylinder_forces(torch.zeros((2, cube.n), dtype=torch.float64, device="cuda"),
                           torch.zeros(cube.n, dtype=torch.float64, device="cuda"), (0.5, 0.5), 0.2, 0.01)


@pytest.mark.parametrize("k", [3, 5])
def test_cylinder_forces_periodic_cell(ctx, orc, k):
    """One cell of a periodic cylinder array, with a smooth periodic flow: the
    force and the traction match the oracle's (1e-10 and 1e-9 of the traction
    scale)."""
    c = W.periodic_cylinder_cell()
    cx, cy, r = c.meta["holes"][0]
    x, y = 2 * np.pi * c.xyz[:, 0], 2 * np.pi * c.xyz[:, 1]
    vel = np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)])
    p = 0.25 * (np.cos(2 * x) + np.cos(2 * y))
    mu = 0.05
    Fo, tro = orc.cylinder_forces(orc.build_operators(c, k), vel, p, (cx, cy), 2 * r, mu, 360)
    s = R.Solver(ctx, c, k)
    F, tr = s.cylinder_forces(torch.tensor(vel, device="cuda"), torch.tensor(p, device="cuda"), (cx, cy), 2 * r, mu,
                              360, return_traction=True)
    tr = tr.cpu().numpy()
    scale = np.abs(tro).max()
    print(f"[forces] periodic cell k={k}: F gpu {F} oracle {Fo}; traction diff {np.abs(tr - tro).max() / scale:.1e}",
          flush=True)
    assert np.abs(tr - tro).max() <= 1e-9 * scale
    assert np.abs(np.array(F) - Fo).max() <= 1e-10 * scale * 2 * math.pi * r
