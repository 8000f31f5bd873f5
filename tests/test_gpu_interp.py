"""Off-node interpolation through the C ABI (rbffd_interpolate) against the
FP64 oracle: clouds bit-exact, weights within 1e-10 (row-relative), values
within 1e-12 of the oracle's weights applied to the same fields; degree-k
polynomials reproduced; a query on a node returns the nodal value."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2106_07616_amd as R  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


CASES = {
    # the centre line of the Kovasznay square (the paper's profile plots)
    "kovasznay40_k3": (lambda: W.kovasznay_square(nx=40), 3),
    "tg_disk_k4": (lambda: W.taylor_green_disk(r=0.06), 4),
    "couette2080_k6": (lambda: W.couette_annulus(W.COUETTE_RADII[2080]), 6),   # 84 unknowns
    "cube9_k2": (lambda: W.beltrami_cube(n=9), 2),
    "cube9_k4": (lambda: W.beltrami_cube(n=9), 4),                               # 105 unknowns
}


def _queries(c, rng):
    lo, hi = c.xyz.min(0), c.xyz.max(0)
    mid = 0.5 * (lo + hi)
    line = np.repeat(mid[None, :], 100, axis=0)
    line[:, 0] = np.linspace(lo[0] + 0.01 * (hi[0] - lo[0]), hi[0] - 0.01 * (hi[0] - lo[0]), 100)
    if c.meta.get("flow") == "couette":   # the radial line y = 0, x in [r1, r2]
        line[:, 1] = 0.0
        line[:, 0] = np.linspace(0.51, 0.99, 100)
    scat = lo + (hi - lo) * rng.uniform(0.05, 0.95, size=(60, c.dim))
    if c.meta.get("flow") == "couette":
        r = rng.uniform(0.52, 0.98, 60)
        th = rng.uniform(0, 2 * np.pi, 60)
        scat = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    return np.concatenate([line, scat, c.xyz[[3, c.n // 2]]])   # two queries on nodes


@pytest.mark.parametrize("name", list(CASES))
def test_interpolation_parity(ctx, orc, name):
    gen, k = CASES[name]
    c = gen()
    pts = _queries(c, np.random.default_rng(21))
    vel, p = W.flow_fields(c) if "flow" in c.meta else (None, None)
    fields = np.concatenate([vel, p[None, :]]) if vel is not None else np.sin(c.xyz[:, :1].T)
    dc = R.DeviceCloud.from_numpy(c)
    out, nbr, w = R.rbffd_interpolate(ctx, dc, k, torch.tensor(pts, device="cuda"),
                                      torch.tensor(fields, device="cuda"), return_stencils=True)
    vo, nbr_o, w_o = orc.interpolate(c.xyz, k, pts, fields)
    np.testing.assert_array_equal(nbr.cpu().numpy(), nbr_o)
    wg = w.cpu().numpy()
    werr = float((np.abs(wg - w_o).max(1) / np.abs(w_o).max(1)).max())
    og = out.cpu().numpy()
    verr = float(np.abs(og - vo).max() / np.abs(vo).max())
    print(f"[interp] {name}: nq={len(pts)} q={nbr.shape[1]} weights {werr:.1e} values {verr:.1e}", flush=True)
    assert werr <= 1e-10
    assert verr <= 1e-12
    # queries on nodes return the nodal values
    np.testing.assert_allclose(og[:, -2:], fields[:, [3, c.n // 2]], rtol=1e-10,
                               atol=1e-12 * np.abs(fields).max())
    # against the exact flow on the sampled points (discretization error only)
    if vel is not None and c.meta.get("flow") != "taylor_green":
        ue, pe = W.flow_fields(W.Cloud(dim=c.dim, xyz=pts, kind=np.zeros(len(pts), np.uint8),
                                       normal=np.zeros_like(pts), pin=-1, meta=c.meta))
        du = float(np.abs(og[:c.dim] - ue).max() / np.abs(ue).max())
        print(f"[interp] {name}: max velocity error vs the closed form {du:.1e}", flush=True)
        assert du <= 1e-3


@pytest.mark.parametrize("dim,k", [(2, 3), (3, 3)])
def test_interpolation_reproduces_polynomials(ctx, dim, k):
    c = W.kovasznay_square(nx=20) if dim == 2 else W.scattered_cube(9, seed=5)
    rng = np.random.default_rng(5)
    lo, hi = c.xyz.min(0), c.xyz.max(0)
    pts = lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(200, dim))
    import itertools
    ex = [np.array(e) for e in itertools.product(range(k + 1), repeat=dim) if sum(e) <= k]
    coef = rng.standard_normal(len(ex))
    poly = lambda x: sum(cf * np.prod(x ** e, axis=1) for cf, e in zip(coef, ex))
    out = R.rbffd_interpolate(ctx, R.DeviceCloud.from_numpy(c), k, torch.tensor(pts, device="cuda"),
                              torch.tensor(poly(c.xyz), device="cuda"))
    ref = poly(pts)
    assert float(np.abs(out.cpu().numpy()[0] - ref).max()) <= 1e-9 * np.abs(ref).max()


def test_interpolation_edge_cases(ctx):
    c = W.kovasznay_square(nx=12)
    dc = R.DeviceCloud.from_numpy(c)
    f = torch.tensor(c.xyz[:, 0].copy(), device="cuda")
    # no query points: a no-op
    out = R.rbffd_interpolate(ctx, dc, 2, torch.zeros((0, 2), dtype=torch.float64, device="cuda"), f)
    assert out.shape == (1, 0)
    # weights only (no fields)
    out, nbr, w = R.rbffd_interpolate(ctx, dc, 2, torch.tensor([[0.3, 0.4]], dtype=torch.float64, device="cuda"), None,
                                      return_stencils=True)
    assert out is None and abs(float(w.sum()) - 1.0) < 1e-12    # the constant is reproduced
    # a query outside the cloud's bounding box still finds its exact neighbours
    far = np.array([[3.0, -2.0]])
    _, nbr, _ = R.rbffd_interpolate(ctx, dc, 2, torch.tensor(far, device="cuda"), None, return_stencils=True)
    np.testing.assert_array_equal(nbr.cpu().numpy(), __import__("oracle").knn_points(c.xyz, nbr.shape[1], far))
    # argument errors through the C ABI
    import ctypes as C
    L = R.lib()
    o = R.binding.StencilOptsT(3, 2, 0)
    cs = dc.struct()
    bad = C.c_int64()
    assert L.rbffd_interpolate(ctx.handle, C.byref(cs), C.byref(o), -1, None, 0, None, None, None, None,
                               C.byref(bad), R.binding._stream()) == -1
    q1 = torch.tensor([[0.3, 0.4]], dtype=torch.float64, device="cuda")
    assert L.rbffd_interpolate(ctx.handle, C.byref(cs), C.byref(o), 1, R.binding._ptr(q1), 1, None, None, None,
                               None, C.byref(bad), R.binding._stream()) == -1      # fields missing
    # non-finite query coordinates are rejected before any search
    for bad_q in (np.nan, np.inf):
        qn = torch.tensor([[0.3, bad_q]], dtype=torch.float64, device="cuda")
        assert L.rbffd_interpolate(ctx.handle, C.byref(cs), C.byref(o), 1, R.binding._ptr(qn), 0, None, None, None,
                                   None, C.byref(bad), R.binding._stream()) == -1
    o7 = R.binding.StencilOptsT(3, 7, 0)
    assert L.rbffd_interpolate(ctx.handle, C.byref(cs), C.byref(o7), 1, R.binding._ptr(q1), 0, None, None, None,
                               None, C.byref(bad), R.binding._stream()) == -1      # degree 7


@pytest.mark.parametrize("dim,k,q", [(2, 5, 59), (2, 6, 68), (3, 4, 61), (3, 4, 90)])
def test_interpolation_system_sizes(ctx, orc, dim, k, q):
    """Interpolation weights (one right-hand side) through the register
    Gauss-Jordan kernel's tile shapes 5 x 6 (80 + 1 unknowns), 6 x 7 (96 + 1,
    2D and 3D) and 8 x 8 (125 + 1): clouds bit-exact with the oracle, weights
    within 1e-10 row-relative, values within 1e-12."""
    c = W.kovasznay_square(nx=14) if dim == 2 else W.scattered_cube(8, seed=5)
    rng = np.random.default_rng(31)
    lo, hi = c.xyz.min(0), c.xyz.max(0)
    pts = lo + (hi - lo) * rng.uniform(0.05, 0.95, size=(40, dim))
    f = np.stack([np.sin(c.xyz[:, 0]) + c.xyz[:, 1] ** 2])
    vo, nbr_o, w_o = orc.interpolate(c.xyz, k, pts, f, q=q)
    out, nbr, w = R.rbffd_interpolate(ctx, R.DeviceCloud.from_numpy(c), k, torch.tensor(pts, device="cuda"),
                                      torch.tensor(f, device="cuda"), q=q, return_stencils=True)
    nbr, w, out = nbr.cpu().numpy(), w.cpu().numpy(), out.cpu().numpy()
    ew = float((np.abs(w - w_o).max(1) / np.abs(w_o).max(1)).max())
    ev = float(np.abs(out - vo).max())
    print(f"[interp] dim {dim} k {k} q {q}: weights {ew:.1e}, values {ev:.1e}", flush=True)
    np.testing.assert_array_equal(nbr, nbr_o)
    assert ew <= 1e-10 and ev <= 1e-12


@pytest.mark.parametrize("k", [4, 6])
def test_periodic_interpolation_matches_oracle(ctx, orc, k):
    """Interpolation on the periodic Taylor-Green square at points next to the
    seams and a period outside the box: clouds bit-exact with the oracle's
    (which searches all images), weights within 1e-10, values within 1e-12;
    k = 6 takes the 84-unknown LDS kernel."""
    c = W.taylor_green_periodic()
    L = c.period[0]
    rng = np.random.default_rng(8)
    m = 200
    pts = rng.uniform(0, L, size=(m, 2))
    pts[: m // 2, 0] = rng.uniform(-c.h, c.h, m // 2) % L           # next to the x seam
    pts[m // 2:, 1] = rng.uniform(-c.h, c.h, m - m // 2) % L
    pts[::7] += np.array([L, -L])                                   # outside the box
    f = np.stack([np.sin(c.xyz[:, 0]) * np.cos(c.xyz[:, 1]), np.cos(2 * c.xyz[:, 0])])
    vo, nbr_o, w_o = orc.interpolate(c.xyz, k, pts, f, period=c.period)
    dc = R.DeviceCloud.from_numpy(c, "cuda")
    out, nbr, w = R.rbffd_interpolate(ctx, dc, k, torch.tensor(pts, device="cuda"), torch.tensor(f, device="cuda"),
                                      return_stencils=True)
    nbr, w, out = nbr.cpu().numpy(), w.cpu().numpy(), out.cpu().numpy()
    ew = float((np.abs(w - w_o).max(1) / np.abs(w_o).max(1)).max())
    ev = float(np.abs(out - vo).max())
    ex = np.abs(out[0] - np.sin(pts[:, 0]) * np.cos(pts[:, 1])).max()
    print(f"[interp] periodic k={k}: weights {ew:.1e}, values {ev:.1e}, error vs the exact field {ex:.1e}", flush=True)
    np.testing.assert_array_equal(nbr, nbr_o)
    assert ew <= 1e-10 and ev <= 1e-12


def test_periodic_interpolation_period_too_small(ctx, orc):
    """A period too small for the cloud size (36 points, q = 34): a query's
    cloud would hold two images of one point. The library refuses with
    RBFFD_E_ARG, as the oracle refuses; q = 32 is accepted by both."""
    c = W.taylor_green_periodic(nx=6)
    pts = np.array([[0.1, 0.1], [3.0, 3.0]])
    with pytest.raises(ValueError):
        orc.interpolate(c.xyz, 3, pts, [np.ones(c.n)], q=34, period=c.period)
    dc = R.DeviceCloud.from_numpy(c, "cuda")
    ones = torch.ones((1, c.n), dtype=torch.float64, device="cuda")
    with pytest.raises(R.RbffdError) as e:
        R.rbffd_interpolate(ctx, dc, 3, torch.tensor(pts, device="cuda"), ones, q=34)
    assert e.value.code == -1
    out = R.rbffd_interpolate(ctx, dc, 3, torch.tensor(pts, device="cuda"), ones, q=32)
    np.testing.assert_allclose(out.cpu().numpy(), 1.0, rtol=0, atol=1e-12)
