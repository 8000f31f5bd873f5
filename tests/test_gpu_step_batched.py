"""simple_step_batched: one time step of several clouds at once, each against
the oracle's step (Sec. 3, the step list of Sec. 3.2) and against itself
alone (bitwise: every batched Krylov system owns its blocks and reductions).
Clouds of different sizes, dimensions, degrees and boundary closures, each
with its own time step."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2106_07616_amd as R  # noqa: E402

PP = W.PRESCRIBED_PRESSURE


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


def _clouds():
    return [
        (W.kovasznay_square(nx=14, boundary_kind=PP), 3),
        (W.holed_square(1400, seed=1003, edge_kind=PP, hole_kind=PP), 2),
        (W.taylor_green_disk(r=0.09), 4),
        (W.beltrami_cube(7), 3),
        (W.kovasznay_square(nx=12), 2),   # velocity walls, Neumann p' and the boundary-pressure block
    ]


def _setup(ctx, clouds, rho=1.0, mu=0.025):
    items = []
    for c, k in clouds:
        s = R.Solver(ctx, c, k)
        vel, p = W.flow_fields(c)
        u0 = torch.tensor(vel, device="cuda")
        dt = 0.5 * s.dt_from_courant(u0, 1.0, rho, mu)
        items.append((c, k, s, vel, p, dt))
    return items


def _run_batched(ctx, items, idx, **kw):
    u, up, p, ub, pb, dts, ops = [], [], [], [], [], [], []
    for j in idx:
        c, k, s, vel, pres, dt = items[j]
        u.append(torch.tensor(vel, device="cuda"))
        up.append(torch.tensor(vel, device="cuda"))
        p.append(torch.tensor(pres, device="cuda"))
        ub.append(torch.tensor(vel, device="cuda"))
        pb.append(torch.tensor(pres, device="cuda") if (c.kind == PP).any() else None)
        dts.append(dt)
        ops.append(s.ops)
    st = R.simple_step_batched(ctx, ops, u, up, p, ub, 1.0, 0.025, dts, alpha=R.BDF1, p_bc=pb, **kw)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in u], [x.cpu().numpy() for x in p], st


def test_batched_step_matches_the_oracle_and_alone(ctx, orc):
    items = _setup(ctx, _clouds())
    kw = dict(tol_outer=0.0, tol_krylov=1e-12, max_outer=2, max_krylov=40000)
    u, p, st = _run_batched(ctx, items, range(len(items)), **kw)
    for j, (c, k, s, vel, pres, dt) in enumerate(items):
        ops_o = orc.build_operators(c, k)
        pb = pres if (c.kind == PP).any() else None
        uo, _, po, st_o = orc.simple_step(ops_o, vel, vel, pres, vel, 1.0, 0.025, dt, alpha=orc.BDF1, p_bc=pb, **kw)
        eu = float(np.abs(u[j] - uo).max() / np.abs(uo).max())
        ep = float(np.abs(p[j] - po).max() / max(np.abs(po).max(), 1e-300))
        print(f"[step batched] {c.name} k={k} n={c.n}: outer {st[j]['outer_iters']} status {st[j]['status']} "
              f"(oracle {st_o['status']}), u {eu:.1e} p {ep:.1e}", flush=True)
        assert st[j]["outer_iters"] == 2
        if st_o["status"] == 0 and st[j]["status"] == 0:
            assert eu <= 1e-8 and ep <= 1e-8
        # alone equals in the batch
        ua, pa, sa = _run_batched(ctx, items, [j], **kw)
        np.testing.assert_array_equal(ua[0], u[j])
        np.testing.assert_array_equal(pa[0], p[j])
        assert sa[0] == st[j]


def test_batched_step_outer_tolerance_per_cloud(ctx):
    """With the outer tolerance of Sec. 3.2 each cloud stops on its own Delta:
    the iteration counts are the single-cloud step's, and the fields agree with
    simple_step to the Krylov tolerance."""
    items = _setup(ctx, _clouds()[:4])
    kw = dict(tol_outer=1e-7, tol_krylov=1e-11, max_outer=30, max_krylov=40000)
    u, p, st = _run_batched(ctx, items, range(len(items)), **kw)
    for j, (c, k, s, vel, pres, dt) in enumerate(items):
        u1 = torch.tensor(vel, device="cuda")
        p1 = torch.tensor(pres, device="cuda")
        pb = torch.tensor(pres, device="cuda") if (c.kind == PP).any() else None
        s1 = R.simple_step(ctx, s.ops, u1, u1.clone(), p1, torch.tensor(vel, device="cuda"), 1.0, 0.025, dt,
                           alpha=R.BDF1, p_bc=pb, **kw)
        eu = float(np.abs(u[j] - u1.cpu().numpy()).max() / np.abs(u1.cpu().numpy()).max())
        print(f"[step batched tol] {c.name}: outer {st[j]['outer_iters']} vs {s1['outer_iters']}, "
              f"status {st[j]['status']}, u vs single {eu:.1e}", flush=True)
        assert st[j]["status"] == s1["status"]
        assert abs(st[j]["outer_iters"] - s1["outer_iters"]) <= 1
        if s1["status"] == 0:
            assert eu <= 1e-8


def test_batched_step_argument_errors(ctx):
    items = _setup(ctx, _clouds()[:2])
    c, k, s, vel, pres, dt = items[0]
    u = torch.tensor(vel, device="cuda")
    with pytest.raises(R.RbffdError):          # the same operators twice
        R.simple_step_batched(ctx, [s.ops, s.ops], [u, u.clone()], [u.clone(), u.clone()],
                              [torch.tensor(pres, device="cuda")] * 2, [u.clone(), u.clone()], 1.0, 0.025, [dt, dt],
                              p_bc=[torch.tensor(pres, device="cuda")] * 2)
    with pytest.raises(R.RbffdError):          # prescribed pressure without p_bc
        R.simple_step_batched(ctx, [s.ops], [u], [u.clone()], [torch.tensor(pres, device="cuda")], [u.clone()],
                              1.0, 0.025, [dt])
