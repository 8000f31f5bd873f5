"""Serving flow requests (paper_2106_07616_amd.serve): concurrent slots, each
with its own context and stream, under an HBM budget. Each request's result
(fields and step statistics) is bitwise the same alone and in a mix, and the
budget bounds how many requests run at once."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2106_07616_amd as R  # noqa: E402
from paper_2106_07616_amd import serve as S  # noqa: E402


def _requests():
    pp = W.PRESCRIBED_PRESSURE
    kw = dict(steps=2, max_krylov=2000)
    return [
        S.FlowRequest(W.kovasznay_square(nx=24, seed=7001, boundary_kind=pp), 3, tag="kovasznay24_k3", **kw),
        S.FlowRequest(W.holed_square(2500, seed=7002, edge_kind=pp, hole_kind=pp), 2, tag="holed2500_k2", **kw),
        S.FlowRequest(W.beltrami_cube(n=9, seed=7003), 2, tag="cube9_k2", **kw),
        S.FlowRequest(W.taylor_green_disk(r=0.1), 4, tag="tg_disk_k4", **kw),
        S.FlowRequest(W.kovasznay_square(nx=30, seed=7004, boundary_kind=pp), 4, tag="kovasznay30_k4", **kw),
        S.FlowRequest(W.beltrami_cube(n=8, seed=7005), 3, tag="cube8_k3", **kw),
    ]


@pytest.fixture(scope="module")
def alone():
    """Every request run alone, one after the other, on the default stream."""
    ctx = R.Context(0)
    out = {}
    for req in _requests():
        req.flow_fields = W.flow_fields
        print(f"[serve] alone {req.tag}: n={req.cloud.n}", flush=True)
        out[req.tag] = S.run_request(ctx, req)
    torch.cuda.synchronize()
    ctx.close()
    return out


def _same(a, b):
    """Bitwise the same fields and step statistics (NaN equal to NaN: the small
    cubes' steps blow up under these readings, identically alone and in a mix)."""
    np.testing.assert_array_equal(a.u, b.u)
    np.testing.assert_array_equal(a.p, b.p)
    assert a.dt == b.dt
    assert len(a.stats) == len(b.stats)
    for sa, sb in zip(a.stats, b.stats):
        assert sa.keys() == sb.keys()
        for key in sa:
            np.testing.assert_array_equal(np.float64(sa[key]), np.float64(sb[key]), err_msg=key)


def test_results_in_a_mix_equal_alone(alone):
    """Six requests submitted at once into three slots: the device runs their
    work concurrently, and every result equals the request's result alone."""
    with S.FlowServer(slots=3) as sv:
        futs = [sv.submit(r) for r in _requests()]
        res = [f.result() for f in futs]
        peak = sv.peak_active
    print(f"[serve] mix: peak concurrent requests {peak}", flush=True)
    assert peak >= 2
    for r in res:
        print(f"[serve] {r.tag}: slot {r.slot} build {r.t_build * 1e3:.1f} ms steps {r.t_steps * 1e3:.1f} ms "
              f"outer {[s['outer_iters'] for s in r.stats]}", flush=True)
        _same(r, alone[r.tag])


def test_budget_limits_concurrency(alone):
    """With a budget that holds the largest request alone, the reserved bytes
    never exceed it, fewer requests run at once than without it, and the
    results are the same; a request larger than the budget fails with E_OOM."""
    reqs = _requests()
    sizes = []
    for r in reqs:
        q, _, _ = R.rbffd_stencil_sizes(r.cloud.dim, r.poly_degree)
        sizes.append(S.estimate_bytes(r.cloud.dim, r.cloud.n, q))
    budget = max(sizes)
    with S.FlowServer(slots=len(reqs), hbm_budget=budget) as sv:
        futs = [sv.submit(r) for r in reqs]
        res = [f.result() for f in futs]
        print(f"[serve] budget {budget}: peak reserved {sv.peak_reserved}, peak concurrent {sv.peak_active}",
              flush=True)
        assert sv.peak_reserved <= budget
        assert sv.peak_active < len(reqs)
    for r in res:
        _same(r, alone[r.tag])
    with S.FlowServer(slots=1, hbm_budget=min(sizes) - 1) as sv:
        with pytest.raises(R.RbffdError) as e:
            sv.submit(_requests()[0]).result()
        assert e.value.code == R.binding.RBFFD_E_OOM
