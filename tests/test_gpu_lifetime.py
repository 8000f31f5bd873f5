"""Object lifetimes across the C ABI: operators and servers that outlive their
context are orphaned, not dangling."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2106_07616_amd as R  # noqa: E402


def test_operators_and_server_outliving_their_context():
    c = W.kovasznay_square(nx=10)
    ctx = R.Context(0)
    s = R.Solver(ctx, c, 2)
    sv = R.Server(ctx)
    b = torch.tensor(np.random.default_rng(0).standard_normal(c.n), device="cuda")
    x = torch.zeros_like(b)
    ctx.close()
    with pytest.raises(R.RbffdError) as e:
        R.poisson_solve(R.Context(0), s.ops, b, x)
    assert e.value.code == -1
    with pytest.raises(R.RbffdError):
        sv.submit(s.ops, b, x)
    s.ops.free()
    sv.close()
    # a fresh context works normally afterwards
    ctx2 = R.Context(0)
    s2 = R.Solver(ctx2, c, 2)
    st = R.poisson_solve(ctx2, s2.ops, b, x, tol=1e-10, max_iter=5000)
    assert st["status"] == 0
    ctx2.close()
