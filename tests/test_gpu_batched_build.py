"""The batched stencil build (rbffd_build_stencils_batched) against the
one-cloud build and the oracle: clouds of uneven sizes, degrees, cloud sizes,
PHS powers and dimensions in one call, one weight launch per (dimension,
register width). Clouds and weights must be bitwise those of
rbffd_build_stencils (the same arithmetic per point), and so within the weight
bar of the oracle; a singular cloud is reported as that cloud's."""
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


def _mix():
    """(cloud, k, q (0 = 2m), phs) with widths 16..64, an LDS-sized system and a 3D pair."""
    return [
        (W.kovasznay_square(nx=23, seed=101), 2, 0, 3),                 # 18 unknowns, ragged n
        (W.holed_square(1800, seed=1003, n_holes=2), 3, 0, 3),           # 30
        (W.kovasznay_square(nx=31, seed=102), 4, 0, 3),                  # 45
        (W.holed_square(2600, seed=1004, n_holes=1), 5, 0, 3),           # 63
        (W.kovasznay_square(nx=17, seed=103), 3, 0, 5),                  # r^5
        (W.kovasznay_square(nx=9, seed=104), 2, 0, 3),                   # width 24 again, tiny
        (W.kovasznay_square(nx=14, seed=105), 6, 0, 3),                  # 84 unknowns: the LDS kernel
        (W.scattered_cube(7, seed=106), 2, 0, 3),                        # 3D, 30 unknowns
        (W.beltrami_cube(n=8, seed=107), 3, 0, 3),                       # 3D, 60 unknowns
        (W.holed_square(900, seed=1005, n_holes=0), 4, 36, 3),           # q wider than 2m
    ]


def test_batched_build_equals_one_cloud_builds(ctx, orc):
    mix = _mix()
    dcs = [R.DeviceCloud.from_numpy(c) for c, _, _, _ in mix]
    nbrs, ws, bad = R.rbffd_build_stencils_batched(ctx, dcs, [k for _, k, _, _ in mix], [q for _, _, q, _ in mix],
                                                   [ph for _, _, _, ph in mix])
    assert bad == [-1] * len(mix)
    for (c, k, q, ph), dc, nb, w in zip(mix, dcs, nbrs, ws):
        nb1, w1, _ = R.rbffd_build_stencils(ctx, dc, k, q, ph)
        np.testing.assert_array_equal(nb.cpu().numpy(), nb1.cpu().numpy())
        np.testing.assert_array_equal(w.cpu().numpy(), w1.cpu().numpy())
        qq = nb.shape[1]
        rows = np.unique(np.r_[0, c.n - 1, np.linspace(0, c.n - 1, 40).astype(int)])
        wo = orc.weights(c.xyz, orc.knn(c.xyz, qq), k, ph, queries=rows)
        wg = w.cpu().numpy()[:, rows]
        err = float((np.abs(wg - wo).max(-1) / np.abs(wo).max(-1)).max())
        print(f"[batched build] {c.name}: n={c.n} k={k} q={qq} phs={ph}: bitwise equal to one-cloud; "
              f"oracle rows {err:.1e}", flush=True)
        assert err <= 1e-10


def test_batched_build_reports_the_singular_cloud(ctx):
    xyz = np.stack([np.arange(70.0), np.zeros(70)], 1)
    line = W.Cloud(dim=2, xyz=xyz, kind=np.zeros(70, np.uint8), normal=np.zeros((70, 2)), pin=0)
    good = W.kovasznay_square(nx=10, seed=108)
    dcs = [R.DeviceCloud.from_numpy(good), R.DeviceCloud.from_numpy(line), R.DeviceCloud.from_numpy(good)]
    with pytest.raises(R.RbffdError) as e:
        R.rbffd_build_stencils_batched(ctx, dcs, [2, 1, 3])
    assert e.value.code == -3 and "cloud 1" in str(e.value)
    _, _, bad = R.rbffd_build_stencils_batched(ctx, dcs, [2, 1, 3], allow_singular=True)
    assert bad[0] == -1 and bad[2] == -1 and bad[1] >= 0


def test_batched_build_refuses_bad_input_before_launch(ctx):
    c = W.kovasznay_square(nx=6, seed=109)
    dc = R.DeviceCloud.from_numpy(c)
    per = R.DeviceCloud.from_numpy(W.taylor_green_periodic(nx=12))
    for clouds, ks, qs in (([dc, dc], [3, 3], [0, c.n + 5]), ([dc, per], [2, 2], None)):
        with pytest.raises(R.RbffdError) as e:
            R.rbffd_build_stencils_batched(ctx, clouds, ks, qs)
        assert e.value.code == -1 and "cloud 1" in str(e.value)
