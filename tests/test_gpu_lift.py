"""GPU parity of tg_lift (the step upstream of the rasterizer: §4.1 disparity
to depth, §4.2 unprojection of the foreground pixels with their encoder maps)
against the oracle's lifting, through the C ABI.

The compaction's count and (view, row-major pixel) order, the copied maps
(scale, opacity, features) and the identity quaternion must match bit for
bit.  Positions: both sides evaluate the same FP64 operation sequence with
correctly rounded IEEE double operations, so the GPU's float32 position is
the oracle's FP64 position rounded once -- bit for bit as well."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import compare_forward, compare_lists, gpu_render, torch_cuda

pytestmark = pytest.mark.gpu


def _gpu_lift(views, cap=None, sentinel=None):
    torch = torch_cuda()
    from paper_2405_14866_amd.lift import GaussianBuffers, Lifter, SourceViewMaps
    total = sum(v.mask.size for v in views)
    print(f"[gpu] lift {len(views)} views, {total} pixels, c={views[0].c}, cap={cap}", flush=True)
    maps = []
    for v in views:
        m = SourceViewMaps.from_source_view(v)
        if v.disparity is None or getattr(v, "_use_depth", False):
            m = SourceViewMaps(v.cam, m.mask, m.feat, m.scale, m.opacity,
                               depth=torch.as_tensor(v._depth, device="cuda"))
        maps.append(m)
    lf = Lifter(0, max_pixels=max(total, 1))
    out = GaussianBuffers(total if cap is None else cap, views[0].c)
    if sentinel is not None:
        for t in (out.mean, out.scale, out.quat, out.opacity, out.feat):
            t.fill_(sentinel)
    n_out = lf.enqueue(maps, out)
    torch.cuda.synchronize()
    n = int(n_out.item())
    return n, out


def _as_np(out, n):
    g = out.view(n)
    return dict(mean=g.mean.cpu().numpy(), scale=g.scale.cpu().numpy(), quat=g.quat.cpu().numpy(),
                opacity=g.opacity.cpu().numpy(), feat=g.feat.cpu().numpy())


def _assert_bitwise(got, ref):
    n = ref["opacity"].shape[0]
    for k in ("mean", "scale", "quat", "opacity", "feat"):
        want = ref[k].astype(np.float32)
        a = got[k]
        assert a.shape == want.shape, (k, a.shape, want.shape)
        if n == 0:
            continue
        diff = a.view(np.uint32) != want.view(np.uint32)
        assert not diff.any(), f"{k}: {diff.sum()} of {diff.size} differ, first at {np.argwhere(diff)[:3].tolist()}"


def _random_view(rng, W, H, c, frac=0.5, depth=False, fx=None, yaw=0.0):
    fx = float(fx or max(W, H))
    cam = scenes.orbit_camera(yaw, 3.0, (0.0, 0.0, 1.5), 1.5, fx, fx * 1.1, W / 2.0 + 0.3, H / 2.0 - 0.2, W, H)
    z = rng.uniform(0.8, 1.5, (H, W))
    disp = (fx * 0.1 / z).astype(np.float32)
    mask = (rng.uniform(0, 1, (H, W)) < frac).astype(np.uint8)
    v = scenes.SourceView(cam, disp, mask, rng.standard_normal((H, W, c)),
                          rng.uniform(0.001, 0.01, (H, W, 3)), rng.uniform(0.05, 0.95, (H, W)), 0.1)
    if depth:
        v._use_depth = True
        v._depth = z.astype(np.float32)
    return v


def test_lift_realistic_views_bit_exact():
    """The realistic frame's four 512x512 source views (C = 32)."""
    views = scenes.make_source_views()
    ref = oracle.lift(views)
    n, out = _gpu_lift(views)
    assert n == ref["opacity"].shape[0] == int(sum(int(v.mask.sum()) for v in views))
    _assert_bitwise(_as_np(out, n), ref)


def test_lifted_set_renders_like_the_oracle():
    """Lift on the GPU, render the lifted set on the GPU, and compare the
    image with the oracle's render of the oracle's own lifting (the two sets
    are bitwise equal, the previous test)."""
    views = scenes.make_source_views()
    ref = oracle.lift(views)
    n, out = _gpu_lift(views)
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    sc = scenes.Scene(f32(ref["mean"]), f32(ref["scale"]), f32(ref["quat"]), f32(ref["opacity"]),
                      f32(ref["feat"]), scenes.make_cfg2().cam, None, "lifted realistic")
    ora = oracle.Oracle(sc)
    gpu, _, _ = gpu_render(sc)
    compare_lists(gpu, ora)
    compare_forward(gpu, ora)
    # and the GPU-lifted buffers themselves render to the same image
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import Rasterizer
    g = out.view(n)
    rast = Rasterizer(0, max_n=n, max_w=sc.cam.width, max_h=sc.cam.height)
    feat, alpha = rast.forward(g, sc.cam)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(feat.cpu().numpy(), gpu["feat"])
    np.testing.assert_array_equal(alpha.cpu().numpy(), gpu["alpha"])


@pytest.mark.parametrize("c", [8, 16, 64])
def test_lift_ragged_views_and_channels(c):
    """Views whose pixel counts are not multiples of the 1024-pixel block,
    of different sizes, one given as depth instead of disparity; the maps
    hold zero, negative and NaN disparities inside the mask."""
    rng = np.random.default_rng(100 + c)
    views = [_random_view(rng, 37, 23, c, 0.6), _random_view(rng, 1, 1, c, 1.0),
             _random_view(rng, 1000, 3, c, 0.3, yaw=20.0), _random_view(rng, 129, 64, c, 0.9, depth=True)]
    d = views[0].disparity
    d[0, :5] = 0.0
    d[1, :5] = -1.0
    d[2, :5] = np.nan
    views[0].mask[:3, :5] = 1
    # the oracle takes either all disparities or all depths: lift the depth
    # view on its own and concatenate (order is view-major)
    r1 = oracle.lift(views[:3])
    r2 = oracle.lift([views[3]], use_depth=[views[3]._depth])
    ref = {k: np.concatenate([r1[k], r2[k]], axis=1 if r1[k].ndim == 2 and k != "feat" else 0)
           for k in r1}
    n, out = _gpu_lift(views)
    assert n == ref["opacity"].shape[0]
    _assert_bitwise(_as_np(out, n), ref)


def test_lift_eight_views_and_empty_masks():
    rng = np.random.default_rng(7)
    views = [_random_view(rng, 64 + 9 * k, 48 + 5 * k, 16, frac=(0.0 if k in (2, 5) else 0.4),
                          yaw=-20.0 + 5 * k) for k in range(8)]
    ref = oracle.lift(views)
    n, out = _gpu_lift(views)
    assert n == ref["opacity"].shape[0]
    _assert_bitwise(_as_np(out, n), ref)
    empty = [_random_view(rng, 50, 40, 8, frac=0.0)]
    n0, _ = _gpu_lift(empty)
    assert n0 == 0


def test_lift_overflow_writes_nothing():
    rng = np.random.default_rng(8)
    views = [_random_view(rng, 100, 100, 8, frac=0.5)]
    need = int(views[0].mask.sum())
    n, out = _gpu_lift(views, cap=need - 1, sentinel=-7.0)
    assert n == need
    for t in (out.mean, out.scale, out.quat, out.opacity, out.feat):
        assert bool((t == -7.0).all())
    n2, out2 = _gpu_lift(views, cap=need)
    assert n2 == need
    _assert_bitwise(_as_np(out2, n2), oracle.lift(views))


def test_lift_serving_grid_full_size():
    """The serving workload's source view at its largest size: a 1000x1000
    grid with the first 999,000 pixels in the mask."""
    v = scenes.make_grid_source_view(44, 1000, 999000)
    ref = oracle.lift([v])
    n, out = _gpu_lift([v])
    assert n == 999000
    _assert_bitwise(_as_np(out, n), ref)


def test_lift_invalid_arguments():
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.lift import GaussianBuffers, Lifter, SourceViewMaps
    rng = np.random.default_rng(9)
    v = SourceViewMaps.from_source_view(_random_view(rng, 40, 30, 8))
    lf = Lifter(0, max_pixels=1200)
    out = GaussianBuffers(1200, 8)
    s = int(torch.cuda.current_stream().cuda_stream)
    n_out = lf.n_out.data_ptr()
    assert N.tg_lift(lf.handle, [v.struct()], 12, out.struct(), n_out, s) == N.TG_ERR_UNSUPPORTED
    assert N.tg_lift(lf.handle, [v.struct()] * 9, 8, out.struct(), n_out, s) == N.TG_ERR_INVALID
    assert N.tg_lift(lf.handle, [v.struct()] * 2, 8, out.struct(), n_out, s) == N.TG_ERR_CAPACITY
    assert N.tg_lift(lf.handle, [v.struct()], 8, out.struct(), None, s) == N.TG_ERR_INVALID
    bad = v.struct()
    bad.mask = None
    assert N.tg_lift(lf.handle, [bad], 8, out.struct(), n_out, s) == N.TG_ERR_INVALID
    bad = v.struct()
    bad.baseline = 0.0
    assert N.tg_lift(lf.handle, [bad], 8, out.struct(), n_out, s) == N.TG_ERR_INVALID
    mis = out.struct()
    mis.feat = mis.feat + 4
    assert N.tg_lift(lf.handle, [v.struct()], 8, mis, n_out, s) == N.TG_ERR_INVALID
    torch.cuda.synchronize()
