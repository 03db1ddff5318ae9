"""tg_render_noalloc (the render sequence with its workspace in a static
device array, for callers that cannot allocate) through the C ABI, against
the frame-based entry points tg_project + tg_bin_sort + tg_render_fwd: the
same kernels, so the images must be bit-identical; the small frame is also
checked against the FP64 oracle.  Two calls in a row, the second smaller,
then a call whose keys overflow the array and one after it."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import compare_forward, gpu_render, torch_cuda

pytestmark = pytest.mark.gpu


def _noalloc(scene, torch, bg=None):
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.rasterize import Context, GaussianSoA, _ptr, camera_struct
    print(f"[gpu] tg_render_noalloc {scene.name} n={scene.n} c={scene.c} "
          f"{scene.cam.width}x{scene.cam.height}", flush=True)
    ctx = Context.get(0)
    g = GaussianSoA.from_scene(scene)
    H, W = scene.cam.height, scene.cam.width
    feat = torch.full((scene.c, H, W), float("nan"), device="cuda")
    alpha = torch.full((H, W), float("nan"), device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    bgt = None if bg is None else torch.as_tensor(bg, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    st = N.tg_render_noalloc(ctx.handle, g.struct(), camera_struct(scene.cam), _ptr(bgt),
                             feat.data_ptr(), alpha.data_ptr(), status.data_ptr(), s)
    torch.cuda.synchronize()
    return st, int(status.item()), feat.cpu().numpy(), alpha.cpu().numpy()


def test_noalloc_matches_frame_path_twice_then_smaller():
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    big = scenes.make_cfg2()
    small = scenes.make_cfg1()
    for sc, bg in ((big, None), (small, np.linspace(-1, 1, small.c).astype(np.float32))):
        st, status, feat, alpha = _noalloc(sc, torch, bg)
        assert st == N.TG_OK and status == N.TG_OK, (st, status)
        ref, _, _ = gpu_render(sc, bg=bg, lists=False)
        np.testing.assert_array_equal(feat, ref["feat"])
        np.testing.assert_array_equal(alpha, ref["alpha"])
        if sc is small:
            bg64 = bg.astype(np.float64)
            compare_forward(dict(feat=feat, alpha=alpha, last=ref["last"]), oracle.Oracle(sc), bg=bg64)


def test_noalloc_limits_and_key_overflow():
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.rasterize import Context, GaussianSoA, _ptr, camera_struct
    ctx = Context.get(0)
    sc = scenes.make_cfg1()
    g = GaussianSoA.from_scene(sc)
    out = torch.empty((sc.c, 64, 64), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    # too many Gaussians, pixels or tiles: refused before anything is enqueued
    gs = g.struct(); gs.n = N.TG_NOALLOC_MAX_N + 1
    assert N.tg_render_noalloc(ctx.handle, gs, camera_struct(sc.cam), None, out.data_ptr(), None, None,
                               s) == N.TG_ERR_CAPACITY
    wide = scenes.Camera(sc.cam.R, sc.cam.t, 64, 64, 32, 32, 2048, 1024)
    assert N.tg_render_noalloc(ctx.handle, g.struct(), camera_struct(wide), None, out.data_ptr(), None,
                               None, s) == N.TG_ERR_CAPACITY
    thin = scenes.Camera(sc.cam.R, sc.cam.t, 64, 64, 0.5, 32, 1, 200000)   # 12,500 tiles
    assert N.tg_render_noalloc(ctx.handle, g.struct(), camera_struct(thin), None, out.data_ptr(), None,
                               None, s) == N.TG_ERR_CAPACITY
    gs = g.struct(); gs.c = 12
    assert N.tg_render_noalloc(ctx.handle, gs, camera_struct(sc.cam), None, out.data_ptr(), None, None,
                               s) == N.TG_ERR_UNSUPPORTED
    # the realistic frame with doubled scales needs ~3.7M keys: reported on the device
    big = scenes.make_cfg2()
    fat = scenes.Scene(big.mean, big.scale * 2.0, big.quat, big.opacity, big.feat, big.cam, name="cfg2x2")
    st, status, _, _ = _noalloc(fat, torch)
    assert st == N.TG_OK and status == N.TG_ERR_CAPACITY, (st, status)
    # the next call starts from a clean state
    st, status, feat, alpha = _noalloc(sc, torch)
    assert st == N.TG_OK and status == N.TG_OK
    ref, _, _ = gpu_render(sc, lists=False)
    np.testing.assert_array_equal(feat, ref["feat"])
    np.testing.assert_array_equal(alpha, ref["alpha"])
