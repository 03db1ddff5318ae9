"""GPU parity of the occlusion-aware view blending (tg_blend_views, §4.3
Eq. 6-10) and of the depth-map normals it weighs with (tg_depth_normals),
through the C ABI.  Both sides evaluate the same FP64 operation sequence,
so the float32 outputs must match the oracle bit for bit."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import torch_cuda

pytestmark = pytest.mark.gpu

DELTA = float(np.float32(0.02))


def _t(a, dt=None):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda") if dt is None else \
        torch.as_tensor(np.ascontiguousarray(a, dt)).to("cuda")


def _fused_depth(views, novel):
    """z_fused of the oracle: every view's lifted points splatted into the
    novel camera, nearest depth per pixel."""
    pts = np.concatenate([oracle.lift([v])["mean"] for v in views], axis=1).astype(np.float32)
    zb, _ = oracle.zsplat(pts, novel)
    return zb


def _check_bitwise(a, b, what):
    a, b = np.asarray(a, np.float32), np.asarray(b, np.float32)
    diff = a.view(np.uint32) != b.view(np.uint32)
    assert not diff.any(), f"{what}: {diff.sum()} of {diff.size} differ, first {np.argwhere(diff)[:3].tolist()}"


def _gpu_blend(srcs, novel, zf):
    torch = torch_cuda()
    from paper_2405_14866_amd.lift import blend_views
    print(f"[gpu] blend {len(srcs)} views into {novel.width}x{novel.height}", flush=True)
    views = [(cam, _t(rgba, np.uint8), _t(depth, np.float32), _t(mask, np.uint8), _t(nm, np.float32))
             for cam, rgba, depth, mask, nm in srcs]
    rgb, ws = blend_views(views, novel, _t(zf, np.float32), DELTA)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), ws.cpu().numpy()


def _sources(views, seed=70):
    out = []
    for k, v in enumerate(views):
        depth = scenes.source_depth(v)
        out.append((v.cam, scenes.source_rgba(v, seed + k), depth, v.mask, oracle.normals(depth, v.cam)))
    return out


def test_normals_of_the_source_depth_maps():
    torch = torch_cuda()
    from paper_2405_14866_amd.lift import depth_normals
    for v in scenes.make_source_views(seed=12):
        depth = scenes.source_depth(v)
        print("[gpu] normals 512^2", flush=True)
        got = depth_normals(_t(depth, np.float32), v.cam)
        torch.cuda.synchronize()
        _check_bitwise(got.cpu().numpy(), oracle.normals(depth, v.cam), "normals")
    # ragged and tiny maps
    rng = np.random.default_rng(3)
    for (W, H) in [(37, 23), (1, 1), (3, 2), (130, 17)]:
        cam = scenes.orbit_camera(7.0, -3.0, (0.0, 0.0, 1.5), 1.5, 40.0, 44.0, W / 2.0, H / 2.0, W, H).as_f32()
        depth = rng.uniform(0.9, 1.4, (H, W)).astype(np.float32)
        depth[rng.uniform(0, 1, (H, W)) < 0.1] = 0.0
        got = depth_normals(_t(depth, np.float32), cam)
        torch.cuda.synchronize()
        _check_bitwise(got.cpu().numpy(), oracle.normals(depth, cam), f"normals {W}x{H}")


def test_blend_four_views_into_the_frontal_target():
    """The realistic frame's four source views (512^2) blended into the
    frontal 1024^2 target, with z_fused from the lifted points."""
    views = scenes.make_source_views(seed=12, c=8)
    novel = scenes.make_cfg2().cam
    srcs = _sources(views)
    zf = _fused_depth(views, novel)
    rgb, ws = _gpu_blend(srcs, novel, zf)
    ref_rgb, ref_ws = oracle.blend(srcs, novel, zf, DELTA)
    _check_bitwise(rgb, ref_rgb, "rgb")
    _check_bitwise(ws, ref_ws, "wsum")
    assert (ref_ws > 0).sum() > 100000          # most of the body is blended


def test_blend_ragged_sizes_and_degenerate_views():
    """A ragged 37x23 novel view, source views of different sizes including
    a 1x1 and a 2x1 view, a view behind the points, no views at all, and
    fused depths that are zero, negative or infinite."""
    rng = np.random.default_rng(5)
    views = scenes.make_source_views(seed=14, src_res=64, src_fx=90.0, c=8)
    srcs = _sources(views)
    tiny = []
    for (W, H) in [(1, 1), (2, 1)]:
        cam = scenes.orbit_camera(0.0, 0.0, (0.0, 0.0, 0.0), 1.2, 2.0, 2.0, W / 2.0, H / 2.0, W, H).as_f32()
        depth = np.full((H, W), 1.2, np.float32)
        tiny.append((cam, np.full((H, W, 4), 200, np.uint8), depth, np.ones((H, W), np.uint8),
                     rng.normal(0, 1, (H, W, 3)).astype(np.float32)))
    behind = scenes.orbit_camera(180.0, 0.0, (0.0, 0.0, 0.0), 1.2, 90.0, 90.0, 32.0, 32.0, 64, 64).as_f32()
    srcs2 = srcs + tiny + [(behind,) + srcs[0][1:]]
    novel = scenes.orbit_camera(3.0, 2.0, (0.0, 0.0, 0.0), 1.2, 50.0, 50.0, 18.5, 11.5, 37, 23).as_f32()
    zf = _fused_depth(views, novel)
    zf[0, :3] = [0.0, -1.0, np.inf]
    for s in (srcs2, srcs[:1], []):
        rgb, ws = _gpu_blend(s, novel, zf)
        ref_rgb, ref_ws = oracle.blend(s, novel, zf, DELTA)
        _check_bitwise(rgb, ref_rgb, "rgb")
        _check_bitwise(ws, ref_ws, "wsum")


def test_whole_chain_on_the_device_at_full_resolution():
    """The §4.3 chain at the paper's 2048^2 output: lift every source view
    (tg_lift), warp the points onto the novel view (tg_zsplat), normals of
    each depth map (tg_depth_normals), blend (tg_blend_views) -- all on the
    device -- against the oracle's chain on the same inputs."""
    torch = torch_cuda()
    from paper_2405_14866_amd.lift import (GaussianBuffers, Lifter, SourceViewMaps, blend_views, depth_normals,
                                           zsplat)
    views = scenes.make_source_views(seed=55, src_res=2048, src_fx=2800.0, c=8)
    novel = scenes.look_at_camera(0.0, 1.2, 2800.0, 1024.0, 2048).as_f32()
    print("[gpu] 2048^2 chain: lift, zsplat, normals, blend", flush=True)
    total = sum(v.mask.size for v in views)
    lf = Lifter(0, max_pixels=total)
    out = GaussianBuffers(total, 8)
    lf.enqueue([SourceViewMaps.from_source_view(v) for v in views], out)
    torch.cuda.synchronize()
    n = int(lf.n_out.item())
    (zf, _), = zsplat(out.view(n).mean, [novel], None, with_disparity=False)
    dev_views = []
    srcs = []
    for k, v in enumerate(views):
        depth = scenes.source_depth(v)
        rgba = scenes.source_rgba(v, 90 + k)
        dd = _t(depth, np.float32)
        nm = depth_normals(dd, v.cam)
        dev_views.append((v.cam, _t(rgba, np.uint8), dd, _t(v.mask, np.uint8), nm))
        srcs.append((v.cam, rgba, depth, v.mask, oracle.normals(depth, v.cam)))
    rgb, ws = blend_views(dev_views, novel, zf, DELTA)
    torch.cuda.synchronize()
    zf_ref = _fused_depth(views, novel)
    _check_bitwise(zf.cpu().numpy(), zf_ref, "z_fused")
    ref_rgb, ref_ws = oracle.blend(srcs, novel, zf_ref, DELTA)
    _check_bitwise(rgb.cpu().numpy(), ref_rgb, "rgb")
    _check_bitwise(ws.cpu().numpy(), ref_ws, "wsum")


def test_blend_invalid_arguments():
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.rasterize import Context, camera_struct
    ctx = Context.get(0).handle
    cam = camera_struct(scenes.make_cfg1().cam)
    zf = torch.zeros(64 * 64, device="cuda")
    rgb = torch.empty(3 * 64 * 64, device="cuda")
    ws = torch.empty(64 * 64, device="cuda")
    rgba = torch.zeros(64 * 64 * 4 + 4, dtype=torch.uint8, device="cuda")
    dep = torch.zeros(64 * 64, device="cuda")
    nm = torch.zeros(64 * 64 * 3, device="cuda")
    v = N.tg_blend_view()
    v.cam, v.rgba, v.depth, v.mask, v.normal = cam, rgba.data_ptr(), dep.data_ptr(), rgba.data_ptr(), nm.data_ptr()
    s = int(torch.cuda.current_stream().cuda_stream)
    args = (ctx, [v], cam, zf.data_ptr())
    assert N.tg_blend_views(*args, 0.02, rgb.data_ptr(), ws.data_ptr(), s) == N.TG_OK
    assert N.tg_blend_views(*args, 0.0, rgb.data_ptr(), ws.data_ptr(), s) == N.TG_ERR_INVALID
    assert N.tg_blend_views(ctx, [v] * 9, cam, zf.data_ptr(), 0.02, rgb.data_ptr(), ws.data_ptr(), s) == \
        N.TG_ERR_INVALID
    bad = N.tg_blend_view()
    bad.cam, bad.rgba, bad.depth, bad.mask, bad.normal = cam, rgba.data_ptr() + 1, dep.data_ptr(), \
        rgba.data_ptr(), nm.data_ptr()
    assert N.tg_blend_views(ctx, [bad], cam, zf.data_ptr(), 0.02, rgb.data_ptr(), ws.data_ptr(), s) == \
        N.TG_ERR_INVALID
    assert N.tg_depth_normals(ctx, cam, None, nm.data_ptr(), s) == N.TG_ERR_INVALID
    torch.cuda.synchronize()
