"""Pins of the oracle's lifting of source views to Gaussians (§4.1: the
predicted disparity becomes depth; §4.2: Gaussian positions are unprojected
from the depth maps with the camera parameters, the foreground pixels become
pixel-aligned Gaussians carrying the encoder's per-pixel maps, rotation
fixed to identity): closed forms of the unprojection, the round trip through
the source camera, the count and order of the compaction, and agreement with
the scene generator's own unprojection of the realistic frame."""
import numpy as np

import oracle
import scenes


def _view(cam, disp, mask, c=2, seed=0, baseline=0.1):
    H, W = disp.shape
    rng = np.random.default_rng(seed)
    feat = rng.standard_normal((H, W, c))
    scale = rng.uniform(0.001, 0.01, (H, W, 3))
    opac = rng.uniform(0.1, 0.9, (H, W))
    return scenes.SourceView(cam, disp, mask, feat, scale, opac, baseline)


def _eye_cam(fx=50.0, fy=40.0, cx=8.0, cy=6.0, W=16, H=12):
    return scenes.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), fx, fy, cx, cy, W, H)


def test_closed_form_identity_camera():
    """One foreground pixel (5, 3) with disparity d: depth z = fx B / d and
    the world point ((5.5 - cx) z / fx, (3.5 - cy) z / fy, z)."""
    cam = _eye_cam()
    disp = np.zeros((12, 16), np.float32)
    mask = np.zeros((12, 16), np.uint8)
    disp[3, 5] = 2.5
    mask[3, 5] = 1
    v = _view(cam, disp, mask, baseline=0.1)
    out = oracle.lift([v])
    assert out["mean"].shape == (3, 1)
    z = 50.0 * float(np.float32(0.1)) / 2.5
    np.testing.assert_allclose(out["mean"][:, 0], [(5.5 - 8.0) * z / 50.0, (3.5 - 6.0) * z / 40.0, z],
                               rtol=0, atol=1e-15)
    np.testing.assert_array_equal(out["quat"][:, 0], [1.0, 0.0, 0.0, 0.0])
    np.testing.assert_array_equal(out["scale"][:, 0], v.scale[3, 5].astype(np.float64))
    assert out["opacity"][0] == np.float64(v.opacity[3, 5])
    np.testing.assert_array_equal(out["feat"][0], v.feat[3, 5].astype(np.float64))


def test_closed_form_turned_camera():
    """A camera at (2, 0, 0) looking along -x (yaw -90 deg about the origin
    on a 2 m arc): the camera's forward axis is -x, its right axis +z, so
    pixel (i, j) at depth z lifts to (2 - z, (j + 0.5 - cy) z / fy,
    (i + 0.5 - cx) z / fx)."""
    cam = scenes.look_at_camera(-90.0, 2.0, 30.0, 4.0, 8)
    disp = np.zeros((8, 8), np.float32)
    mask = np.zeros((8, 8), np.uint8)
    disp[2, 6] = 4.0
    mask[2, 6] = 1
    v = _view(cam, disp, mask, baseline=0.2)
    out = oracle.lift([v])
    z = 30.0 * float(np.float32(0.2)) / 4.0
    want = [2.0 - z, (2.5 - 4.0) * z / 30.0, (6.5 - 4.0) * z / 30.0]
    np.testing.assert_allclose(out["mean"][:, 0], want, rtol=0, atol=1e-6)


def test_round_trip_through_the_source_camera():
    """Every lifted point projects back through its own (rotated, translated)
    source camera to the centre of the pixel it came from, at the depth its
    disparity gives (to the 1e-7 by which the float32 rotation misses being
    orthonormal)."""
    views = scenes.make_source_views(seed=3, src_res=64, src_fx=90.0, c=4)
    out = oracle.lift(views)
    k = 0
    for v in views:
        js, is_ = np.nonzero(v.mask & (v.disparity > 0))
        n = len(js)
        m = out["mean"][:, k:k + n]
        R = v.cam.R.astype(np.float64)
        t = v.cam.t.astype(np.float64)
        xc = R @ m + t[:, None]
        z = v.cam.fx * v.baseline / v.disparity[js, is_].astype(np.float64)
        np.testing.assert_allclose(xc[2], z, rtol=3e-7)
        np.testing.assert_allclose(v.cam.fx * xc[0] / xc[2] + v.cam.cx, is_ + 0.5, rtol=0, atol=1e-4)
        np.testing.assert_allclose(v.cam.fy * xc[1] / xc[2] + v.cam.cy, js + 0.5, rtol=0, atol=1e-4)
        k += n
    assert k == out["mean"].shape[1]


def test_count_and_order_of_the_compaction():
    """Pixels are lifted where the mask is set and the disparity is positive
    (zero, negative and NaN disparities are not), in (view, row-major pixel)
    order: with feature 0 holding view * 10^6 + pixel index, the lifted
    features list exactly the selected pixels in increasing order."""
    rng = np.random.default_rng(4)
    views, want = [], []
    for vi in range(3):
        H, W = 10 + vi, 14 - vi
        disp = rng.uniform(-1.0, 3.0, (H, W)).astype(np.float32)
        disp[0, 0] = np.nan
        disp[1, 1] = 0.0
        mask = (rng.uniform(size=(H, W)) < 0.6).astype(np.uint8)
        mask[0, 0] = mask[1, 1] = 1
        v = _view(_eye_cam(W=W, H=H), disp, mask, c=3, seed=vi)
        v.feat[:, :, 0] = (vi * 10 ** 6 + np.arange(H * W)).reshape(H, W)
        sel = (mask != 0) & (disp > 0)
        want.append(vi * 10 ** 6 + np.flatnonzero(sel.reshape(-1)))
        views.append(v)
    out = oracle.lift(views)
    want = np.concatenate(want)
    assert out["mean"].shape[1] == len(want)
    np.testing.assert_array_equal(out["feat"][:, 0], want.astype(np.float64))


def test_depth_maps_equal_their_disparities():
    """Given the depth maps fx B / d directly instead of the disparities,
    the lift is the same."""
    views = scenes.make_source_views(seed=5, src_res=48, src_fx=70.0, c=2)
    a = oracle.lift(views)
    depths = [np.where(v.disparity > 0, v.cam.fx * v.baseline / v.disparity.astype(np.float64), 0.0)
              for v in views]
    b = oracle.lift(views, use_depth=depths)
    for k in ("mean", "scale", "opacity", "feat"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-15, atol=0)


def test_realistic_views_lift_to_the_body_scene_geometry():
    """The four realistic source views lift to the point set the scene
    generator unprojects for the realistic frame (same mask, same depth
    surface, same cameras): equal counts and positions within float32
    rounding of the disparity and the camera (1e-5 m)."""
    views = scenes.make_source_views()
    out = oracle.lift(views)
    body = scenes.make_cfg2()
    assert out["mean"].shape[1] == body.n == 471384
    np.testing.assert_allclose(out["mean"], body.mean.astype(np.float64), rtol=0, atol=1e-5)
