"""Pins of the oracle's z-buffer point splat (the cascaded disparity
initialisation of §4.1: the point cloud of cam0 rasterized into another
viewpoint, its z-buffer extracted and converted back to disparity): closed
forms of the landing pixel and depth, the nearest point winning regardless
of order, culling, and the round trip lift -> splat into the same camera."""
import numpy as np

import oracle
import scenes


def _cam(W=16, H=12, fx=50.0, fy=40.0, cx=8.0, cy=6.0):
    return scenes.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), fx, fy, cx, cy, W, H)


def test_closed_form_landing_pixel_and_depth():
    """A point at (X, Y, Z) lands in pixel (floor(fx X / Z + cx),
    floor(fy Y / Z + cy)) with depth Z; its disparity is fx B / Z."""
    cam = _cam()
    X, Y, Z = 0.09, -0.06, 2.0          # u = 50 * 0.045 + 8 = 10.25, v = 40 * -0.03 + 6 = 4.8
    zb, dp = oracle.zsplat(np.array([[X], [Y], [Z]], np.float32), cam, baseline=0.1)
    hit = np.argwhere(np.isfinite(zb))
    assert hit.tolist() == [[4, 10]]
    assert zb[4, 10] == np.float32(Z)
    assert dp[4, 10] == np.float32(50.0 * float(np.float32(0.1)) / 2.0)
    assert np.count_nonzero(dp) == 1


def test_pixel_is_the_floor_of_the_projection():
    """u = 5.75 lands in column 5 (the pixel that contains it, not the
    nearest pixel centre's neighbour)."""
    cam = _cam()
    Z = 1.0
    zb, _ = oracle.zsplat(np.array([[(5.75 - 8.0) / 50.0], [(2.25 - 6.0) / 40.0], [Z]], np.float32), cam)
    assert np.argwhere(np.isfinite(zb)).tolist() == [[2, 5]]


def test_nearest_point_wins_in_any_order():
    """Three points on one pixel's ray at depths 3, 1.5 and 2: the z-buffer
    holds 1.5 whatever the order of the points."""
    cam = _cam()
    zs = np.array([3.0, 1.5, 2.0])
    u, v = 3.5, 7.5
    pts = np.stack([(u - 8.0) * zs / 50.0, (v - 6.0) * zs / 40.0, zs]).astype(np.float32)
    for perm in ([0, 1, 2], [1, 0, 2], [2, 0, 1], [0, 2, 1]):
        zb, _ = oracle.zsplat(pts[:, perm], cam)
        assert zb[7, 3] == np.float32(1.5)
        assert np.isfinite(zb).sum() == 1


def test_culled_points_land_nowhere():
    """Behind the camera, in front of the near plane, left of or below the
    image, exactly on the right edge, and NaN: none lands."""
    cam = _cam()
    pts = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 0.1], [-0.5, 0.0, 1.0], [0.0, 0.3, 1.0],
                    [(16.0 - 8.0) / 50.0, 0.0, 1.0], [np.nan, 0.0, 1.0]]).T.astype(np.float32)
    zb, dp = oracle.zsplat(pts, cam)
    assert not np.isfinite(zb).any() and not dp.any()


def test_lift_then_splat_into_the_same_camera_is_the_identity():
    """Lifting a view and splatting its points back into the same camera
    puts every lifted pixel's point on its own pixel (the lifted point
    projects to the pixel centre), so the z-buffer is finite exactly on the
    lifted pixels and the disparity comes back to float32 rounding."""
    for v in scenes.make_source_views(seed=13, src_res=80, src_fx=110.0, c=2):
        lifted = oracle.lift([v])
        zb, dp = oracle.zsplat(lifted["mean"].astype(np.float32), v.cam, v.baseline)
        sel = (v.mask > 0) & (v.disparity > 0)
        np.testing.assert_array_equal(np.isfinite(zb), sel)
        np.testing.assert_allclose(dp[sel], v.disparity[sel], rtol=2e-6)
        assert not dp[~sel].any()
