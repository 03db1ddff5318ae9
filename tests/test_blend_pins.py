"""Pins of the oracle's occlusion-aware view blending (§4.3, Eq. 6-10) and
of its depth-map normals: closed forms of the normals of planes, of the
weights of Eq. 8 on a plane seen by two cameras, of the bilinear fetch of
Eq. 7 on a colour ramp, of the occlusion check of Eq. 9, of the mask term,
and the empty cases."""
import numpy as np

import oracle
import scenes


def _cam(W=24, H=20, fx=40.0, fy=44.0, cx=12.0, cy=10.0, R=None, t=(0.0, 0.0, 0.0)):
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    return scenes.Camera(R, np.asarray(t, np.float32), fx, fy, cx, cy, W, H).as_f32()


def _plane_depth(cam, n, d):
    """Depth map of the plane {P : <n, P> = d} (camera frame) seen by cam."""
    j, i = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
    xt = (i + 0.5 - cam.cx) / cam.fx
    yt = (j + 0.5 - cam.cy) / cam.fy
    return (d / (n[0] * xt + n[1] * yt + n[2])).astype(np.float32)


def test_normals_of_a_fronto_parallel_plane():
    cam = _cam()
    nm = oracle.normals(np.full((20, 24), 1.7, np.float32), cam)
    np.testing.assert_array_equal(nm[1:-1, 1:-1], np.broadcast_to([0.0, 0.0, -1.0], (18, 22, 3)))
    assert not nm[0].any() and not nm[-1].any() and not nm[:, 0].any() and not nm[:, -1].any()


def test_normals_of_a_tilted_plane_in_a_turned_camera():
    """Points of a plane differ by vectors in the plane, so the normal of
    the stencil is the plane's normal (turned toward the camera), up to the
    float32 rounding of the depth map; in the world frame it is R^T n."""
    R = scenes.rot_y(20.0).astype(np.float32)
    cam = _cam(R=R, t=(0.1, -0.05, 0.3))
    n = np.array([0.3, -0.2, -1.0])
    n /= np.linalg.norm(n)
    depth = _plane_depth(cam, n, -1.5)           # <n, P> = -1.5: the plane faces the camera
    assert (depth > 0).all()
    nm = oracle.normals(depth, cam).astype(np.float64)
    want = np.asarray(cam.R, np.float64).T @ n
    np.testing.assert_allclose(nm[1:-1, 1:-1].reshape(-1, 3), np.broadcast_to(want, (18 * 22, 3)), atol=2e-5)


def test_normals_need_five_positive_depths():
    cam = _cam()
    d = np.full((20, 24), 1.5, np.float32)
    d[7, 9] = 0.0
    nm = oracle.normals(d, cam)
    for (y, x) in [(7, 9), (6, 9), (8, 9), (7, 8), (7, 10)]:
        assert not nm[y, x].any()
    assert nm[7, 11].any() and nm[9, 9].any()


def _rgba(H, W, r, g=0, b=0):
    a = np.zeros((H, W, 4), np.uint8)
    a[..., 0], a[..., 1], a[..., 2], a[..., 3] = r, g, b, 255
    return a


def _plane_view(cam, Z, rgba, mask=None):
    depth = np.full((cam.height, cam.width), Z, np.float32)
    m = np.ones((cam.height, cam.width), np.uint8) if mask is None else mask
    return (cam, rgba, depth, m, oracle.normals(depth, cam))


def test_single_view_returns_its_colour_on_a_ramp():
    """Novel camera = source camera, plane at Z, z_fused = Z: each novel
    pixel back-projects onto its own pixel centre, and the bilinear fetch of
    a colour ramp returns the pixel's own value (the weight cancels with one
    view)."""
    cam = _cam(W=32, H=24)
    j, i = np.mgrid[0:24, 0:32]
    rgba = np.zeros((24, 32, 4), np.uint8)
    rgba[..., 0] = 7 * i
    rgba[..., 1] = 9 * j
    rgba[..., 2] = 3 * i + 2 * j
    view = _plane_view(cam, 1.25, rgba)
    rgb, ws = oracle.blend([view], cam, np.full((24, 32), 1.25, np.float32), 0.02)
    inner = (slice(1, -1), slice(1, -1))            # normals vanish on the border
    for q in range(3):
        np.testing.assert_allclose(rgb[q][inner], rgba[..., q][inner] / 255.0, rtol=0, atol=2e-6)
    assert (ws[inner] > 0).all()
    assert not ws[0].any() and not rgb[:, 0].any()


def test_weights_of_two_views_of_a_plane():
    """Plane Z = 1.6 (normal (0, 0, -1) toward every camera), novel camera at
    the origin, source cameras at x = -0.2 and x = +0.35 (identity rotation):
    w_k = cos<r, n> / |X - C_k| with cos = r_z, the whole mask and no
    occlusion, so I_blend = (w0 c0 + w1 c1) / (w0 + w1) per pixel."""
    Z = 1.6
    novel = _cam(W=40, H=30, fx=50.0, fy=50.0, cx=20.0, cy=15.0)
    c0 = _cam(W=80, H=60, fx=60.0, fy=60.0, cx=40.0, cy=30.0, t=(0.2, 0.0, 0.0))      # centre x = -0.2
    c1 = _cam(W=80, H=60, fx=60.0, fy=60.0, cx=40.0, cy=30.0, t=(-0.35, 0.0, 0.0))    # centre x = +0.35
    views = [_plane_view(c0, Z, _rgba(60, 80, 200, 40, 10)), _plane_view(c1, Z, _rgba(60, 80, 100, 240, 30))]
    rgb, ws = oracle.blend(views, novel, np.full((30, 40), Z, np.float32), 0.02)
    j, i = np.mgrid[0:30, 0:40].astype(np.float64)
    X = np.stack([(i + 0.5 - 20.0) / 50.0 * Z, (j + 0.5 - 15.0) / 50.0 * Z, np.full_like(i, Z)])
    rz = Z / np.linalg.norm(X, axis=0)
    w0 = rz / np.linalg.norm(X - np.array([-0.2, 0.0, 0.0])[:, None, None], axis=0)
    w1 = rz / np.linalg.norm(X - np.array([0.35, 0.0, 0.0])[:, None, None], axis=0)
    for q, (a, b) in enumerate([(200, 100), (40, 240), (10, 30)]):
        np.testing.assert_allclose(rgb[q], (w0 * a + w1 * b) / (w0 + w1) / 255.0, rtol=1e-6)
    np.testing.assert_allclose(ws, w0 + w1, rtol=1e-6)


def test_occluded_view_gets_no_weight():
    """View 1 sees an occluder 10 cm in front of the plane over part of its
    image: novel pixels whose point falls there take view 0's colour alone;
    elsewhere both views blend."""
    Z = 1.5
    novel = _cam(W=40, H=30, fx=50.0, fy=50.0, cx=20.0, cy=15.0)
    c0 = _cam(W=80, H=60, fx=60.0, fy=60.0, cx=40.0, cy=30.0, t=(0.1, 0.0, 0.0))
    c1 = _cam(W=80, H=60, fx=60.0, fy=60.0, cx=40.0, cy=30.0, t=(-0.1, 0.0, 0.0))
    v0 = _plane_view(c0, Z, _rgba(60, 80, 250))
    d1 = np.full((60, 80), Z, np.float32)
    d1[:, :40] = Z - 0.1
    v1 = (c1, _rgba(60, 80, 50), d1, np.ones((60, 80), np.uint8), oracle.normals(d1, c1))
    rgb, ws = oracle.blend([v0, v1], novel, np.full((30, 40), Z, np.float32), 0.02)
    # view 1's centre is at x = +0.1 (t = -R C), so novel pixel column i
    # sees it at u1 = 60 (X - 0.1) / Z + 40 with X = (i + 0.5 - 20) / 50 Z
    i = np.arange(40)
    u1 = 60.0 * ((i + 0.5 - 20.0) / 50.0 * Z - 0.1) / Z + 40.0
    occl = u1 < 39.0                                # all four taps on the occluder
    free = u1 > 42.0
    inner = slice(2, -2)
    np.testing.assert_array_equal(rgb[0][inner][:, occl], np.float32(250 / 255.0))
    both = rgb[0][inner][:, free]
    assert (both < 250 / 255.0 - 0.05).all() and (both > 50 / 255.0 + 0.05).all()


def test_mask_zero_removes_a_view_and_fades_at_its_border():
    cam = _cam(W=32, H=24)
    other = _cam(W=32, H=24, t=(-0.05, 0.0, 0.0))
    mask = np.ones((24, 32), np.uint8)
    mask[:, 16:] = 0
    v0 = _plane_view(cam, 1.4, _rgba(24, 32, 255), mask)
    v1 = _plane_view(other, 1.4, _rgba(24, 32, 0))
    rgb, ws = oracle.blend([v0, v1], cam, np.full((24, 32), 1.4, np.float32), 0.02)
    # where view 0's mask is 0 only view 1 (black) contributes
    assert not rgb[0][2:-2, 17:-2].any()
    assert (rgb[0][2:-2, 2:15] > 0.3).all()


def test_no_fused_depth_gives_nothing():
    cam = _cam()
    v = _plane_view(cam, 1.5, _rgba(20, 24, 255))
    zf = np.full((20, 24), 1.5, np.float32)
    zf[3, 4], zf[5, 6], zf[7, 8] = 0.0, np.inf, -1.0
    rgb, ws = oracle.blend([v], cam, zf, 0.02)
    for (y, x) in [(3, 4), (5, 6), (7, 8)]:
        assert ws[y, x] == 0 and not rgb[:, y, x].any()
    assert ws[10, 10] > 0
    rgb, ws = oracle.blend([v], cam, np.full((20, 24), 3.0, np.float32), 0.02)   # no view agrees
    assert not ws.any() and not rgb.any()
