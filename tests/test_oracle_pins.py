"""Pins of the FP64 oracle against what the mathematics fixes.

The oracle (oracle/tgo.cpp) is the parity reference of the GPU path, so it
is checked here against things other than itself: closed forms of the EWA
splat (§4.2's Gaussian record with identity and non-identity rotations),
the front-to-back compositing closed form, invariants (weights + final T
= 1, linearity, opacity 0), brute force on tiny scenes, permutation
invariance and finite differences for its analytic backward.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _cam(fx=64.0, cx=32.0, size=64, R=None, t=None):
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    t = np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32)
    return scenes.Camera(R, t, fx, fx, cx, cx, size, size)


def _f32(x):
    return float(np.float32(x))


# ---------------------------------------------------------------- closed forms
def test_closed_form_A_on_axis_isotropic():
    g = _gold("closed_form_A.json")
    sc = scenes.single_gaussian_scene(g["mean"], g["scale"], opacity=g["opacity"],
                                      feat=[[1.0, -2.0, 0.5]], cam=_cam())
    o = oracle.Oracle(sc)
    rect, key, culled = o.spec()
    assert not culled[0]
    assert list(rect[:, 0]) == g["rect"]
    assert key[0] == np.float32(1.5).view(np.uint32)
    r = o.render()
    for e in g["alpha"]:
        i, j = e["pixel"]
        assert abs(r["alpha"][j, i] - e["value"]) < g["tolerance"]
        # F = alpha * f for a single Gaussian on a black background
        np.testing.assert_allclose(r["feat"][:, j, i], r["alpha"][j, i] * np.array([1.0, -2.0, 0.5]),
                                   rtol=0, atol=1e-15)
    # exact closed form with the float32-rounded inputs, every pixel
    s = _f32(0.03)
    v = (s * 64 / 1.5) ** 2 + 0.3
    jj, ii = np.mgrid[0:64, 0:64]
    d2 = (ii + 0.5 - 32) ** 2 + (jj + 0.5 - 32) ** 2
    a = _f32(0.8) * np.exp(-d2 / (2 * v))
    inrect = (ii >= 16) & (ii < 48) & (jj >= 16) & (jj < 48)
    expect = np.where(inrect & (a >= 1 / 255), a, 0.0)
    np.testing.assert_allclose(r["alpha"], expect, rtol=0, atol=1e-12)
    # contributing radius: pixels with alpha >= 1/255 lie within 4.5406 px
    assert np.sqrt(d2[r["alpha"] > 0]).max() < 4.5406


def test_worked_example_B_rect_is_support():
    g = _gold("worked_B.json")
    Z = g["depth"]
    s = math.sqrt(g["sigma2_raw_px2"]) * Z / 64.0
    sc = scenes.single_gaussian_scene(g["mean"], s, opacity=g["opacity"], c=1, cam=_cam())
    o = oracle.Oracle(sc)
    rect, _, _ = o.spec()
    assert rect[0, 0] == g["rect_x0"]
    r = o.render()
    ei, ej = g["empty_pixel"]
    li, lj = g["lit_pixel"]
    assert r["alpha"][ej, ei] == 0.0
    assert abs(r["alpha"][lj, li] - g["lit_alpha"]) < g["tolerance"]
    g2 = g["second"]
    o2 = oracle.Oracle(scenes.single_gaussian_scene(g2["mean"], s, opacity=g["opacity"], c=1, cam=_cam()))
    assert o2.spec()[0][0, 0] == g2["rect_x0"]
    i, j = g2["pixel"]
    assert abs(o2.render()["alpha"][j, i] - g2["alpha"]) < g["tolerance"]


def test_closed_form_C_front_to_back():
    g = _gold("closed_form_C.json")
    def run(front_depth, back_depth):
        # both on the centre of pixel (32, 32): u = fx X / Z + cx = 32.5
        means = np.array([[0.5 * front_depth / 64, 0.5 * back_depth / 64],
                          [0.5 * front_depth / 64, 0.5 * back_depth / 64],
                          [front_depth, back_depth]])
        sc = scenes.single_gaussian_scene(means, 0.01,
                                          opacity=[g["front"]["opacity"], g["back"]["opacity"]],
                                          feat=[[g["front"]["feature"]], [g["back"]["feature"]]],
                                          cam=_cam())
        r = oracle.Oracle(sc).render()
        return r["feat"][0, 32, 32], r["alpha"][32, 32]
    F, A = run(g["front"]["depth"], g["back"]["depth"])
    assert abs(F - g["F"]) < g["tolerance"]
    assert abs(A - g["alpha_out"]) < g["tolerance"]
    F2, A2 = run(g["back"]["depth"], g["front"]["depth"])
    assert abs(F2 - g["F_swapped"]) < g["tolerance"]
    assert abs(A2 - g["alpha_out"]) < g["tolerance"]


def _conic_of_diag(a, c):
    a += 0.3
    c += 0.3
    return 1.0 / a, 0.0, 1.0 / c


@pytest.mark.parametrize("case", ["aniso", "quat90z", "cam90y"])
def test_closed_form_axis_swaps(case):
    """Anisotropic scales under 90-degree rotations of the Gaussian and of the
    camera: the 2D covariance is diagonal with the permuted scales."""
    s = np.array([0.01, 0.02, 0.04])
    Z = 1.6
    fx = 64.0
    if case == "aniso":
        q = (1.0, 0.0, 0.0, 0.0); cam = _cam(); mean = [0, 0, Z]; sx, sy = s[0], s[1]
    elif case == "quat90z":
        h = math.sqrt(0.5)
        q = (h, 0.0, 0.0, h); cam = _cam(); mean = [0, 0, Z]; sx, sy = s[1], s[0]
    else:
        W = [[0, 0, -1], [0, 1, 0], [1, 0, 0]]
        q = (1.0, 0.0, 0.0, 0.0); cam = _cam(R=W); mean = [Z, 0, 0]; sx, sy = s[2], s[1]
    sc = scenes.single_gaussian_scene(mean, s, quat=q, opacity=0.7, c=1, cam=cam)
    p = oracle.Oracle(sc).proj()[0]
    A, B, C = _conic_of_diag((fx * sx / Z) ** 2, (fx * sy / Z) ** 2)
    np.testing.assert_allclose(p[:2], [32.0, 32.0], atol=1e-6)
    np.testing.assert_allclose(p[2:5], [A, B, C], rtol=2e-6, atol=2e-9)


def test_closed_form_off_axis_full_jacobian():
    """Isotropic Gaussian off the optical axis: Sigma2D = s^2 J J^T with the
    full perspective Jacobian (third column -f X / Z^2, -f Y / Z^2)."""
    X, Y, Z, s, fx = 0.4, -0.3, 1.25, 0.02, 64.0
    sc = scenes.single_gaussian_scene([X, Y, Z], s, opacity=0.9, c=1, cam=_cam())
    X, Y, Z, s = (_f32(X), _f32(Y), _f32(Z), _f32(s))
    o = oracle.Oracle(sc)
    p = o.proj()[0]
    J = np.array([[fx / Z, 0, -fx * X / Z ** 2], [0, fx / Z, -fx * Y / Z ** 2]])
    S2 = s * s * J @ J.T + 0.3 * np.eye(2)
    Q = np.linalg.inv(S2)
    np.testing.assert_allclose(p[:2], [fx * X / Z + 32, fx * Y / Z + 32], rtol=1e-12)
    np.testing.assert_allclose(p[2:5], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-9)
    # one pixel's alpha from the closed form
    r = o.render()
    i, j = int(p[0]), int(p[1])
    d = np.array([i + 0.5 - p[0], j + 0.5 - p[1]])
    assert abs(r["alpha"][j, i] - _f32(0.9) * math.exp(-0.5 * d @ Q @ d)) < 1e-12
    # the tile rectangle from the closed-form largest eigenvalue
    lam = np.linalg.eigvalsh(S2).max()
    rad = math.ceil(3 * math.sqrt(lam))
    rect, _, _ = o.spec()
    u, v = p[0], p[1]
    assert list(rect[:, 0]) == [max(0, math.floor((u - rad) / 16)), max(0, math.floor((v - rad) / 16)),
                                min(3, math.floor((u + rad) / 16)), min(3, math.floor((v + rad) / 16))]


def test_clamp_and_stop_rule():
    """o = 1 at the pixel centre clamps alpha to 0.99; three stacked o = 0.98
    Gaussians: T goes 1 -> 0.02 -> 4e-4 -> 8e-6 < 1e-4, so the third is not
    blended and the pixel stops with T = 4e-4."""
    cam = _cam()
    m = lambda z: [0.5 * z / 64, 0.5 * z / 64, z]
    sc = scenes.single_gaussian_scene(np.array(m(1.5))[:, None], 0.01, opacity=1.0, c=1, cam=cam)
    r = oracle.Oracle(sc).render()
    assert abs(r["alpha"][32, 32] - 0.99) < 1e-9
    means = np.array([m(1.2), m(1.4), m(1.6)]).T
    sc = scenes.single_gaussian_scene(means, 0.01, opacity=0.98, feat=[[1.0], [10.0], [100.0]], cam=cam)
    r = oracle.Oracle(sc).render()
    a = _f32(0.98) * math.exp(-0.0)  # centre of the pixel up to float rounding of the mean
    assert abs(r["T"][32, 32] - (1 - a) ** 2) < 1e-9
    assert r["last"][32, 32] == 1
    assert abs(r["feat"][0, 32, 32] - (a * 1 + a * (1 - a) * 10)) < 1e-7


def test_opacity_zero_gives_background(cfg1):
    sc = scenes.Scene(cfg1.mean, cfg1.scale, cfg1.quat, np.zeros(cfg1.n), cfg1.feat, cfg1.cam,
                      np.arange(cfg1.c, dtype=np.float32))
    r = oracle.Oracle(sc).render()
    assert np.all(r["alpha"] == 0.0)
    np.testing.assert_array_equal(r["feat"], np.broadcast_to(np.arange(cfg1.c)[:, None, None], r["feat"].shape))


def test_tiny_opacity_is_skipped():
    sc = scenes.single_gaussian_scene([0, 0, 1.5], 0.03, opacity=0.003, c=1, cam=_cam())
    r = oracle.Oracle(sc).render()
    assert np.all(r["alpha"] == 0.0) and np.all(r["last"] == -1)


# ---------------------------------------------------------------- invariants
def test_weights_plus_T_is_one(cfg1):
    ones = np.ones((cfg1.n, 1), np.float32)
    sc = scenes.Scene(cfg1.mean, cfg1.scale, cfg1.quat, cfg1.opacity, ones, cfg1.cam)
    r = oracle.Oracle(sc).render()
    np.testing.assert_allclose(r["feat"][0] + r["T"], 1.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["alpha"], 1.0 - r["T"], rtol=0, atol=0)


def test_linearity_in_features(cfg1):
    rng = np.random.default_rng(11)
    f2 = rng.standard_normal(cfg1.feat.shape).astype(np.float32).astype(np.float64)
    base = oracle.Oracle(cfg1).render()["feat"]
    o2 = oracle.Oracle(cfg1.with_cam(cfg1.cam), feat=f2)
    other = o2.render()["feat"]
    mix = oracle.Oracle(cfg1, feat=2.0 * cfg1.feat.astype(np.float64) - 3.0 * f2).render()["feat"]
    np.testing.assert_allclose(mix, 2.0 * base - 3.0 * other, rtol=0, atol=1e-11)
    k = oracle.Oracle(cfg1, feat=np.full(cfg1.feat.shape, 2.5)).render()
    np.testing.assert_allclose(k["feat"], np.broadcast_to(2.5 * k["alpha"][None], k["feat"].shape), rtol=0, atol=1e-12)


def test_background_enters_with_final_T(cfg1):
    bg = np.linspace(-1, 1, cfg1.c)
    o = oracle.Oracle(cfg1)
    r0 = o.render(bg=np.zeros(cfg1.c))
    r1 = o.render(bg=bg)
    np.testing.assert_allclose(r1["feat"] - r0["feat"], r0["T"][None] * bg[:, None, None], atol=1e-14)


def test_bucketed_equals_brute_force(cfg1):
    o = oracle.Oracle(cfg1)
    a, b = o.render(), o.render_brute()
    np.testing.assert_array_equal(a["feat"], b["feat"])
    np.testing.assert_array_equal(a["alpha"], b["alpha"])


def test_bucketed_equals_brute_force_body_ragged():
    """A small body scene on a ragged 72x40 target (partial edge tiles)."""
    sc = scenes.make_body_scene(7, 48, 66.0, 4, 72, 132.0)
    cam = sc.cam
    cam2 = scenes.Camera(cam.R, cam.t, cam.fx, cam.fy, 36.0, 20.0, 72, 40)
    sc = sc.with_cam(cam2)
    o = oracle.Oracle(sc)
    a, b = o.render(), o.render_brute()
    assert a["feat"].shape == (4, 40, 72)
    np.testing.assert_array_equal(a["feat"], b["feat"])
    assert (a["alpha"] > 0).mean() > 0.2


def test_tile_lists_are_the_rect_membership_sorted(cfg1):
    o = oracle.Oracle(cfg1)
    rect, key, culled = o.spec()
    start, lst = o.tile_lists()
    for t in range(o.tiles_x * o.tiles_y):
        tx, ty = t % o.tiles_x, t // o.tiles_x
        members = np.nonzero(~culled & (rect[0] <= tx) & (rect[2] >= tx) & (rect[1] <= ty) & (rect[3] >= ty))[0]
        want = members[np.lexsort((members, key[members]))]
        np.testing.assert_array_equal(lst[start[t]:start[t + 1]], want)


def test_permutation_invariance(cfg1):
    o = oracle.Oracle(cfg1)
    _, key, culled = o.spec()
    assert len(np.unique(key[~culled])) == (~culled).sum()     # distinct depths
    perm = np.random.default_rng(5).permutation(cfg1.n)
    a = o.render()
    b = oracle.Oracle(cfg1.permuted(perm)).render()
    np.testing.assert_array_equal(a["feat"], b["feat"])
    np.testing.assert_array_equal(a["alpha"], b["alpha"])


def test_principal_point_shift_by_one_tile(cfg1):
    a = oracle.Oracle(cfg1).render()
    b = oracle.Oracle(cfg1.with_cam(cfg1.cam.shifted(16.0, 16.0))).render()
    np.testing.assert_allclose(b["feat"][:, 16:, 16:], a["feat"][:, :-16, :-16], atol=1e-9)


def test_culling_cases():
    cam = _cam()
    means = np.array([[0, 0, -1.0], [0, 0, 0.1], [-5.0, 0, 1.0], [-0.53, 0, 1.0], [0, 0, 1.0]]).T
    sc = scenes.single_gaussian_scene(means, 0.01, opacity=0.5, c=1, cam=cam)
    rect, key, culled = oracle.Oracle(sc).spec()
    # behind, in front of the near plane, off-image, partly on-image, centre
    assert list(culled) == [True, True, True, False, False]
    assert rect[0, 3] == 0 and rect[2, 3] == 0


def test_variants_cover_flagged_pixels(cfg1):
    o = oracle.Oracle(cfg1)
    r = o.render()
    ys, xs = np.nonzero(r["nflags"])
    for y, x in zip(ys[:5], xs[:5]):
        v = o.pixel_variants(int(x), int(y))
        assert v is not None and v.shape[0] >= 2
        assert np.any(np.all(np.isclose(v[:, :-1], r["feat"][:, y, x][None], atol=1e-15), 1))
    v = o.pixel_variants(0, 0)
    assert v.shape[0] == 1


# ---------------------------------------------------------------- backward
def _check_fd(o, sel, dF, dA=None, bg=None):
    g = o.backward(dF, dA, bg=bg)
    fd, ex = o.finite_differences(sel, dF, dA, eps=1e-6, bg=bg)
    an = oracle.analytic_as_matrix(g, sel)
    assert ex.mean() < 0.05
    scale = np.sqrt(np.mean(an[~ex] ** 2))
    err = np.abs(fd - an)
    bad = (~ex) & (err > 1e-6 * np.abs(an) + 2e-8 * scale + 1e-9)
    assert not bad.any(), (np.argwhere(bad)[:5], err[bad][:5], an[bad][:5])
    return g, fd, ex


@pytest.mark.slow
def test_fd_cfg3_small_2048_subset(cfg1):
    """FP64 central differences (eps = 1e-6) on a seeded 2048-of-4096 subset
    of the 64x64 scene with dL/dF ~ N(0, 1) pin the analytic backward."""
    dF = scenes.make_cfg3_upstream(3, cfg1.c, 64, 64)
    sel = np.random.default_rng(3).choice(cfg1.n, 2048, replace=False)
    _check_fd(oracle.Oracle(cfg1), sel, dF)


def test_fd_anisotropic_rotated_with_alpha_grad_and_bg():
    """Anisotropic scales and random rotations (so quaternion gradients are
    non-zero), an upstream gradient on alpha and a non-black background."""
    sc = scenes.make_grid_scene(21, 24, 24.0, 3, 40, 40.0, yaw=12.0, pitch=-4.0)
    rng = np.random.default_rng(22)
    scale = sc.scale * np.exp(0.5 * rng.standard_normal(sc.scale.shape)).astype(np.float32)
    sc = scenes.Scene(sc.mean, scale, sc.quat, sc.opacity, sc.feat, sc.cam,
                      np.array([0.2, -0.1, 0.05], np.float32))
    dF = rng.standard_normal((3, 40, 40))
    dA = rng.standard_normal((40, 40))
    o = oracle.Oracle(sc)
    sel = rng.choice(sc.n, 160, replace=False)
    g, fd, ex = _check_fd(o, sel, dF, dA, bg=sc.bg)
    assert np.abs(g["quat"][:, sel]).max() > 1e-2


def test_analytic_feature_gradient_is_weight_sum(cfg1):
    """dL/df_i = sum_p alpha_i T_i dL/dF(p): with dL/dF = 1 on channel 0 and
    f = 1, the channel-0 feature gradients sum to the total rendered alpha."""
    dF = np.zeros((cfg1.c, 64, 64)); dF[0] = 1.0
    o = oracle.Oracle(cfg1)
    g = o.backward(dF)
    r = o.render()
    assert abs(g["feat"][:, 0].sum() - r["alpha"].sum()) < 1e-9
    assert np.all(g["feat"][:, 1:] == 0)


def test_backward_under_a_chosen_branch(cfg1):
    """The backward of a pixel evaluated under another branch of its
    near-threshold decisions differentiates that branch's image: with
    dL/dF = 1 at that pixel only, the feature gradient of Gaussian i is its
    blending weight alpha_i T_i in that branch, so sum_i g_i f_i reproduces
    the branch's F (given by pixel_variants) in every channel, and the
    gradients of the branches differ.  A zero mask is the plain backward."""
    o = oracle.Oracle(cfg1)
    r = o.render()
    y, x = (int(v) for v in np.argwhere(r["nflags"] > 0)[0])
    var = o.pixel_variants(x, y)
    assert var is not None and len(var) >= 2
    dF = np.zeros((cfg1.c, 64, 64)); dF[:, y, x] = 1.0
    f = np.asarray(cfg1.feat, np.float64)
    plain = o.backward(dF)
    feats = []
    for m in range(len(var)):
        mask = np.zeros((64, 64), np.uint8); mask[y, x] = m
        g = o.backward(dF, flip_mask=mask)
        np.testing.assert_allclose((g["feat"] * f).sum(0), var[m, :-1], rtol=1e-12, atol=1e-15)
        feats.append(g["feat"])
        if m == 0:
            for k in ("g2d", "feat", "mean", "quat"):
                assert np.array_equal(g[k], plain[k]), k
    assert np.abs(feats[1] - feats[0]).max() > 1e-6


# ------------------------------------------------- near-threshold branch variants
def _iso_alpha(mean, s, o, px, py, fx=64.0, cx=32.0, clamp=True):
    """Closed-form alpha of an isotropic Gaussian (identity camera) at pixel
    centre (px + 0.5, py + 0.5), from the float32-rounded inputs: Sigma2D =
    s^2 J J^T with the full perspective Jacobian, 0.3 px^2 on the diagonal,
    alpha = min(0.99, o exp(-d^T Sigma'^-1 d / 2)) (o G without the clamp
    when clamp is False)."""
    X, Y, Z = (_f32(v) for v in mean)
    s, o = _f32(s), _f32(o)
    J = np.array([[fx / Z, 0, -fx * X / Z ** 2], [0, fx / Z, -fx * Y / Z ** 2]])
    S2 = s * s * J @ J.T + 0.3 * np.eye(2)
    d = np.array([px + 0.5 - (fx * X / Z + cx), py + 0.5 - (fx * Y / Z + cx)])
    a = o * math.exp(-0.5 * d @ np.linalg.solve(S2, d))
    return min(0.99, a) if clamp else a


@pytest.mark.parametrize("delta", [3e-5, -3e-5])
def test_variants_alpha_band_closed_form(delta):
    """One Gaussian whose alpha at pixel (35, 31) is 1/255 (1 + delta), inside
    the band where an FP32 renderer may skip or blend it, on a non-black
    background.  The two variants are, in the plain walk's order first, the
    closed forms skip = (bg, 0) and blend = (alpha f + (1 - alpha) bg, alpha)."""
    mean, s = (0.0, 0.0, 1.5), 0.03
    g1 = _iso_alpha(mean, s, 1.0, 35, 31, clamp=False)    # the Gaussian factor at the pixel
    o = (1.0 / 255.0) * (1.0 + delta) / g1
    a = _iso_alpha(mean, s, o, 35, 31)
    assert abs(a * 255.0 - 1.0) < 5e-5 and (a >= 1 / 255) == (delta > 0)
    f = np.array([1.0, -2.0, 0.5])
    bg = np.array([0.3, -0.7, 0.2])
    sc = scenes.single_gaussian_scene(mean, s, opacity=o, feat=[f], cam=_cam())
    ora = oracle.Oracle(sc)
    assert ora.render(bg=bg)["nflags"][31, 35] == 1
    var = ora.pixel_variants(35, 31, bg=bg)
    skip = np.concatenate([bg, [0.0]])
    blend = np.concatenate([a * f + (1.0 - a) * bg, [a]])
    want = [blend, skip] if delta > 0 else [skip, blend]
    assert var.shape == (2, 4)
    np.testing.assert_allclose(var, np.array(want), rtol=0, atol=1e-12)


@pytest.mark.parametrize("delta", [5e-5, -5e-5])
def test_variants_transmittance_band_closed_form(delta):
    """Three Gaussians stacked on the centre of pixel (32, 32) at depths 1.2,
    1.4, 1.6 with alphas 0.95, 0.95 and a third chosen so that the
    transmittance after it is 1e-4 (1 + delta), inside the band where an FP32
    renderer may stop before it or blend it, on a non-black background.  The
    variants are the closed forms: blend all three, (sum w_i f_i + T3 bg,
    1 - T3), and stop before the third, (w1 f1 + w2 f2 + T2 bg, 1 - T2)."""
    depths = (1.2, 1.4, 1.6)
    means = [(0.5 * z / 64, 0.5 * z / 64, z) for z in depths]
    s = 0.01
    G = [_iso_alpha(m, s, 1.0, 32, 32, clamp=False) for m in means]
    o12 = [_f32(0.95 / G[0]), _f32(0.95 / G[1])]
    a1, a2 = (_iso_alpha(means[k], s, o12[k], 32, 32) for k in range(2))
    T1 = 1.0 - a1
    T2 = T1 * (1.0 - a2)
    o3 = _f32((1.0 - 1e-4 * (1.0 + delta) / T2) / G[2])
    a3 = _iso_alpha(means[2], s, o3, 32, 32)
    T3 = T2 * (1.0 - a3)
    assert abs(T3 / 1e-4 - 1.0) < 3e-4 and (T3 >= 1e-4) == (delta > 0)
    f = np.array([[1.0, 0.5], [10.0, -1.0], [100.0, 2.0]])
    bg = np.array([0.25, -0.5])
    sc = scenes.single_gaussian_scene(np.array(means).T, s, opacity=[o12[0], o12[1], o3], feat=f,
                                      cam=_cam())
    ora = oracle.Oracle(sc)
    assert ora.render(bg=bg)["nflags"][32, 32] == 1
    var = ora.pixel_variants(32, 32, bg=bg)
    w = [a1, a2 * T1, a3 * T2]
    blend = np.concatenate([w[0] * f[0] + w[1] * f[1] + w[2] * f[2] + T3 * bg, [1.0 - T3]])
    stop = np.concatenate([w[0] * f[0] + w[1] * f[1] + T2 * bg, [1.0 - T2]])
    want = [blend, stop] if delta > 0 else [stop, blend]
    assert var.shape == (2, 3)
    np.testing.assert_allclose(var, np.array(want), rtol=0, atol=1e-12)
