"""Seeded synthetic scene generators.

These produce the inputs of the latent Gaussian rasterizer (Tele-Aloha §4.2:
per-pixel Gaussians {x, f, s, alpha} lifted from source-view depth maps and
splatted into a target camera).  They hold none of the rasterizer's
arithmetic: they only draw random numbers, unproject depth maps into world
points and build cameras.  Both the GPU path and the FP64 oracle read the
arrays produced here.

Conventions (shared by every consumer):
  * camera: world -> camera x_c = R x_w + t, OpenCV axes (x right, y down,
    z forward), pixel (i, j) has its centre at (i + 0.5, j + 0.5);
  * Gaussian arrays are structure-of-arrays float32:
      mean [3, N], scale [3, N] (activated, > 0), quat [4, N] (w, x, y, z,
      not necessarily normalised), opacity [N] in [0, 1], feat [N, C];
  * raw parameters for differentiation: log_scale = log(scale),
    opacity_logit = logit(opacity).

Random draws use numpy PCG64 (``default_rng(seed)``) in the fixed order
depth -> scale jitter -> quaternion -> opacity -> features.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Camera", "Scene", "rot_y", "rot_x", "orbit_camera", "look_at_camera",
    "make_cfg1", "make_cfg2", "make_cfg3_upstream", "make_cfg3_scaled",
    "make_cfg4_request", "make_cfg5", "make_grid_scene", "single_gaussian_scene",
    "SourceView", "make_source_views", "make_grid_source_view", "stereo_pair", "source_rgba",
    "source_depth",
]


@dataclass
class Camera:
    R: np.ndarray            # [3,3] float32, world -> camera rotation
    t: np.ndarray            # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    def as_f32(self) -> "Camera":
        return Camera(np.asarray(self.R, np.float32).reshape(3, 3),
                      np.asarray(self.t, np.float32).reshape(3),
                      float(np.float32(self.fx)), float(np.float32(self.fy)),
                      float(np.float32(self.cx)), float(np.float32(self.cy)),
                      int(self.width), int(self.height),
                      float(np.float32(self.znear)))

    def shifted(self, dcx: float, dcy: float) -> "Camera":
        return Camera(self.R.copy(), self.t.copy(), self.fx, self.fy,
                      self.cx + dcx, self.cy + dcy, self.width, self.height,
                      self.znear)


@dataclass
class Scene:
    mean: np.ndarray         # [3, N] f32
    scale: np.ndarray        # [3, N] f32 (activated)
    quat: np.ndarray         # [4, N] f32
    opacity: np.ndarray      # [N] f32 (activated)
    feat: np.ndarray         # [N, C] f32
    cam: Camera
    bg: np.ndarray = field(default=None)   # [C] f32
    name: str = ""

    def __post_init__(self):
        self.mean = np.ascontiguousarray(self.mean, np.float32)
        self.scale = np.ascontiguousarray(self.scale, np.float32)
        self.quat = np.ascontiguousarray(self.quat, np.float32)
        self.opacity = np.ascontiguousarray(self.opacity, np.float32)
        self.feat = np.ascontiguousarray(self.feat, np.float32)
        self.cam = self.cam.as_f32()
        if self.bg is None:
            self.bg = np.zeros(self.feat.shape[1], np.float32)
        self.bg = np.ascontiguousarray(self.bg, np.float32)

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @property
    def c(self) -> int:
        return int(self.feat.shape[1])

    # raw (pre-activation) parameters used by the differentiable path
    @property
    def log_scale(self) -> np.ndarray:
        return np.log(self.scale.astype(np.float64)).astype(np.float32)

    @property
    def opacity_logit(self) -> np.ndarray:
        o = self.opacity.astype(np.float64)
        o = np.clip(o, 1e-7, 1 - 1e-7)
        return np.log(o / (1 - o)).astype(np.float32)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.mean[:, idx], self.scale[:, idx], self.quat[:, idx],
                     self.opacity[idx], self.feat[idx], self.cam, self.bg,
                     self.name + "[subset]")

    def permuted(self, perm) -> "Scene":
        return self.subset(perm)

    def with_cam(self, cam: Camera) -> "Scene":
        return Scene(self.mean, self.scale, self.quat, self.opacity, self.feat,
                     cam, self.bg, self.name)


# ----------------------------------------------------------------- cameras
def rot_y(deg: float) -> np.ndarray:
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_x(deg: float) -> np.ndarray:
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _cam_from_c2w(R_c2w, C, fx, fy, cx, cy, w, h, znear=0.2) -> Camera:
    R = np.asarray(R_c2w, np.float64).T
    t = -R @ np.asarray(C, np.float64)
    return Camera(R.astype(np.float32), t.astype(np.float32), fx, fy, cx, cy,
                  w, h, znear)


def orbit_camera(yaw_deg, pitch_deg, pivot, radius, fx, fy, cx, cy, w, h):
    """Camera on a sphere of `radius` about `pivot`, looking at the pivot.
    yaw = 0, pitch = 0 is the camera at pivot - radius * z looking along +z."""
    Rc = rot_y(yaw_deg) @ rot_x(pitch_deg)
    C = np.asarray(pivot, np.float64) + Rc @ np.array([0.0, 0.0, -radius])
    return _cam_from_c2w(Rc, C, fx, fy, cx, cy, w, h)


def look_at_camera(yaw_deg, radius, fx, cx, size):
    """Camera on a horizontal arc of `radius` about the world origin."""
    return orbit_camera(yaw_deg, 0.0, (0.0, 0.0, 0.0), radius, fx, fx, cx, cx,
                        size, size)


def _unproject(cam_c2w_R, cam_C, fx, fy, cx, cy, us, vs, z):
    """Pixel centres (us + 0.5, vs + 0.5) at camera depth z -> world points."""
    xc = (us + 0.5 - cx) / fx * z
    yc = (vs + 0.5 - cy) / fy * z
    pc = np.stack([xc, yc, z], 0)                       # [3, n]
    return cam_c2w_R @ pc + np.asarray(cam_C, np.float64)[:, None]


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


# ------------------------------------------------------- config generators
def make_grid_scene(seed: int, grid: int, fx: float, c: int, target_res: int,
                    target_fx: float, yaw: float = 5.0, pitch: float = 0.0,
                    n: int | None = None, name: str = "") -> Scene:
    """The small-scene generator: a source camera at the origin looking along
    +z, one Gaussian per pixel of a `grid` x `grid` image (the first `n`
    pixels in row-major order), depth U[1, 2] m, isotropic scale
    depth/fx * lognormal(0, 0.2), random unit quaternions, opacity
    U[0.05, 0.95], C features N(0, 1).  The target camera orbits the point
    (0, 0, 1.5) by `yaw` about y (and `pitch` about x)."""
    rng = np.random.default_rng(seed)
    n_all = grid * grid
    n = n_all if n is None else int(n)
    vs, us = np.divmod(np.arange(n, dtype=np.float64), grid)
    cx = cy = grid / 2.0
    z = rng.uniform(1.0, 2.0, n)
    jit = np.exp(0.2 * rng.standard_normal(n))
    q = _random_quats(rng, n)
    o = rng.uniform(0.05, 0.95, n)
    f = rng.standard_normal((n, c))
    mean = _unproject(np.eye(3), np.zeros(3), fx, fx, cx, cy, us, vs, z)
    s = (z / fx) * jit
    scale = np.stack([s, s, s], 0)
    tc = target_res / 2.0
    cam = orbit_camera(yaw, pitch, (0.0, 0.0, 1.5), 1.5, target_fx, target_fx,
                       tc, tc, target_res, target_res)
    return Scene(mean, scale, q, o, f, cam, None, name or f"grid{grid}")


def make_cfg1(seed: int = 1) -> Scene:
    """Plain forward, tiny: 4096 Gaussians from a 64x64 source grid,
    fx = fy = 64, C = 8, target rotated 5 deg about y, 64x64, black bg."""
    return make_grid_scene(seed, 64, 64.0, 8, 64, 64.0, 5.0, name="cfg1")


def _body_mask(res: int):
    """Upper-body silhouette in normalised coordinates u', v' in [-1, 1]:
    a head ellipse over a torso rectangle, covering about 45% of the image."""
    g = (np.arange(res, dtype=np.float64) + 0.5 - res / 2.0) / (res / 2.0)
    vv, uu = np.meshgrid(g, g, indexing="ij")
    head = (uu / 0.24) ** 2 + ((vv + 0.6) / 0.30) ** 2 <= 1.0
    torso = (np.abs(uu) <= 0.63) & (vv >= -0.25)
    return head | torso, uu, vv


def _body_depth(uu, vv):
    """A smooth ellipsoidal bulge with a sine bump, clamped to [0.8, 1.5] m."""
    bulge = np.sqrt(np.maximum(0.0, 1.0 - (uu / 0.9) ** 2 - (vv / 1.2) ** 2))
    z = 1.25 - 0.35 * bulge + 0.03 * np.sin(6 * np.pi * uu) * np.sin(6 * np.pi * vv)
    return np.clip(z, 0.8, 1.5)


def make_body_scene(seed: int, src_res: int, src_fx: float, c: int,
                    target_res: int, target_fx: float, name: str = "") -> Scene:
    """Four source views on a 30 deg horizontal arc (yaw -15, -5, 5, 15 deg)
    at 1.2 m from the subject, each lifting the pixels inside an upper-body
    mask to Gaussians (depth from a smooth ellipsoid + sine bump in
    [0.8, 1.5] m), per-axis pixel-footprint scales with lognormal jitter,
    identity rotation, opacity U[0.3, 1], C features N(0, 1).  The target is
    the frontal view on the same arc."""
    rng = np.random.default_rng(seed)
    mask, uu, vv = _body_mask(src_res)
    zmap = _body_depth(uu, vv)
    vs, us = np.nonzero(mask)
    z = zmap[vs, us]
    cxs = src_res / 2.0
    means = []
    for yaw in (-15.0, -5.0, 5.0, 15.0):
        Rc = rot_y(yaw)
        C = Rc @ np.array([0.0, 0.0, -1.2])
        means.append(_unproject(Rc, C, src_fx, src_fx, cxs, cxs,
                                us.astype(np.float64), vs.astype(np.float64), z))
    mean = np.concatenate(means, 1)
    zz = np.concatenate([z] * 4)
    n = mean.shape[1]
    jit = np.exp(0.2 * rng.standard_normal((3, n)))
    scale = (zz / src_fx)[None, :] * jit
    q = np.zeros((4, n)); q[0] = 1.0
    o = rng.uniform(0.3, 1.0, n)
    f = rng.standard_normal((n, c))
    cam = look_at_camera(0.0, 1.2, target_fx, target_res / 2.0, target_res)
    return Scene(mean, scale, q, o, f, cam, None, name or f"body{src_res}")


def make_cfg2(seed: int = 2) -> Scene:
    """Realistic frame: 4 views of 512x512 (fx = 700), about 470k Gaussians,
    C = 32, 1024x1024 target with the same field of view (fx = 1400)."""
    return make_body_scene(seed, 512, 700.0, 32, 1024, 1400.0, name="cfg2")


def make_cfg3_upstream(seed: int, c: int, h: int, w: int) -> np.ndarray:
    """Upstream gradient dL/dF ~ N(0, 1), shape [C, H, W] float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((c, h, w)).astype(np.float32)


def make_cfg3_scaled(seed: int = 3) -> Scene:
    """The small-scene generator scaled to a 1024x1024 grid (N = 1,048,576,
    fx = 1024) at a 1024x1024 target with C = 32."""
    return make_grid_scene(seed, 1024, 1024.0, 32, 1024, 1024.0, 5.0,
                           name="cfg3_scaled")


def make_cfg4_request(req_id: int, base_seed: int = 40000):
    """One serving request: N ~ U{100k..1M} Gaussians from the small-scene
    generator on a ceil(sqrt(N)) grid, C = 32, target resolution drawn from
    {512, 768, 1024}, target pose jittered +-10 deg yaw / +-5 deg pitch about
    frontal."""
    rng = np.random.default_rng(base_seed + req_id)
    n = int(rng.integers(100_000, 1_000_001))
    res = int(rng.choice([512, 768, 1024]))
    yaw = float(rng.uniform(-10.0, 10.0))
    pitch = float(rng.uniform(-5.0, 5.0))
    g = int(math.ceil(math.sqrt(n)))
    sc = make_grid_scene(base_seed + req_id, g, float(g), 32, res, float(res),
                         yaw, pitch, n=n, name=f"req{req_id}")
    return sc


def serving_camera(req_id: int, base_seed: int = 41000) -> Camera:
    """Target camera of one serving request: resolution drawn from {512, 768,
    1024} (focal length equal to the resolution, as in make_cfg4_request),
    pose jittered +-10 deg yaw / +-5 deg pitch about frontal."""
    rng = np.random.default_rng(base_seed + req_id)
    res = int(rng.choice([512, 768, 1024]))
    yaw = float(rng.uniform(-10.0, 10.0))
    pitch = float(rng.uniform(-5.0, 5.0))
    return orbit_camera(yaw, pitch, (0.0, 0.0, 1.5), 1.5, float(res), float(res), res / 2.0, res / 2.0,
                        res, res)


def make_cfg5(seed: int = 50, frame: int = 0, base: Scene | None = None) -> Scene:
    """Full-resolution stress: 4 views of 2048x2048 (about 7.5M Gaussians),
    C = 32, 2048x2048 target.  Frame k perturbs the features by N(0, 0.05)."""
    sc = base if base is not None else make_body_scene(5, 2048, 2800.0, 32, 2048,
                                                       2800.0, name="cfg5")
    if frame == 0:
        return sc
    rng = np.random.default_rng(seed + frame)
    f = sc.feat + 0.05 * rng.standard_normal(sc.feat.shape).astype(np.float32)
    return Scene(sc.mean, sc.scale, sc.quat, sc.opacity, f, sc.cam, sc.bg,
                 f"cfg5_f{frame}")


def single_gaussian_scene(mean, scale, quat=(1.0, 0.0, 0.0, 0.0), opacity=0.8,
                          feat=None, cam: Camera | None = None, c: int = 8) -> Scene:
    """Tiny hand-built scenes (any number of Gaussians) for closed-form checks.
    `mean`/`scale` may be [3] or [3, N]."""
    mean = np.asarray(mean, np.float64)
    if mean.ndim == 1:
        mean = mean[:, None]
    n = mean.shape[1]
    scale = np.asarray(scale, np.float64)
    if scale.ndim == 0:
        scale = np.full((3, n), float(scale))
    elif scale.ndim == 1:
        scale = np.repeat(scale[:, None], n, 1) if scale.shape[0] == 3 else \
            np.stack([scale] * 3, 0)
    quat = np.asarray(quat, np.float64)
    if quat.ndim == 1:
        quat = np.repeat(quat[:, None], n, 1)
    op = np.broadcast_to(np.asarray(opacity, np.float64), (n,)).copy()
    if feat is None:
        feat = np.ones((n, c))
    feat = np.asarray(feat, np.float64).reshape(n, -1)
    if cam is None:
        cam = Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32),
                     64.0, 64.0, 32.0, 32.0, 64, 64)
    return Scene(mean, scale, quat, op, feat, cam, None, "hand")


# ------------------------------------------------------------ source views
@dataclass
class SourceView:
    """One source view as the lifting step receives it: the stereo module's
    disparity map (a rectified pair of baseline `baseline` metres), the
    foreground mask and the encoder's per-pixel maps.  Arrays are numpy,
    float32 unless noted: disparity [H, W], mask [H, W] uint8, feat [H, W, C],
    scale [H, W, 3] (activated), opacity [H, W] (activated)."""
    cam: Camera
    disparity: np.ndarray
    mask: np.ndarray
    feat: np.ndarray
    scale: np.ndarray
    opacity: np.ndarray
    baseline: float

    def __post_init__(self):
        self.cam = self.cam.as_f32()
        self.disparity = np.ascontiguousarray(self.disparity, np.float32)
        self.mask = np.ascontiguousarray(self.mask, np.uint8)
        self.feat = np.ascontiguousarray(self.feat, np.float32)
        self.scale = np.ascontiguousarray(self.scale, np.float32)
        self.opacity = np.ascontiguousarray(self.opacity, np.float32)
        self.baseline = float(np.float32(self.baseline))

    @property
    def c(self) -> int:
        return int(self.feat.shape[2])


def make_source_views(seed: int = 12, src_res: int = 512, src_fx: float = 700.0, c: int = 32,
                      baseline: float = 0.12, yaws=(-15.0, -5.0, 5.0, 15.0)):
    """The realistic frame's four source views as maps: the upper-body mask
    and depth surface of make_body_scene on each view of the 30 deg arc, the
    depth given as the disparity of a rectified pair with `baseline` metres
    (disparity = fx B / depth, the stand-in for the stereo module's output;
    0 outside the mask), per-pixel scale depth/fx * lognormal(0, 0.2) per
    axis, opacity U[0.3, 1], C features N(0, 1) (the stand-in for the
    encoder's heads).  Background pixels carry random maps too; only the mask
    and a positive disparity select a pixel."""
    rng = np.random.default_rng(seed)
    mask, uu, vv = _body_mask(src_res)
    zmap = _body_depth(uu, vv)
    views = []
    for yaw in yaws:
        cam = look_at_camera(yaw, 1.2, src_fx, src_res / 2.0, src_res)
        disp = np.where(mask, src_fx * baseline / zmap, 0.0)
        jit = np.exp(0.2 * rng.standard_normal((src_res, src_res, 3)))
        scale = (zmap / src_fx)[:, :, None] * jit
        o = rng.uniform(0.3, 1.0, (src_res, src_res))
        f = rng.standard_normal((src_res, src_res, c))
        views.append(SourceView(cam, disp, mask.astype(np.uint8), f, scale, o, baseline))
    return views


def make_grid_source_view(seed: int, grid: int, n: int, c: int = 32, baseline: float = 0.1):
    """One source view of the small-scene generator as maps: a camera at the
    origin looking along +z (fx = fy = grid, principal point at the centre),
    depth U[1, 2] m per pixel as a disparity map, the first `n` pixels in
    row-major order as the foreground mask, isotropic scale
    depth/fx * lognormal(0, 0.2), opacity U[0.05, 0.95], C features N(0, 1)."""
    rng = np.random.default_rng(seed)
    fx = float(grid)
    z = rng.uniform(1.0, 2.0, (grid, grid))
    jit = np.exp(0.2 * rng.standard_normal((grid, grid)))
    o = rng.uniform(0.05, 0.95, (grid, grid))
    f = rng.standard_normal((grid, grid, c))
    mask = (np.arange(grid * grid) < n).reshape(grid, grid).astype(np.uint8)
    s = (z / fx) * jit
    cam = Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), fx, fx, grid / 2.0, grid / 2.0,
                 grid, grid)
    return SourceView(cam, fx * baseline / z, mask, f, np.repeat(s[:, :, None], 3, 2), o, baseline)


def stereo_pair(cam: Camera, ipd: float = 0.064):
    """The user's left and right eye views around a target camera (§4.2
    renders both): the camera centre moved by -ipd/2 and +ipd/2 along the
    camera's own x axis, same orientation and intrinsics.  With
    x_c = R x_w + t, moving the centre by d along camera x gives
    t' = t - (d, 0, 0)."""
    out = []
    for d in (-0.5 * ipd, 0.5 * ipd):
        t = np.asarray(cam.t, np.float64) - np.array([d, 0.0, 0.0])
        out.append(Camera(np.asarray(cam.R, np.float32).copy(), t.astype(np.float32), cam.fx, cam.fy,
                          cam.cx, cam.cy, cam.width, cam.height, cam.znear))
    return out


def source_rgba(view: SourceView, seed: int) -> np.ndarray:
    """A seeded 8-bit RGBA image [H, W, 4] for a source view (the stand-in
    for the captured colour frame): smooth colour bands over the image plus
    per-pixel noise, alpha 255."""
    rng = np.random.default_rng(seed)
    H, W = view.mask.shape
    j, i = np.mgrid[0:H, 0:W].astype(np.float64)
    ph = rng.uniform(0, 2 * np.pi, 3)
    img = np.zeros((H, W, 4), np.uint8)
    for q in range(3):
        band = 128.0 + 90.0 * np.sin(2 * np.pi * (i / W * (q + 1.5)) + ph[q]) * np.cos(2 * np.pi * j / H * 1.3)
        img[..., q] = np.clip(band + rng.normal(0.0, 12.0, (H, W)), 0, 255).astype(np.uint8)
    img[..., 3] = 255
    return img


def source_depth(view: SourceView) -> np.ndarray:
    """The view's depth map [H, W] float32 from its disparity (fx B / d, 0
    where the disparity is not positive)."""
    d = view.disparity.astype(np.float64)
    z = np.where(d > 0, view.cam.fx * view.baseline / np.where(d > 0, d, 1.0), 0.0)
    return z.astype(np.float32)
