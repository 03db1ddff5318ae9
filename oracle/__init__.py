"""FP64 CPU oracle for the latent Gaussian rasterizer (Tele-Aloha §4.2).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark; never by the product package.  It
shares no code with the HIP path; both only read the same seeded scenes.

The arithmetic lives in ``tgo.cpp`` (plain C++, FP64 except for the float32
binning spec that fixes every discrete decision).  This module only marshals
numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtgo.so")
_lib = None

NPARAM_FIXED = 11   # mean(3) + log-scale(3) + quat(4) + opacity logit(1)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "tgo.cpp")
    path = os.environ.get("TGO_LIB_OVERRIDE", "") or _LIB_PATH
    if path == _LIB_PATH and (not os.path.exists(_LIB_PATH)
                              or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src)):
        from . import build as _b
        _b.build()
    lib = ct.CDLL(path)
    P = ct.c_void_p
    lib.tgo_create.restype = P
    lib.tgo_create.argtypes = [ct.c_int64, ct.c_int, P, P, P, P, P, P, ct.c_int]
    lib.tgo_destroy.argtypes = [P]
    lib.tgo_num_keys.restype = ct.c_int64
    lib.tgo_num_keys.argtypes = [P]
    lib.tgo_spec.argtypes = [P, P, P, P]
    lib.tgo_proj.argtypes = [P, P]
    lib.tgo_tile_lists.argtypes = [P, P, P]
    lib.tgo_render_fwd.argtypes = [P, P, P, P, P, P, P, P]
    lib.tgo_pixel_variants.restype = ct.c_int
    lib.tgo_pixel_variants.argtypes = [P, ct.c_int, ct.c_int, P, P]
    lib.tgo_render_brute.argtypes = [P, P, P, P]
    lib.tgo_pixel_walk.restype = ct.c_int
    lib.tgo_pixel_walk.argtypes = [P, ct.c_int, ct.c_int, P, ct.c_int]
    lib.tgo_render_bwd.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
    lib.tgo_fd.argtypes = [P, P, P, P, ct.c_int64, P, ct.c_double, P, P]
    lib.tgo_zsplat.argtypes = [P, P, ct.c_int64, ct.c_double, P, P]
    lib.tgo_normals.argtypes = [P, P, P]
    lib.tgo_blend.argtypes = [ct.c_int, P, P, P, P, P, P, P, ct.c_double, P, P]
    lib.tgo_lift.restype = ct.c_int64
    lib.tgo_lift.argtypes = [ct.c_int, ct.c_int, P, P, P, P, P, P, P, P, P, P, P, P]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cam_vector(cam) -> np.ndarray:
    """R[9], t[3], fx, fy, cx, cy, width, height, znear as FP64."""
    v = np.zeros(19, np.float64)
    v[0:9] = np.asarray(cam.R, np.float64).reshape(9)
    v[9:12] = np.asarray(cam.t, np.float64).reshape(3)
    v[12:19] = [cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.znear]
    return v


class Oracle:
    """Projection, tile lists and per-pixel FP64 blending of one scene.

    The arrays are converted to FP64 exactly (they are float32 scenes), or
    may be given directly as FP64 (perturbed parameters)."""

    def __init__(self, scene, nthreads: int = 0, *, mean=None, scale=None,
                 quat=None, opacity=None, feat=None):
        lib = _load()
        self.scene = scene
        self.cam = scene.cam
        self.n = scene.n
        self.c = scene.c
        self.W, self.H = int(scene.cam.width), int(scene.cam.height)
        self.tiles_x = (self.W + 15) // 16
        self.tiles_y = (self.H + 15) // 16
        self._arrs = [_f64(scene.mean if mean is None else mean),
                      _f64(scene.scale if scale is None else scale),
                      _f64(scene.quat if quat is None else quat),
                      _f64(scene.opacity if opacity is None else opacity),
                      _f64(scene.feat if feat is None else feat),
                      cam_vector(scene.cam)]
        self.bg = _f64(scene.bg)
        self._h = lib.tgo_create(self.n, self.c, *[_p(a) for a in self._arrs],
                                 int(nthreads))
        if not self._h:
            raise ValueError("oracle rejected the scene")

    def close(self):
        if getattr(self, "_h", None):
            _load().tgo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- binning
    @property
    def num_keys(self) -> int:
        return int(_load().tgo_num_keys(self._h))

    def spec(self):
        """(rect [4, n] int32 x0,y0,x1,y1 (-1 if culled), key [n] uint32,
        culled [n] bool) from the float32 binning spec."""
        rect = np.empty((4, self.n), np.int32)
        key = np.empty(self.n, np.uint32)
        culled = np.empty(self.n, np.uint8)
        _load().tgo_spec(self._h, _p(rect), _p(key), _p(culled))
        return rect, key, culled.astype(bool)

    def proj(self) -> np.ndarray:
        out = np.empty((self.n, 6), np.float64)
        _load().tgo_proj(self._h, _p(out))
        return out

    def tile_lists(self):
        """(tile_start [tiles + 1] int64, list [K] int32)."""
        T = self.tiles_x * self.tiles_y
        start = np.empty(T + 1, np.int64)
        lst = np.empty(self.num_keys, np.int32)
        _load().tgo_tile_lists(self._h, _p(start), _p(lst))
        return start, lst

    # ---------------------------------------------------------- forward
    def render(self, bg=None):
        """dict(feat [c, H, W], alpha, T, last, nflags [H, W], work (eval, contrib))."""
        bg = self.bg if bg is None else _f64(bg)
        F = np.empty((self.c, self.H, self.W), np.float64)
        A = np.empty((self.H, self.W), np.float64)
        T = np.empty((self.H, self.W), np.float64)
        last = np.empty((self.H, self.W), np.int32)
        nfl = np.empty((self.H, self.W), np.int32)
        work = np.zeros(2, np.int64)
        _load().tgo_render_fwd(self._h, _p(bg), _p(F), _p(A), _p(T), _p(last),
                               _p(nfl), _p(work))
        return dict(feat=F, alpha=A, T=T, last=last, nflags=nfl,
                    work=(int(work[0]), int(work[1])))

    def pixel_variants(self, px: int, py: int, bg=None):
        """Array [nv, c + 1] of (F, alpha) under every branch of the pixel's
        near-threshold decisions, or None when it has more than two."""
        bg = self.bg if bg is None else _f64(bg)
        out = np.empty((4, self.c + 1), np.float64)
        nv = _load().tgo_pixel_variants(self._h, int(px), int(py), _p(bg), _p(out))
        if nv < 0:
            return None
        return out[:nv].copy()

    def pixel_walk(self, px: int, py: int) -> np.ndarray:
        """Indices of the Gaussians a pixel's walk evaluates, in order."""
        cap = 1 << 16
        out = np.empty(cap, np.int32)
        n = _load().tgo_pixel_walk(self._h, int(px), int(py), _p(out), cap)
        return out[:min(n, cap)].copy()

    def render_brute(self, bg=None):
        bg = self.bg if bg is None else _f64(bg)
        F = np.empty((self.c, self.H, self.W), np.float64)
        A = np.empty((self.H, self.W), np.float64)
        _load().tgo_render_brute(self._h, _p(bg), _p(F), _p(A))
        return dict(feat=F, alpha=A)

    # ---------------------------------------------------------- backward
    def backward(self, d_feat, d_alpha=None, bg=None, flip_mask=None):
        """Analytic FP64 gradients w.r.t. the raw parameters.  flip_mask
        [H, W] uint8 (optional): per pixel, which near-threshold decisions
        to invert, as the index of a pixel_variants variant.

        Returns dict(g2d [n, 6] (du, dv, dA, dB, dC, d_opacity), mean [3, n],
        log_scale [3, n], quat [4, n], opacity_logit [n], feat [n, c])."""
        bg = self.bg if bg is None else _f64(bg)
        dF = _f64(d_feat)
        dA = None if d_alpha is None else _f64(d_alpha)
        fm = None
        if flip_mask is not None:
            fm = np.ascontiguousarray(flip_mask, np.uint8)
            assert fm.shape == (self.H, self.W), fm.shape
        n, c = self.n, self.c
        out = dict(g2d=np.empty((n, 6)), mean=np.empty((3, n)),
                   log_scale=np.empty((3, n)), quat=np.empty((4, n)),
                   opacity_logit=np.empty(n), feat=np.empty((n, c)))
        _load().tgo_render_bwd(self._h, _p(bg), _p(dF), _p(dA), _p(out["g2d"]),
                               _p(out["mean"]), _p(out["log_scale"]),
                               _p(out["quat"]), _p(out["opacity_logit"]),
                               _p(out["feat"]), _p(fm))
        return out

    def finite_differences(self, sel, d_feat, d_alpha=None, eps=1e-6, bg=None):
        """FP64 central differences for the Gaussians `sel`.

        Returns (fd [len(sel), 11 + c], excluded [len(sel), 11 + c] bool);
        parameter order: mean xyz, log-scale xyz, quat wxyz, opacity logit,
        features."""
        bg = self.bg if bg is None else _f64(bg)
        sel = np.ascontiguousarray(sel, np.int64)
        npar = NPARAM_FIXED + self.c
        fd = np.zeros((len(sel), npar), np.float64)
        ex = np.zeros((len(sel), npar), np.uint8)
        dF = _f64(d_feat)
        dA = None if d_alpha is None else _f64(d_alpha)
        _load().tgo_fd(self._h, _p(bg), _p(dF), _p(dA), len(sel), _p(sel),
                       float(eps), _p(fd), _p(ex))
        return fd, ex.astype(bool)


def analytic_as_matrix(grads: dict, sel) -> np.ndarray:
    """Gather the analytic gradients of `sel` in finite-difference order."""
    sel = np.asarray(sel)
    return np.concatenate([grads["mean"][:, sel].T, grads["log_scale"][:, sel].T,
                           grads["quat"][:, sel].T,
                           grads["opacity_logit"][sel][:, None],
                           grads["feat"][sel]], 1)


def lift(views, use_depth=None):
    """Gaussians lifted from source views (scenes.SourceView list) by the
    oracle, FP64: dict(mean [3, n], scale [3, n], quat [4, n] (identity),
    opacity [n], feat [n, c]) in (view, row-major pixel) order.  use_depth:
    optional list of [H, W] depth maps given instead of the disparities."""
    lib = _load()
    nv = len(views)
    c = views[0].c
    keep = []

    def arr(x, dt=np.float64):
        a = np.ascontiguousarray(x, dt)
        keep.append(a)
        return a.ctypes.data

    def ptrs(xs, dt=np.float64):
        return (ct.c_void_p * nv)(*[arr(x, dt) for x in xs])

    cams = np.concatenate([cam_vector(v.cam) for v in views])
    disp = None if use_depth is not None else ptrs([v.disparity for v in views])
    depth = ptrs(use_depth) if use_depth is not None else None
    mask = ptrs([v.mask for v in views], np.uint8)
    feat = ptrs([v.feat for v in views])
    scale = ptrs([v.scale for v in views])
    opac = ptrs([v.opacity for v in views])
    base = np.array([v.baseline for v in views], np.float64)
    args = [nv, c, _p(cams), disp, depth, mask, feat, scale, opac, _p(base)]
    n = int(lib.tgo_lift(*args, None, None, None, None))
    out = dict(mean=np.empty((3, n)), scale=np.empty((3, n)), opacity=np.empty(n), feat=np.empty((n, c)))
    lib.tgo_lift(*args, _p(out["mean"]), _p(out["scale"]), _p(out["opacity"]), _p(out["feat"]))
    q = np.zeros((4, n)); q[0] = 1.0
    out["quat"] = q
    return out


def zsplat(mean, cam, baseline=0.0):
    """Z-buffer of the points mean [3, n] (float32 values) splatted into
    `cam`, one pixel per point, nearest view depth kept: (zbuf [H, W] float32,
    +inf where empty; disparity [H, W] float32 = fx B / z, 0 where empty)."""
    m = _f64(mean)
    n = m.shape[1] if m.ndim == 2 else 0
    zb = np.empty((int(cam.height), int(cam.width)), np.float32)
    dp = np.empty_like(zb)
    _load().tgo_zsplat(_p(cam_vector(cam)), _p(m), n, float(baseline), _p(zb), _p(dp))
    return zb, dp


def normals(depth, cam):
    """Unit normals [H, W, 3] (float32, world frame) of the depth map [H, W]
    seen by `cam`, from central differences of the unprojected pixel
    centres, turned toward the camera; 0 at the border and where a depth of
    the five-point stencil is not positive."""
    d = np.ascontiguousarray(depth, np.float32)
    out = np.empty(d.shape + (3,), np.float32)
    _load().tgo_normals(_p(cam_vector(cam)), _p(d), _p(out))
    return out


def blend(views, novel_cam, z_fused, delta):
    """Occlusion-aware blending of source views into the novel camera (§4.3,
    Eq. 6-10).  views: sequence of (cam, rgba [H, W, 4] uint8, depth [H, W]
    float32, mask [H, W] uint8, normal [H, W, 3] float32).  Returns
    (rgb [3, H, W] float32 in [0, 1], wsum [H, W] float32)."""
    lib = _load()
    nv = len(views)
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dt)
        keep.append(a)
        return a.ctypes.data

    cams = np.concatenate([cam_vector(v[0]) for v in views]) if nv else np.zeros(19)
    ptrs = lambda k, dt: (ct.c_void_p * max(nv, 1))(*[arr(v[k], dt) for v in views])
    zf = np.ascontiguousarray(z_fused, np.float32)
    H, W = zf.shape
    rgb = np.empty((3, H, W), np.float32)
    ws = np.empty((H, W), np.float32)
    lib.tgo_blend(nv, _p(cams), ptrs(1, np.uint8), ptrs(2, np.float32), ptrs(3, np.uint8),
                  ptrs(4, np.float32), _p(cam_vector(novel_cam)), _p(zf), float(delta), _p(rgb), _p(ws))
    return rgb, ws
