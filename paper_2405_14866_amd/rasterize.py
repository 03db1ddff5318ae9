"""Torch-facing wrapper of libtg: device memory and streams only.

Every step of the rasterizer runs in the HIP kernels behind include/tg.h;
this module allocates output tensors, passes raw device pointers and the
current HIP stream, and applies the parameter activations of the
differentiable path (scale = exp(log_scale), opacity = sigmoid(logit)),
which the paper's encoder heads produce directly (§4.2, Eq. 4).
"""
from __future__ import annotations

import ctypes as ct
import math
import threading
import weakref
from typing import Optional

import torch

from . import _native as N

__all__ = ["Context", "Frame", "Rasterizer", "rasterize", "camera_struct", "GaussianSoA", "empty_grads"]


def empty_grads(n: int, c: int, device="cuda") -> dict:
    """Gradient buffers of one Gaussian set, SoA like the inputs: mean [3, N],
    log_scale [3, N], quat [4, N], opacity_logit [N], feat [N, C]."""
    f = lambda *shape: torch.empty(shape, dtype=torch.float32, device=device)
    return dict(mean=f(3, n), log_scale=f(3, n), quat=f(4, n), opacity_logit=f(n), feat=f(n, c))


def camera_struct(cam) -> N.tg_camera:
    """tg_camera from an object (or dict) with R, t, fx, fy, cx, cy, width,
    height and optional znear."""
    get = (lambda k, d=None: cam.get(k, d)) if isinstance(cam, dict) else \
        (lambda k, d=None: getattr(cam, k, d))
    c = N.tg_camera()
    R = [float(x) for x in torch.as_tensor(get("R"), dtype=torch.float32).reshape(-1).tolist()]
    t = [float(x) for x in torch.as_tensor(get("t"), dtype=torch.float32).reshape(-1).tolist()]
    c.R = (ct.c_float * 9)(*R)
    c.t = (ct.c_float * 3)(*t)
    c.fx, c.fy, c.cx, c.cy = float(get("fx")), float(get("fy")), float(get("cx")), float(get("cy"))
    c.width, c.height = int(get("width")), int(get("height"))
    c.znear = float(get("znear", 0.2))
    return c


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libtg takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libtg takes contiguous tensors")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class GaussianSoA:
    """Structure-of-arrays device tensors of one Gaussian set (float32):
    mean [3, N], scale [3, N], quat [4, N], opacity [N], feat [N, C]."""

    def __init__(self, mean, scale, quat, opacity, feat):
        self.mean, self.scale, self.quat = mean, scale, quat
        self.opacity, self.feat = opacity, feat
        for t in (mean, scale, quat, opacity, feat):
            if t.dtype != torch.float32:
                raise ValueError("float32 tensors expected")
        self.n = int(mean.shape[1])
        self.c = int(feat.shape[1])

    @staticmethod
    def from_scene(scene, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        return GaussianSoA(f(scene.mean), f(scene.scale), f(scene.quat), f(scene.opacity),
                           f(scene.feat))

    def struct(self) -> N.tg_gaussians:
        g = N.tg_gaussians()
        g.mean, g.scale, g.quat = _ptr(self.mean), _ptr(self.scale), _ptr(self.quat)
        g.opacity, g.feat = _ptr(self.opacity), _ptr(self.feat)
        g.n, g.c = self.n, self.c
        return g


class Context:
    _by_device = {}

    def __init__(self, device: int = 0):
        self.device = int(device)
        self.handle = N.tg_ctx_create(self.device)

    @classmethod
    def get(cls, device: int = 0) -> "Context":
        if device not in cls._by_device:
            cls._by_device[device] = Context(device)
        return cls._by_device[device]


class Frame:
    """Resident workspace of one render (see tg_frame_create)."""

    def __init__(self, ctx: Context, max_n: int, max_w: int, max_h: int, max_keys: int, max_views: int = 1):
        self.ctx = ctx
        self.max_n, self.max_w, self.max_h, self.max_keys = int(max_n), int(max_w), int(max_h), int(max_keys)
        self.max_views = int(max_views)
        self.handle = N.tg_frame_create_views(ctx.handle, self.max_views, self.max_n, self.max_w, self.max_h,
                                              self.max_keys)
        self.generation = 0

    def close(self):
        if getattr(self, "handle", None):
            N.tg_frame_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fits(self, n, w, h, keys=0, views=1):
        return (n <= self.max_n and w <= self.max_w and h <= self.max_h and keys <= self.max_keys
                and views <= self.max_views)


class Rasterizer:
    """Runs project -> bin_sort -> render_fwd (and the adjoint) on one frame,
    growing the frame when a scene needs more room."""

    def __init__(self, device: int = 0, max_n: int = 1 << 16, max_w: int = 256, max_h: int = 256,
                 keys_per_gaussian: float = 8.0, max_keys: Optional[int] = None, max_views: int = 1):
        self.device = int(device)
        self.ctx = Context.get(self.device)
        self.kpg = float(keys_per_gaussian)
        self.frame = Frame(self.ctx, max_n, max_w, max_h,
                           max_keys or max(1024, int(max_n * self.kpg * max_views)), max_views)
        self.n_keys = 0
        # the autograd node of the last differentiable render still awaiting
        # its backward (a weak reference: dead once that graph is dropped)
        self.pending = None

    def busy(self) -> bool:
        return self.pending is not None and self.pending() is not None

    def _ensure(self, n, w, h, keys=0, views=1):
        f = self.frame
        if not f.fits(n, w, h, keys, views):
            nn, ww, hh = max(n, f.max_n), max(w, f.max_w), max(h, f.max_h)
            vv = max(views, f.max_views)
            kk = max(keys, f.max_keys, int(nn * self.kpg * vv))
            f.close()
            self.frame = Frame(self.ctx, nn, ww, hh, min(kk, (1 << 31) - 1), vv)

    def project_bin(self, g: GaussianSoA, cam, stream=None, check: bool = True):
        c = camera_struct(cam)
        self._ensure(g.n, c.width, c.height)
        s = _stream(stream)
        gs = g.struct()
        for _ in range(3):
            N.check(N.tg_project(self.frame.handle, gs, c, s), "tg_project")
            N.check(N.tg_bin_sort(self.frame.handle, s), "tg_bin_sort")
            if not check:
                return c
            st, nk = N.tg_frame_check(self.frame.handle)
            self.n_keys = nk
            if st == N.TG_OK:
                return c
            if st != N.TG_ERR_CAPACITY:
                N.check(st, "tg_frame_check")
            self._ensure(g.n, c.width, c.height, int(nk * 1.25) + 1024)
        raise N.TgError(N.TG_ERR_CAPACITY, "binning")

    def forward(self, g: GaussianSoA, cam, bg: Optional[torch.Tensor] = None, stream=None,
                check: bool = True, out=None):
        """Returns (feat [C, H, W], alpha [H, W]) float32 on the device."""
        c = self.project_bin(g, cam, stream, check)
        H, W = c.height, c.width
        dev = g.mean.device
        if out is None:
            feat = torch.empty((g.c, H, W), dtype=torch.float32, device=dev)
            alpha = torch.empty((H, W), dtype=torch.float32, device=dev)
        else:
            feat, alpha = out
        N.check(N.tg_render_fwd(self.frame.handle, g.struct(), _ptr(bg), _ptr(feat), _ptr(alpha),
                                _stream(stream)), "tg_render_fwd")
        self.frame.generation += 1
        return feat, alpha

    def backward(self, g: GaussianSoA, d_feat: torch.Tensor, d_alpha: Optional[torch.Tensor] = None,
                 bg: Optional[torch.Tensor] = None, stream=None):
        """Gradients w.r.t. the raw parameters of the last forward, SoA:
        dict(mean [3, N], log_scale [3, N], quat [4, N], opacity_logit [N],
        feat [N, C])."""
        out = empty_grads(g.n, g.c, g.mean.device)
        gr = N.tg_grads()
        gr.d_mean, gr.d_log_scale, gr.d_quat = _ptr(out["mean"]), _ptr(out["log_scale"]), _ptr(out["quat"])
        gr.d_opacity_logit, gr.d_feat = _ptr(out["opacity_logit"]), _ptr(out["feat"])
        N.check(N.tg_render_bwd(self.frame.handle, g.struct(), _ptr(bg), _ptr(d_feat.contiguous()),
                                _ptr(None if d_alpha is None else d_alpha.contiguous()), gr,
                                _stream(stream)), "tg_render_bwd")
        return out

    # --------------------------------------------- several target views
    def project_bin_views(self, g: GaussianSoA, cams, stream=None, check: bool = True):
        cs = [camera_struct(c) for c in cams]
        self._ensure(g.n, max(c.width for c in cs), max(c.height for c in cs), views=len(cs))
        s = _stream(stream)
        gs = g.struct()
        for _ in range(3):
            N.check(N.tg_project_views(self.frame.handle, gs, cs, s), "tg_project_views")
            N.check(N.tg_bin_sort(self.frame.handle, s), "tg_bin_sort")
            if not check:
                return cs
            st, nk = N.tg_frame_check(self.frame.handle)
            self.n_keys = nk
            if st == N.TG_OK:
                return cs
            if st != N.TG_ERR_CAPACITY:
                N.check(st, "tg_frame_check")
            self._ensure(g.n, max(c.width for c in cs), max(c.height for c in cs), int(nk * 1.25) + 1024,
                         len(cs))
        raise N.TgError(N.TG_ERR_CAPACITY, "binning")

    def forward_views(self, g: GaussianSoA, cams, bg: Optional[torch.Tensor] = None, stream=None,
                      check: bool = True):
        """Render the set into every camera of `cams` together (one
        projection, one binning, one blend launch; e.g. a stereo pair).
        Returns a list of (feat [C, H, W], alpha [H, W])."""
        cs = self.project_bin_views(g, cams, stream, check)
        dev = g.mean.device
        outs = [(torch.empty((g.c, c.height, c.width), dtype=torch.float32, device=dev),
                 torch.empty((c.height, c.width), dtype=torch.float32, device=dev)) for c in cs]
        N.check(N.tg_render_fwd_views(self.frame.handle, g.struct(), _ptr(bg), [_ptr(f) for f, _ in outs],
                                      [_ptr(a) for _, a in outs], _stream(stream)), "tg_render_fwd_views")
        self.frame.generation += 1
        return outs

    def backward_views(self, g: GaussianSoA, d_feats, d_alphas=None, bg: Optional[torch.Tensor] = None,
                       stream=None):
        """Gradients of the loss summed over the views of the last
        forward_views (layout as backward)."""
        out = empty_grads(g.n, g.c, g.mean.device)
        gr = N.tg_grads()
        gr.d_mean, gr.d_log_scale, gr.d_quat = _ptr(out["mean"]), _ptr(out["log_scale"]), _ptr(out["quat"])
        gr.d_opacity_logit, gr.d_feat = _ptr(out["opacity_logit"]), _ptr(out["feat"])
        df = [d.contiguous() for d in d_feats]
        da = None if d_alphas is None else [None if d is None else d.contiguous() for d in d_alphas]
        N.check(N.tg_render_bwd_views(self.frame.handle, g.struct(), _ptr(bg), [_ptr(d) for d in df],
                                      None if da is None else [_ptr(d) for d in da], gr, _stream(stream)),
                "tg_render_bwd_views")
        return out

    # -------------------------------------------------------- introspection
    def tile_lists(self, cam, stream=None):
        """(tile_start [n_tiles + 1], sorted [K]) int32 device copies of the last binning."""
        c = camera_struct(cam)
        nt = ((c.width + 15) // 16) * ((c.height + 15) // 16)
        st, nk = N.tg_frame_check(self.frame.handle)
        N.check(st, "tg_frame_check")
        dev = torch.device("cuda", self.device)
        ts = torch.empty(nt + 1, dtype=torch.int32, device=dev)
        so = torch.empty(max(nk, 1), dtype=torch.int32, device=dev)
        N.check(N.tg_frame_lists(self.frame.handle, _ptr(ts), _ptr(so), nk, _stream(stream)), "tg_frame_lists")
        return ts, so[:nk]

    def pixel_state(self, cam, stream=None):
        """(T_final [H, W] float32, last [H, W] int32) device copies of the last forward."""
        c = camera_struct(cam)
        dev = torch.device("cuda", self.device)
        T = torch.empty((c.height, c.width), dtype=torch.float32, device=dev)
        last = torch.empty((c.height, c.width), dtype=torch.int32, device=dev)
        N.check(N.tg_frame_pixel_state(self.frame.handle, _ptr(T), _ptr(last), _stream(stream)),
                "tg_frame_pixel_state")
        return T, last


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, feats, rast, cam, bg):
        g = GaussianSoA(means.detach().t().contiguous(), torch.exp(log_scales.detach()).t().contiguous(),
                        quats.detach().t().contiguous(), torch.sigmoid(opacity_logits.detach()).contiguous(),
                        feats.detach().contiguous())
        img, alpha = rast.forward(g, cam, bg)
        rast.pending = weakref.ref(ctx)
        ctx.rast, ctx.g, ctx.bg = rast, g, bg
        ctx.generation = rast.frame.generation
        ctx.frame = rast.frame
        ctx.hw = tuple(alpha.shape)
        return img, alpha

    @staticmethod
    def backward(ctx, d_img, d_alpha):
        rast = ctx.rast
        if rast.frame is not ctx.frame or rast.frame.generation != ctx.generation:
            raise RuntimeError("the rasterizer rendered again before this backward; "
                               "use one Rasterizer per in-flight differentiable render")
        if d_img is None:
            d_img = torch.zeros((ctx.g.c,) + ctx.hw, device=ctx.g.mean.device)
        gr = rast.backward(ctx.g, d_img.float().contiguous(),
                           None if d_alpha is None else d_alpha.float().contiguous(), ctx.bg)
        if rast.pending is not None and rast.pending() is ctx:
            rast.pending = None
        return (gr["mean"].t(), gr["log_scale"].t(), gr["quat"].t(), gr["opacity_logit"],
                gr["feat"], None, None, None)


def rasterize(means: torch.Tensor, log_scales: torch.Tensor, quats: torch.Tensor,
              opacity_logits: torch.Tensor, feats: torch.Tensor, cam, bg: Optional[torch.Tensor] = None,
              rasterizer: Optional[Rasterizer] = None):
    """F_novel = R_G({G}, Pi_novel) (§4.2) with gradients.

    means [N, 3], log_scales [N, 3], quats [N, 4] (w, x, y, z), opacity_logits
    [N], feats [N, C] (C in 8, 16, 32, 64) -> (feat [C, H, W], alpha [H, W])."""
    if rasterizer is not None:
        return _RasterizeFn.apply(means, log_scales, quats, opacity_logits, feats, rasterizer, cam, bg)
    dev = means.device.index or 0
    c = camera_struct(cam)
    rast = _claim(dev, means.shape[0], c.width, c.height)
    try:
        return _RasterizeFn.apply(means, log_scales, quats, opacity_logits, feats, rast, cam, bg)
    finally:
        if rast.pending is _CLAIMED:
            rast.pending = None


def _CLAIMED():
    return True


_POOL: dict = {}
_POOL_LOCK = threading.Lock()


def _claim(device: int, n: int, w: int, h: int) -> Rasterizer:
    """A cached rasterizer of the device whose last differentiable render
    has been differentiated or dropped (a new one when all are in use): its
    frame is reused and grows as scenes need, so a call allocates nothing in
    the steady state."""
    with _POOL_LOCK:
        pool = _POOL.setdefault(device, [])
        for r in pool:
            if not r.busy():
                r.pending = _CLAIMED
                return r
        r = Rasterizer(device, max_n=max(1, n), max_w=w, max_h=h)
        r.pending = _CLAIMED
        pool.append(r)
        return r
