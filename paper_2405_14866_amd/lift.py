"""Torch-facing wrapper of tg_lift (include/tg.h): device memory and streams
only.  The lifting itself -- disparity to depth (§4.1), unprojection of the
foreground pixels and their encoder maps into a Gaussian set (§4.2) -- runs
in the HIP kernels of libtg."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _native as N
from .rasterize import Context, GaussianSoA, _ptr, _stream, camera_struct

__all__ = ["SourceViewMaps", "GaussianBuffers", "Lifter", "zsplat", "depth_normals", "blend_views"]


class SourceViewMaps:
    """Device maps of one source view: disparity [H, W] (or depth [H, W]),
    mask [H, W] uint8, feat [H, W, C] (channels last), scale [H, W, 3],
    opacity [H, W]; `cam` is the source camera (anything camera_struct
    accepts) and `baseline` the stereo baseline in metres."""

    def __init__(self, cam, mask, feat, scale, opacity, disparity=None, depth=None, baseline=0.0):
        if (disparity is None) == (depth is None):
            raise ValueError("give exactly one of disparity and depth")
        self.cam, self.mask, self.feat, self.scale, self.opacity = cam, mask, feat, scale, opacity
        self.disparity, self.depth, self.baseline = disparity, depth, float(baseline)

    @staticmethod
    def from_source_view(v, device="cuda") -> "SourceViewMaps":
        f = lambda a, dt=torch.float32: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        return SourceViewMaps(v.cam, f(v.mask, torch.uint8), f(v.feat), f(v.scale), f(v.opacity),
                              disparity=f(v.disparity), baseline=v.baseline)

    @property
    def c(self) -> int:
        return int(self.feat.shape[2])

    def struct(self) -> N.tg_source_view:
        s = N.tg_source_view()
        s.cam = camera_struct(self.cam)
        s.disparity, s.depth = _ptr(self.disparity), _ptr(self.depth)
        s.mask, s.feat, s.scale, s.opacity = _ptr(self.mask), _ptr(self.feat), _ptr(self.scale), _ptr(self.opacity)
        s.baseline = self.baseline
        return s


class GaussianBuffers:
    """Output buffers for up to `cap` Gaussians of C channels (flat float32
    tensors, laid out as tg_gaussian_buffers describes)."""

    def __init__(self, cap: int, c: int, device="cuda"):
        self.cap, self.c = int(cap), int(c)
        f = lambda k: torch.empty(max(1, k), dtype=torch.float32, device=device)
        self.mean, self.scale, self.quat = f(3 * self.cap), f(3 * self.cap), f(4 * self.cap)
        self.opacity, self.feat = f(self.cap), f(self.cap * self.c)

    def struct(self) -> N.tg_gaussian_buffers:
        b = N.tg_gaussian_buffers()
        b.mean, b.scale, b.quat = _ptr(self.mean), _ptr(self.scale), _ptr(self.quat)
        b.opacity, b.feat, b.cap = _ptr(self.opacity), _ptr(self.feat), self.cap
        return b

    def view(self, n: int) -> GaussianSoA:
        """The first n Gaussians as a GaussianSoA (views, no copy)."""
        n = int(n)
        return GaussianSoA(self.mean[:3 * n].view(3, n), self.scale[:3 * n].view(3, n),
                           self.quat[:4 * n].view(4, n), self.opacity[:n], self.feat[:n * self.c].view(n, self.c))


class Lifter:
    """tg_lifter: lifts source views into GaussianBuffers on the device."""

    def __init__(self, device: int = 0, max_pixels: int = 4 * 512 * 512):
        self.device = int(device)
        self.ctx = Context.get(self.device)
        self.max_pixels = int(max_pixels)
        self.handle = N.tg_lifter_create(self.ctx.handle, self.max_pixels)
        self.n_out = torch.zeros(1, dtype=torch.int64, device=f"cuda:{self.device}")

    def close(self):
        if getattr(self, "handle", None):
            N.tg_lifter_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enqueue(self, views: Sequence[SourceViewMaps], out: GaussianBuffers, stream=None) -> torch.Tensor:
        """Enqueue the lifting on the stream; returns the device count tensor."""
        c = views[0].c
        N.check(N.tg_lift(self.handle, [v.struct() for v in views], c, out.struct(),
                          _ptr(self.n_out), _stream(stream)), "tg_lift")
        return self.n_out

    def __call__(self, views: Sequence[SourceViewMaps], out: Optional[GaussianBuffers] = None,
                 stream=None) -> GaussianSoA:
        """Lift and return the Gaussian set (synchronises to read its count)."""
        if out is None:
            out = GaussianBuffers(sum(int(v.mask.numel()) for v in views), views[0].c,
                                  device=views[0].mask.device)
        self.enqueue(views, out, stream)
        n = int(self.n_out.item())
        if n > out.cap:
            raise N.TgError(N.TG_ERR_CAPACITY, f"tg_lift: {n} Gaussians for {out.cap} slots")
        return out.view(n)


def zsplat(mean: torch.Tensor, cams, baselines=None, with_disparity: bool = True, stream=None):
    """Z-buffer point splat (tg_zsplat) of the points mean [3, n] (float32,
    device) into each camera of `cams`: a list of (zbuf [H, W], disparity
    [H, W] or None) per camera."""
    ctx = Context.get(mean.device.index or 0)
    sizes = [(int(c.height), int(c.width)) for c in cams]
    total = sum(h * w for h, w in sizes)
    zb = torch.empty(max(1, total), dtype=torch.float32, device=mean.device)
    dp = torch.empty_like(zb) if with_disparity else None
    n = int(mean.shape[1]) if mean.dim() == 2 else 0
    N.check(N.tg_zsplat(ctx.handle, _ptr(mean.contiguous()) if n else None, n,
                        [camera_struct(c) for c in cams], baselines, _ptr(zb), _ptr(dp),
                        _stream(stream)), "tg_zsplat")
    out, o = [], 0
    for h, w in sizes:
        out.append((zb[o:o + h * w].view(h, w), None if dp is None else dp[o:o + h * w].view(h, w)))
        o += h * w
    return out


def depth_normals(depth: torch.Tensor, cam, stream=None) -> torch.Tensor:
    """tg_depth_normals: unit normals [H, W, 3] (world frame) of a depth map
    [H, W] (float32, device) seen by `cam`."""
    ctx = Context.get(depth.device.index or 0)
    out = torch.empty(tuple(depth.shape) + (3,), dtype=torch.float32, device=depth.device)
    N.check(N.tg_depth_normals(ctx.handle, camera_struct(cam), _ptr(depth.contiguous()), _ptr(out),
                               _stream(stream)), "tg_depth_normals")
    return out


def blend_views(views, novel_cam, z_fused: torch.Tensor, delta: float, stream=None):
    """tg_blend_views: occlusion-aware blending (§4.3).  views: sequence of
    (cam, rgba [H, W, 4] uint8, depth [H, W], mask [H, W] uint8, normal
    [H, W, 3]) device tensors.  Returns (rgb [3, H, W], wsum [H, W])."""
    ctx = Context.get(z_fused.device.index or 0)
    H, W = int(z_fused.shape[0]), int(z_fused.shape[1])
    rgb = torch.empty((3, H, W), dtype=torch.float32, device=z_fused.device)
    ws = torch.empty((H, W), dtype=torch.float32, device=z_fused.device)
    st = []
    for cam, rgba, depth, mask, normal in views:
        v = N.tg_blend_view()
        v.cam = camera_struct(cam)
        v.rgba, v.depth, v.mask, v.normal = _ptr(rgba), _ptr(depth), _ptr(mask), _ptr(normal)
        st.append(v)
    N.check(N.tg_blend_views(ctx.handle, st, camera_struct(novel_cam), _ptr(z_fused.contiguous()), delta,
                             _ptr(rgb), _ptr(ws), _stream(stream)), "tg_blend_views")
    return rgb, ws
