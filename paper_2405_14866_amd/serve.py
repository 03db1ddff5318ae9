"""Torch-facing wrapper of the serving loop (tg_serve_* in include/tg.h).

Argument marshalling only: requests carry raw device pointers of torch
tensors (or of the server's per-stream arenas); the batching, admission,
graph replay and every rendering step run inside libtg.
"""
from __future__ import annotations

import ctypes as ct
from typing import Optional

import torch

from . import _native as N
from .rasterize import Context, GaussianSoA, _ptr, camera_struct

__all__ = ["Server", "Result"]


class Result:
    def __init__(self, status: int, r: N.tg_result):
        self.status = int(status)
        self.batch_size = int(r.batch_size)
        self.slot = int(r.slot)
        self.retries = int(r.retries)
        self.shared = bool(r.shared)
        self.t_submit_ns = int(r.t_submit_ns)
        self.t_launch_ns = int(r.t_launch_ns)
        self.t_done_ns = int(r.t_done_ns)

    @property
    def latency_ms(self) -> float:
        return (self.t_done_ns - self.t_submit_ns) * 1e-6

    @property
    def queue_ms(self) -> float:
        return (self.t_launch_ns - self.t_submit_ns) * 1e-6


class Server:
    """Continuous-batching render server on one GPU."""

    def __init__(self, device: int = 0, c: int = 32, budget_bytes: int = 64 << 30, slots: int = 3,
                 max_batch: int = 16, max_gauss_per_batch: int = 8_000_000,
                 max_keys_per_batch: int = 40_000_000, max_pixels_per_batch: int = 16 << 20,
                 max_side: int = 1024, use_graph: bool = True, keys_per_gaussian: float = 5.0,
                 batch_window_us: int = 0, backward: bool = False):
        self.device = int(device)
        self.c = int(c)
        self.ctx = Context.get(self.device)
        o = N.tg_serve_opts()
        o.budget_bytes, o.slots, o.max_batch = int(budget_bytes), int(slots), int(max_batch)
        o.max_gauss_per_batch, o.max_keys_per_batch = int(max_gauss_per_batch), int(max_keys_per_batch)
        o.max_pixels_per_batch, o.max_side, o.c = int(max_pixels_per_batch), int(max_side), int(c)
        o.use_graph, o.keys_per_gaussian = int(bool(use_graph)), float(keys_per_gaussian)
        o.batch_window_us = int(batch_window_us)
        o.backward = int(bool(backward))
        self.opts = o
        self.handle = N.tg_serve_create(self.ctx.handle, o)
        self._keep = {}      # ticket -> objects that must outlive the request

    def close(self):
        if getattr(self, "handle", None):
            N.tg_serve_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream_arena(self, stream_id: int, max_n: int) -> N.tg_gaussians:
        """The server-owned resident buffers of a stream (device pointers)."""
        return N.tg_serve_stream_arena(self.handle, stream_id, max_n)

    def submit(self, g, cam, out_feat: torch.Tensor, out_alpha: Optional[torch.Tensor] = None,
               bg: Optional[torch.Tensor] = None, stream_id: int = 0, n: Optional[int] = None,
               d_feat: Optional[torch.Tensor] = None, d_alpha: Optional[torch.Tensor] = None,
               grads: Optional[dict] = None, share: bool = False) -> int:
        """Queue one render; g is a GaussianSoA or a tg_gaussians (arena).
        n renders only the first n Gaussians.  With d_feat (a server built
        with backward) the request also runs the adjoint and writes the
        gradients into `grads` (device tensors keyed mean, log_scale, quat,
        opacity_logit, feat, SoA as in Rasterizer.backward).  share lets it
        reuse the projection and sorted lists of an earlier request of the
        same batch and stream with identical geometry and camera.  Returns
        the ticket; raises TgError when the request is rejected."""
        req = N.tg_request()
        req.stream_id = int(stream_id)
        gs = g.struct() if isinstance(g, GaussianSoA) else g
        if n is not None:
            gs2 = N.tg_gaussians.from_buffer_copy(gs)
            gs2.n = int(n)
            gs = gs2
        req.g = gs
        req.cam = camera_struct(cam)
        req.bg = _ptr(bg)
        req.out_feat = _ptr(out_feat)
        req.out_alpha = _ptr(out_alpha)
        req.d_feat = _ptr(d_feat)
        req.d_alpha = _ptr(d_alpha)
        if grads is not None:
            req.grads.d_mean, req.grads.d_log_scale = _ptr(grads.get("mean")), _ptr(grads.get("log_scale"))
            req.grads.d_quat, req.grads.d_opacity_logit = _ptr(grads.get("quat")), _ptr(grads.get("opacity_logit"))
            req.grads.d_feat = _ptr(grads.get("feat"))
        req.share = int(bool(share))
        st, ticket = N.tg_serve_submit(self.handle, req)
        N.check(st, "tg_serve_submit")
        self._keep[ticket] = (g, out_feat, out_alpha, bg, d_feat, d_alpha, grads)
        return ticket

    def poll(self, ticket: int):
        st, r = N.tg_serve_poll(self.handle, ticket)
        return Result(st, r)

    def wait(self, ticket: int, release: bool = True) -> Result:
        st, r = N.tg_serve_wait(self.handle, ticket)
        res = Result(st, r)
        if release:
            N.tg_serve_release(self.handle, ticket)
            self._keep.pop(ticket, None)
        return res
