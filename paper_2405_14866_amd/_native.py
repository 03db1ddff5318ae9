"""ctypes binding of libtg.so (include/tg.h).  Argument marshalling only.

Every function here has the name and argument order of its C counterpart.
The library must have been built (``python -m paper_2405_14866_amd.build``
or ``__graft_entry__.build()``); there is no fallback: importing this
module without the library raises.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtg.so")

TG_OK = 0
TG_PENDING = 1
TG_ERR_INVALID = -1
TG_ERR_OOM = -2
TG_ERR_CAPACITY = -3
TG_ERR_BUDGET = -4
TG_ERR_HIP = -5
TG_ERR_UNSUPPORTED = -6
TG_ERR_NOT_FOUND = -7

# every symbol include/tg.h declares
EXPORTS = [
    "tg_status_string", "tg_ctx_create", "tg_ctx_destroy", "tg_frame_create",
    "tg_frame_destroy", "tg_project", "tg_bin_sort", "tg_render_fwd", "tg_render_bwd",
    "tg_frame_check", "tg_frame_lists", "tg_frame_pixel_state", "tg_render_fwd_counted",
    "tg_frame_work", "tg_serve_create", "tg_serve_stream_arena", "tg_serve_submit",
    "tg_serve_poll", "tg_serve_wait", "tg_serve_release", "tg_serve_destroy",
    "tg_render_noalloc", "tg_lifter_create", "tg_lifter_destroy", "tg_lift",
    "tg_zsplat", "tg_frame_create_views", "tg_project_views", "tg_render_fwd_views",
    "tg_render_bwd_views", "tg_depth_normals", "tg_blend_views",
]

# limits of tg_render_noalloc (include/tg.h)
TG_NOALLOC_MAX_N = 524288
TG_NOALLOC_MAX_KEYS = 2097152
TG_NOALLOC_MAX_PIXELS = 1048576
TG_NOALLOC_MAX_TILES = 8192


class tg_camera(ct.Structure):
    _fields_ = [("R", ct.c_float * 9), ("t", ct.c_float * 3), ("fx", ct.c_float),
                ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("width", ct.c_int32), ("height", ct.c_int32), ("znear", ct.c_float)]


class tg_gaussians(ct.Structure):
    _fields_ = [("mean", ct.c_void_p), ("scale", ct.c_void_p), ("quat", ct.c_void_p),
                ("opacity", ct.c_void_p), ("feat", ct.c_void_p), ("n", ct.c_int64),
                ("c", ct.c_int32)]


class tg_grads(ct.Structure):
    _fields_ = [("d_mean", ct.c_void_p), ("d_log_scale", ct.c_void_p),
                ("d_quat", ct.c_void_p), ("d_opacity_logit", ct.c_void_p),
                ("d_feat", ct.c_void_p)]


class tg_serve_opts(ct.Structure):
    _fields_ = [("budget_bytes", ct.c_int64), ("slots", ct.c_int32), ("max_batch", ct.c_int32),
                ("max_gauss_per_batch", ct.c_int64), ("max_keys_per_batch", ct.c_int64),
                ("max_pixels_per_batch", ct.c_int64), ("max_side", ct.c_int32), ("c", ct.c_int32),
                ("use_graph", ct.c_int32), ("keys_per_gaussian", ct.c_float),
                ("batch_window_us", ct.c_int32), ("backward", ct.c_int32)]


class tg_request(ct.Structure):
    _fields_ = [("stream_id", ct.c_int32), ("g", tg_gaussians), ("cam", tg_camera),
                ("bg", ct.c_void_p), ("out_feat", ct.c_void_p), ("out_alpha", ct.c_void_p),
                ("d_feat", ct.c_void_p), ("d_alpha", ct.c_void_p), ("grads", tg_grads),
                ("share", ct.c_int32)]


class tg_result(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("batch_size", ct.c_int32), ("slot", ct.c_int32),
                ("retries", ct.c_int32), ("shared", ct.c_int32), ("pad", ct.c_int32),
                ("t_submit_ns", ct.c_int64), ("t_launch_ns", ct.c_int64), ("t_done_ns", ct.c_int64)]


TG_LIFT_MAX_VIEWS = 8
TG_MAX_VIEWS = 8
TG_BLEND_MAX_VIEWS = 8
TG_ZSPLAT_MAX_VIEWS = 8


class tg_source_view(ct.Structure):
    _fields_ = [("cam", tg_camera), ("disparity", ct.c_void_p), ("depth", ct.c_void_p),
                ("mask", ct.c_void_p), ("feat", ct.c_void_p), ("scale", ct.c_void_p),
                ("opacity", ct.c_void_p), ("baseline", ct.c_float)]


class tg_gaussian_buffers(ct.Structure):
    _fields_ = [("mean", ct.c_void_p), ("scale", ct.c_void_p), ("quat", ct.c_void_p),
                ("opacity", ct.c_void_p), ("feat", ct.c_void_p), ("cap", ct.c_int64)]


class tg_blend_view(ct.Structure):
    _fields_ = [("cam", tg_camera), ("rgba", ct.c_void_p), ("depth", ct.c_void_p), ("mask", ct.c_void_p),
                ("normal", ct.c_void_p)]


class TgError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib():
    """Load libtg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2405_14866_amd.build` (hipcc, gfx950)")
    L = ct.CDLL(LIB_PATH)
    P, I, I64, I32 = ct.c_void_p, ct.c_int, ct.c_int64, ct.c_int32
    L.tg_status_string.restype = ct.c_char_p
    L.tg_status_string.argtypes = [I]
    L.tg_ctx_create.restype = I
    L.tg_ctx_create.argtypes = [I, ct.POINTER(P)]
    L.tg_ctx_destroy.argtypes = [P]
    L.tg_frame_create.restype = I
    L.tg_frame_create.argtypes = [P, I64, I32, I32, I64, ct.POINTER(P)]
    L.tg_frame_destroy.argtypes = [P]
    L.tg_project.restype = I
    L.tg_project.argtypes = [P, ct.POINTER(tg_gaussians), ct.POINTER(tg_camera), P]
    L.tg_bin_sort.restype = I
    L.tg_bin_sort.argtypes = [P, P]
    L.tg_render_fwd.restype = I
    L.tg_render_fwd.argtypes = [P, ct.POINTER(tg_gaussians), P, P, P, P]
    L.tg_render_fwd_counted.restype = I
    L.tg_render_fwd_counted.argtypes = [P, ct.POINTER(tg_gaussians), P, P, P, P]
    L.tg_frame_work.restype = I
    L.tg_frame_work.argtypes = [P, ct.POINTER(I64), I32]
    L.tg_serve_create.restype = I
    L.tg_serve_create.argtypes = [P, ct.POINTER(tg_serve_opts), ct.POINTER(P)]
    L.tg_serve_stream_arena.restype = I
    L.tg_serve_stream_arena.argtypes = [P, I32, I64, ct.POINTER(tg_gaussians)]
    L.tg_serve_submit.restype = I
    L.tg_serve_submit.argtypes = [P, ct.POINTER(tg_request), ct.POINTER(ct.c_uint64)]
    L.tg_serve_poll.restype = I
    L.tg_serve_poll.argtypes = [P, ct.c_uint64, ct.POINTER(tg_result)]
    L.tg_serve_wait.restype = I
    L.tg_serve_wait.argtypes = [P, ct.c_uint64, ct.POINTER(tg_result)]
    L.tg_serve_release.restype = I
    L.tg_serve_release.argtypes = [P, ct.c_uint64]
    L.tg_serve_destroy.argtypes = [P]
    L.tg_render_bwd.restype = I
    L.tg_render_bwd.argtypes = [P, ct.POINTER(tg_gaussians), P, P, P, ct.POINTER(tg_grads), P]
    L.tg_frame_check.restype = I
    L.tg_frame_check.argtypes = [P, ct.POINTER(I64)]
    L.tg_frame_lists.restype = I
    L.tg_frame_lists.argtypes = [P, P, P, I64, P]
    L.tg_frame_pixel_state.restype = I
    L.tg_frame_pixel_state.argtypes = [P, P, P, P]
    L.tg_render_noalloc.restype = I
    L.tg_render_noalloc.argtypes = [P, ct.POINTER(tg_gaussians), ct.POINTER(tg_camera), P, P, P, P, P]
    L.tg_lifter_create.restype = I
    L.tg_lifter_create.argtypes = [P, I64, ct.POINTER(P)]
    L.tg_lifter_destroy.argtypes = [P]
    L.tg_lift.restype = I
    L.tg_lift.argtypes = [P, ct.POINTER(tg_source_view), I32, I32, ct.POINTER(tg_gaussian_buffers), P, P]
    L.tg_zsplat.restype = I
    L.tg_zsplat.argtypes = [P, P, I64, ct.POINTER(tg_camera), ct.POINTER(ct.c_float), I32, P, P, P]
    L.tg_frame_create_views.restype = I
    L.tg_frame_create_views.argtypes = [P, I32, I64, I32, I32, I64, ct.POINTER(P)]
    L.tg_project_views.restype = I
    L.tg_project_views.argtypes = [P, ct.POINTER(tg_gaussians), ct.POINTER(tg_camera), I32, P]
    L.tg_render_fwd_views.restype = I
    L.tg_render_fwd_views.argtypes = [P, ct.POINTER(tg_gaussians), P, ct.POINTER(P), ct.POINTER(P), P]
    L.tg_render_bwd_views.restype = I
    L.tg_render_bwd_views.argtypes = [P, ct.POINTER(tg_gaussians), P, ct.POINTER(P), ct.POINTER(P),
                                      ct.POINTER(tg_grads), P]
    L.tg_depth_normals.restype = I
    L.tg_depth_normals.argtypes = [P, ct.POINTER(tg_camera), P, P, P]
    L.tg_blend_views.restype = I
    L.tg_blend_views.argtypes = [P, ct.POINTER(tg_blend_view), I32, ct.POINTER(tg_camera), P, ct.c_float, P, P, P]
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().tg_status_string(int(s)).decode()


def check(status: int, what: str) -> int:
    if status not in (TG_OK, TG_PENDING):
        raise TgError(status, what)
    return status


# ------------------------------------------------------------ thin wrappers
def tg_ctx_create(device: int) -> int:
    out = ct.c_void_p()
    check(lib().tg_ctx_create(int(device), ct.byref(out)), "tg_ctx_create")
    return out.value


def tg_ctx_destroy(ctx: int) -> None:
    lib().tg_ctx_destroy(ctx)


def tg_frame_create(ctx: int, max_n: int, max_w: int, max_h: int, max_keys: int) -> int:
    out = ct.c_void_p()
    check(lib().tg_frame_create(ctx, int(max_n), int(max_w), int(max_h), int(max_keys),
                                ct.byref(out)), "tg_frame_create")
    return out.value


def tg_frame_destroy(frame: int) -> None:
    lib().tg_frame_destroy(frame)


def tg_project(frame: int, g: tg_gaussians, cam: tg_camera, stream: int) -> int:
    return lib().tg_project(frame, ct.byref(g), ct.byref(cam), stream)


def tg_bin_sort(frame: int, stream: int) -> int:
    return lib().tg_bin_sort(frame, stream)


def tg_render_fwd(frame: int, g: tg_gaussians, bg: int, out_feat: int, out_alpha: int,
                  stream: int) -> int:
    return lib().tg_render_fwd(frame, ct.byref(g), bg, out_feat, out_alpha, stream)


def tg_render_fwd_counted(frame: int, g: tg_gaussians, bg: int, out_feat: int, out_alpha: int,
                          stream: int) -> int:
    return lib().tg_render_fwd_counted(frame, ct.byref(g), bg, out_feat, out_alpha, stream)


def tg_frame_work(frame: int, n_counts: int = 5):
    """(n_eval, n_blend, wave_steps, wave_pass, wave_blend)[:n_counts]"""
    arr = (ct.c_int64 * 5)()
    check(lib().tg_frame_work(frame, arr, int(n_counts)), "tg_frame_work")
    return tuple(int(x) for x in arr[:n_counts])


def tg_render_bwd(frame: int, g: tg_gaussians, bg: int, d_feat: int, d_alpha: int,
                  grads: tg_grads, stream: int) -> int:
    return lib().tg_render_bwd(frame, ct.byref(g), bg, d_feat, d_alpha, ct.byref(grads), stream)


def tg_frame_check(frame: int):
    n = ct.c_int64(0)
    st = lib().tg_frame_check(frame, ct.byref(n))
    return st, int(n.value)


def tg_frame_lists(frame: int, tile_start: int, sorted_: int, n_keys: int, stream: int) -> int:
    return lib().tg_frame_lists(frame, tile_start, sorted_, int(n_keys), stream)


def tg_frame_pixel_state(frame: int, T_final: int, last: int, stream: int) -> int:
    return lib().tg_frame_pixel_state(frame, T_final, last, stream)


def tg_render_noalloc(ctx: int, g: tg_gaussians, cam: tg_camera, bg: int, out_feat: int,
                      out_alpha: int, status: int, stream: int) -> int:
    return lib().tg_render_noalloc(ctx, ct.byref(g), ct.byref(cam), bg, out_feat, out_alpha, status,
                                   stream)


def tg_serve_create(ctx: int, opts: tg_serve_opts) -> int:
    out = ct.c_void_p()
    check(lib().tg_serve_create(ctx, ct.byref(opts), ct.byref(out)), "tg_serve_create")
    return out.value


def tg_serve_stream_arena(srv: int, stream_id: int, max_n: int) -> tg_gaussians:
    g = tg_gaussians()
    check(lib().tg_serve_stream_arena(srv, int(stream_id), int(max_n), ct.byref(g)),
          "tg_serve_stream_arena")
    return g


def tg_serve_submit(srv: int, req: tg_request):
    """(status, ticket)"""
    t = ct.c_uint64(0)
    st = lib().tg_serve_submit(srv, ct.byref(req), ct.byref(t))
    return st, int(t.value)


def tg_serve_poll(srv: int, ticket: int):
    r = tg_result()
    st = lib().tg_serve_poll(srv, ct.c_uint64(ticket), ct.byref(r))
    return st, r


def tg_serve_wait(srv: int, ticket: int):
    r = tg_result()
    st = lib().tg_serve_wait(srv, ct.c_uint64(ticket), ct.byref(r))
    return st, r


def tg_serve_release(srv: int, ticket: int) -> int:
    return lib().tg_serve_release(srv, ct.c_uint64(ticket))


def tg_serve_destroy(srv: int) -> None:
    lib().tg_serve_destroy(srv)


def tg_lifter_create(ctx: int, max_pixels: int) -> int:
    out = ct.c_void_p()
    check(lib().tg_lifter_create(ctx, int(max_pixels), ct.byref(out)), "tg_lifter_create")
    return out.value


def tg_lifter_destroy(lifter: int) -> None:
    lib().tg_lifter_destroy(lifter)


def tg_lift(lifter: int, views, c: int, out: tg_gaussian_buffers, n_out: int, stream: int) -> int:
    arr = (tg_source_view * len(views))(*views)
    return lib().tg_lift(lifter, arr, len(views), int(c), ct.byref(out), n_out, stream)


def tg_zsplat(ctx: int, mean: int, n: int, cams, baselines, zbuf: int, disparity: int, stream: int) -> int:
    ca = (tg_camera * len(cams))(*cams)
    ba = None if baselines is None else (ct.c_float * len(cams))(*[float(b) for b in baselines])
    return lib().tg_zsplat(ctx, mean, int(n), ca, ba, len(cams), zbuf, disparity, stream)


def _ptr_array(ptrs):
    return None if ptrs is None else (ct.c_void_p * len(ptrs))(*ptrs)


def tg_frame_create_views(ctx: int, max_views: int, max_n: int, max_w: int, max_h: int, max_keys: int) -> int:
    out = ct.c_void_p()
    check(lib().tg_frame_create_views(ctx, int(max_views), int(max_n), int(max_w), int(max_h), int(max_keys),
                                      ct.byref(out)), "tg_frame_create_views")
    return out.value


def tg_project_views(frame: int, g: tg_gaussians, cams, stream: int) -> int:
    ca = (tg_camera * len(cams))(*cams)
    return lib().tg_project_views(frame, ct.byref(g), ca, len(cams), stream)


def tg_render_fwd_views(frame: int, g: tg_gaussians, bg: int, out_feat, out_alpha, stream: int) -> int:
    return lib().tg_render_fwd_views(frame, ct.byref(g), bg, _ptr_array(out_feat), _ptr_array(out_alpha), stream)


def tg_render_bwd_views(frame: int, g: tg_gaussians, bg: int, d_feat, d_alpha, grads: tg_grads, stream: int) -> int:
    return lib().tg_render_bwd_views(frame, ct.byref(g), bg, _ptr_array(d_feat), _ptr_array(d_alpha),
                                     ct.byref(grads), stream)


def tg_depth_normals(ctx: int, cam: tg_camera, depth: int, normal: int, stream: int) -> int:
    return lib().tg_depth_normals(ctx, ct.byref(cam), depth, normal, stream)


def tg_blend_views(ctx: int, views, novel: tg_camera, z_fused: int, delta: float, out_rgb: int, out_wsum: int,
                   stream: int) -> int:
    arr = (tg_blend_view * max(1, len(views)))(*views)
    return lib().tg_blend_views(ctx, arr, len(views), ct.byref(novel), z_fused, float(delta), out_rgb, out_wsum,
                                stream)
