// tg_api.hip -- host side of the C ABI declared in include/tg.h.
//
// Contexts and frames own device workspaces allocated once at creation;
// the enqueue calls (tg_project, tg_bin_sort, tg_render_fwd, tg_render_bwd)
// validate their arguments on the host, then only launch kernels on the
// caller's stream: no allocation, no host synchronisation, no memset (the
// kernels clear what they accumulate into), so a sequence of calls can be
// captured into a HIP graph and replayed.
#include <new>

#include "../../include/tg.h"
#include "tg_internal.h"

struct tg_ctx {
  int device;
};

struct tg_frame {
  tg_ctx* ctx = nullptr;
  int device = 0;
  int64_t max_n = 0, max_keys = 0;
  int32_t max_w = 0, max_h = 0, max_tiles = 0;
  double2* xy = nullptr;
  float4* conic_o = nullptr;
  float4* wq = nullptr;
  float4* ext = nullptr;
  uint2* rect = nullptr;
  uint32_t* depth = nullptr;
  int32_t* tile_count = nullptr;
  int32_t* tile_start = nullptr;
  int32_t* tile_cursor = nullptr;
  int32_t* tile_order = nullptr;
  uint64_t* keys = nullptr;
  uint64_t* keys_tmp = nullptr;
  int32_t* sorted = nullptr;
  int2* qlist = nullptr;
  int32_t* qcount = nullptr;
  int32_t* qcut = nullptr;
  float* T_final = nullptr;
  int32_t* last = nullptr;
  float* g2d = nullptr;          // [6][g_cap] backward accumulators
  tg::FrameDev* dev = nullptr;
  int64_t g_cap = 0;             // padded Gaussian capacity (all views)
  int32_t max_views = 1;
  int64_t view_pixels = 0;       // max_w * max_h: pixel-state slice of one view
  tg::ReqDev* table_dev = nullptr;   // request table of a multi-view projection
  tg::BatchHdr* hdr_dev = nullptr;
  // state of the last projection / render
  tg::ReqDev req{};              // the request of a single-view projection
  tg::ReqDev views[TG_MAX_VIEWS]{};  // ... of a multi-view projection
  int32_t n_views = 1;
  int64_t n = -1;
  int32_t c = 0;
  tg::CamArgs cam{};
  int32_t n_tiles = 0;           // all views
  int32_t max_req_tiles = 0;     // largest view
  int64_t g_end = 0;             // padded index space of the last projection
  bool binned = false, rendered = false;
  hipStream_t last_stream = nullptr;
};

namespace tg {
int ctx_device(const tg_ctx* c) { return c->device; }
hipError_t noalloc_setup(int device);   // noalloc.hip
}  // namespace tg

namespace {

// The request table of a multi-view frame, copied into device memory by a
// one-lane kernel (stream-ordered and capturable, no host synchronisation).
struct TableUpload {
  tg::ReqDev r[TG_MAX_VIEWS];
  tg::BatchHdr h;
  tg::ReqDev* dst;
  tg::BatchHdr* hdst;
  int32_t n;
};

__global__ void k_put_table(TableUpload t) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < TG_MAX_VIEWS; ++k)
    if (k < t.n) t.dst[k] = t.r[k];
  *t.hdst = t.h;
}

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

bool valid_c(int32_t c) { return c == 8 || c == 16 || c == 32 || c == 64; }

template <class T>
tg_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) return TG_ERR_OOM;
  return TG_OK;
}

void free_frame(tg_frame* f) {
  void* ptrs[] = {f->xy, f->conic_o, f->wq, f->ext, f->rect, f->depth, f->tile_count, f->tile_start,
                  f->tile_cursor, f->tile_order, f->keys, f->keys_tmp, f->sorted, f->qlist, f->qcount, f->qcut, f->T_final,
                  f->last, f->g2d, f->dev, f->table_dev, f->hdr_dev};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

tg_status check_gaussians(const tg_frame* f, const tg_gaussians* g, bool need_c) {
  if (!g || g->n < 0 || g->n > f->max_n) return TG_ERR_INVALID;
  if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity)) return TG_ERR_INVALID;
  if (need_c) {
    if (!valid_c(g->c)) return TG_ERR_UNSUPPORTED;
    if (g->n > 0 && !g->feat) return TG_ERR_INVALID;
  }
  return TG_OK;
}

// Kernel arguments of a frame: a batch of one request passed inline, or
// the views of a multi-view projection through the device table.
tg::BatchArgs frame_args(tg_frame* f) {
  tg::BatchArgs b{};
  if (f->n_views > 1) {
    b.table = f->table_dev;
    b.hdr_dev = f->hdr_dev;
  } else {
    b.table = nullptr;
    b.hdr_dev = nullptr;
    b.one = f->req;
  }
  b.hdr.n_req = f->n_views;
  b.hdr.n_tiles = f->n_tiles;
  b.hdr.g_end = f->g_end;
  b.xy = f->xy;
  b.conic_o = f->conic_o;
  b.wq = f->wq;
  b.ext = f->ext;
  b.rect = f->rect;
  b.depth = f->depth;
  b.tile_count = f->tile_count;
  b.tile_start = f->tile_start;
  b.tile_cursor = f->tile_cursor;
  b.tile_order = f->tile_order;
  b.keys = f->keys;
  b.keys_tmp = f->keys_tmp;
  b.sorted = f->sorted;
  b.qlist = f->qlist;
  b.qcount = f->qcount;
  b.qcut = f->qcut;
  b.g2d = f->g2d;
  b.g_cap = f->g_cap;
  b.key_cap = f->max_keys;
  b.dev = f->dev;
  return b;
}

// Copy the frame's view table (and its header) to the device, on stream s.
hipError_t upload_views(tg_frame* f, hipStream_t s) {
  TableUpload t{};
  for (int k = 0; k < f->n_views; ++k) t.r[k] = f->views[k];
  t.h.n_req = f->n_views;
  t.h.n_tiles = f->n_tiles;
  t.h.g_end = f->g_end;
  t.h.n_shared = 0;
  t.dst = f->table_dev;
  t.hdst = f->hdr_dev;
  t.n = f->n_views;
  hipLaunchKernelGGL(k_put_table, dim3(1), dim3(64), 0, s, t);
  return hipGetLastError();
}

tg::CamArgs cam_args(const tg_camera* cam) {
  tg::CamArgs c;
  for (int i = 0; i < 9; ++i) c.R[i] = cam->R[i];
  for (int i = 0; i < 3; ++i) c.t[i] = cam->t[i];
  c.fx = cam->fx; c.fy = cam->fy; c.cx = cam->cx; c.cy = cam->cy; c.znear = cam->znear;
  c.W = cam->width; c.H = cam->height;
  c.tiles_x = (cam->width + tg::TILE - 1) / tg::TILE;
  c.tiles_y = (cam->height + tg::TILE - 1) / tg::TILE;
  return c;
}

}  // namespace

extern "C" {

const char* tg_status_string(tg_status s) {
  switch (s) {
    case TG_OK: return "ok";
    case TG_PENDING: return "pending";
    case TG_ERR_INVALID: return "invalid argument";
    case TG_ERR_OOM: return "out of device memory";
    case TG_ERR_CAPACITY: return "key capacity of the frame exceeded";
    case TG_ERR_BUDGET: return "request exceeds the memory budget";
    case TG_ERR_HIP: return "HIP runtime error";
    case TG_ERR_UNSUPPORTED: return "unsupported configuration";
    case TG_ERR_NOT_FOUND: return "unknown ticket";
  }
  return "unknown status";
}

tg_status tg_ctx_create(int device, tg_ctx** out) {
  if (!out) return TG_ERR_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TG_ERR_INVALID;
  DeviceGuard guard(device);
  if (tg::bin_set_attributes() != hipSuccess) return TG_ERR_HIP;
  // the static workspace of tg_render_noalloc: its address on this device
  if (tg::noalloc_setup(device) != hipSuccess) return TG_ERR_HIP;
  tg_ctx* c = new (std::nothrow) tg_ctx;
  if (!c) return TG_ERR_OOM;
  c->device = device;
  *out = c;
  return TG_OK;
}

void tg_ctx_destroy(tg_ctx* ctx) { delete ctx; }

tg_status tg_frame_create(tg_ctx* ctx, int64_t max_n, int32_t max_w, int32_t max_h,
                          int64_t max_keys, tg_frame** out) {
  return tg_frame_create_views(ctx, 1, max_n, max_w, max_h, max_keys, out);
}

tg_status tg_frame_create_views(tg_ctx* ctx, int32_t max_views, int64_t max_n, int32_t max_w,
                                int32_t max_h, int64_t max_keys, tg_frame** out) {
  if (!ctx || !out || max_views < 1 || max_views > TG_MAX_VIEWS || max_n < 0 || max_w <= 0 || max_h <= 0 ||
      max_keys <= 0 ||
      max_keys >= (int64_t)1 << 31 || max_n >= (int64_t)1 << 31 || max_w > 65535 * tg::TILE ||
      max_h > 65535 * tg::TILE)
    return TG_ERR_INVALID;
  *out = nullptr;
  DeviceGuard guard(ctx->device);
  tg_frame* f = new (std::nothrow) tg_frame;
  if (!f) return TG_ERR_OOM;
  f->ctx = ctx;
  f->device = ctx->device;
  f->max_n = max_n;
  f->max_keys = max_keys;
  f->max_w = max_w;
  f->max_h = max_h;
  const int64_t tx = (max_w + tg::TILE - 1) / tg::TILE, ty = (max_h + tg::TILE - 1) / tg::TILE;
  if (tx * ty * max_views >= ((int64_t)1 << 31) || tg::padded(max_n > 0 ? max_n : 1) * max_views > tg::MAX_GAUSS_SPACE) {
    delete f;
    return TG_ERR_INVALID;
  }
  f->max_views = max_views;
  f->max_tiles = (int32_t)(tx * ty * max_views);
  f->view_pixels = (int64_t)max_w * max_h;
  const size_t npix = (size_t)max_w * max_h * max_views;
  f->g_cap = tg::padded(max_n > 0 ? max_n : 1) * max_views;
  tg_status st = TG_OK;
  if (st == TG_OK) st = dalloc(&f->xy, f->g_cap);
  if (st == TG_OK) st = dalloc(&f->conic_o, f->g_cap);
  if (st == TG_OK) st = dalloc(&f->wq, f->g_cap);
  if (st == TG_OK) st = dalloc(&f->ext, f->g_cap);
  if (st == TG_OK) st = dalloc(&f->rect, f->g_cap);
  if (st == TG_OK) st = dalloc(&f->depth, f->g_cap);
  if (st == TG_OK) st = dalloc(&f->tile_count, f->max_tiles);
  if (st == TG_OK) st = dalloc(&f->tile_start, (size_t)f->max_tiles + 1);
  if (st == TG_OK) st = dalloc(&f->tile_cursor, f->max_tiles);
  if (st == TG_OK) st = dalloc(&f->tile_order, f->max_tiles);
  if (st == TG_OK) st = dalloc(&f->keys, max_keys);
  if (st == TG_OK) st = dalloc(&f->keys_tmp, max_keys);
  if (st == TG_OK) st = dalloc(&f->sorted, max_keys);
  if (st == TG_OK) st = dalloc(&f->qlist, 4 * (size_t)max_keys);
  if (st == TG_OK) st = dalloc(&f->qcount, 4 * (size_t)f->max_tiles);
  if (st == TG_OK) st = dalloc(&f->qcut, 4 * (size_t)f->max_tiles);
  if (st == TG_OK) st = dalloc(&f->T_final, npix);
  if (st == TG_OK) st = dalloc(&f->last, npix);
  if (st == TG_OK) st = dalloc(&f->g2d, (size_t)8 * f->g_cap);
  if (st == TG_OK) st = dalloc(&f->dev, 1);
  if (st == TG_OK && max_views > 1) st = dalloc(&f->table_dev, TG_MAX_VIEWS);
  if (st == TG_OK && max_views > 1) st = dalloc(&f->hdr_dev, 1);
  if (st == TG_OK && hipMemset(f->dev, 0, sizeof(tg::FrameDev)) != hipSuccess) st = TG_ERR_HIP;
  if (st == TG_OK && hipMemset(f->tile_start, 0, ((size_t)f->max_tiles + 1) * sizeof(int32_t)) != hipSuccess)
    st = TG_ERR_HIP;
  if (st == TG_OK && hipDeviceSynchronize() != hipSuccess) st = TG_ERR_HIP;
  if (st != TG_OK) {
    free_frame(f);
    delete f;
    return st;
  }
  *out = f;
  return TG_OK;
}

void tg_frame_destroy(tg_frame* f) {
  if (!f) return;
  DeviceGuard guard(f->device);
  (void)hipDeviceSynchronize();
  free_frame(f);
  delete f;
}

tg_status tg_project(tg_frame* f, const tg_gaussians* g, const tg_camera* cam, void* stream) {
  if (!f || !cam) return TG_ERR_INVALID;
  tg_status st = check_gaussians(f, g, false);
  if (st != TG_OK) return st;
  if (cam->width <= 0 || cam->height <= 0 || cam->width > f->max_w || cam->height > f->max_h)
    return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  const tg::CamArgs c = cam_args(cam);
  f->cam = c;
  f->n = g->n;
  f->n_views = 1;
  f->n_tiles = c.tiles_x * c.tiles_y;
  f->max_req_tiles = f->n_tiles;
  f->g_end = tg::padded(g->n);
  f->binned = f->rendered = false;
  tg::ReqDev& q = f->req;
  q = tg::ReqDev{};
  q.mean = g->mean; q.scale = g->scale; q.quat = g->quat; q.opacity = g->opacity; q.feat = g->feat;
  q.T_final = f->T_final; q.last = f->last;
  q.n = g->n; q.g_off = 0; q.tile_off = 0;
  q.cam = c;
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  return tg::launch_project(frame_args(f), tg::padded(g->n), s) == hipSuccess ? TG_OK : TG_ERR_HIP;
}

tg_status tg_bin_sort(tg_frame* f, void* stream) {
  if (!f || f->n < 0) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  if (tg::launch_bin_sort(frame_args(f), f->g_end, f->n_tiles, f->max_req_tiles, s) != hipSuccess)
    return TG_ERR_HIP;
  f->binned = true;
  return TG_OK;
}

static tg_status render_fwd_impl(tg_frame* f, const tg_gaussians* g, const float* bg,
                                 float* out_feat, float* out_alpha, void* stream, bool count) {
  if (!f || !f->binned || !out_feat || f->n_views != 1) return TG_ERR_INVALID;
  tg_status st = check_gaussians(f, g, true);
  if (st != TG_OK) return st;
  if (g->n != f->n) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  tg::ReqDev& q = f->req;
  q.feat = g->feat;
  q.bg = bg;
  q.out_feat = out_feat;
  q.out_alpha = out_alpha;
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  f->c = g->c;
  if (tg::launch_render_fwd(frame_args(f), g->c, f->n_tiles, s, count) != hipSuccess) return TG_ERR_HIP;
  f->rendered = true;
  return TG_OK;
}

tg_status tg_render_fwd(tg_frame* f, const tg_gaussians* g, const float* bg, float* out_feat,
                        float* out_alpha, void* stream) {
  return render_fwd_impl(f, g, bg, out_feat, out_alpha, stream, false);
}

tg_status tg_render_fwd_counted(tg_frame* f, const tg_gaussians* g, const float* bg, float* out_feat,
                                float* out_alpha, void* stream) {
  return render_fwd_impl(f, g, bg, out_feat, out_alpha, stream, true);
}

tg_status tg_frame_work(tg_frame* f, int64_t* counts, int32_t n_counts) {
  if (!f || !counts || n_counts < 0) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  if (hipStreamSynchronize(f->last_stream) != hipSuccess) return TG_ERR_HIP;
  tg::FrameDev d;
  if (hipMemcpy(&d, f->dev, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) return TG_ERR_HIP;
  const unsigned long long v[5] = {d.n_eval, d.n_blend, d.wave_steps, d.wave_pass, d.wave_blend};
  for (int i = 0; i < n_counts && i < 5; ++i) counts[i] = (int64_t)v[i];
  return TG_OK;
}

tg_status tg_render_bwd(tg_frame* f, const tg_gaussians* g, const float* bg, const float* d_feat,
                        const float* d_alpha, const tg_grads* out, void* stream) {
  if (!f || !f->rendered || !d_feat || !out || f->n_views != 1) return TG_ERR_INVALID;
  tg_status st = check_gaussians(f, g, true);
  if (st != TG_OK) return st;
  if (g->n != f->n || g->c != f->c) return TG_ERR_INVALID;
  if (g->n > 0 && !out->d_feat) return TG_ERR_INVALID;   // an empty set has no feature gradients
  DeviceGuard guard(f->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  tg::ReqDev& q = f->req;
  q.feat = g->feat;
  q.bg = bg;
  q.d_img = d_feat;
  q.d_alpha = d_alpha;
  q.d_mean = out->d_mean;
  q.d_log_scale = out->d_log_scale;
  q.d_quat = out->d_quat;
  q.d_logit = out->d_opacity_logit;
  q.d_feat = out->d_feat;
  if (tg::launch_render_bwd(frame_args(f), g->c, f->g_end, f->n_tiles, s) != hipSuccess)
    return TG_ERR_HIP;
  return TG_OK;
}

tg_status tg_frame_check(tg_frame* f, int64_t* n_keys) {
  if (!f) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  if (hipStreamSynchronize(f->last_stream) != hipSuccess) return TG_ERR_HIP;
  tg::FrameDev d;
  if (hipMemcpy(&d, f->dev, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) return TG_ERR_HIP;
  if (n_keys) *n_keys = d.n_keys;
  return d.overflow ? TG_ERR_CAPACITY : TG_OK;
}

tg_status tg_frame_lists(tg_frame* f, int32_t* tile_start, int32_t* sorted, int64_t n_keys,
                         void* stream) {
  if (!f || n_keys < 0 || n_keys > f->max_keys || !f->binned) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (tile_start &&
      hipMemcpyAsync(tile_start, f->tile_start, ((size_t)f->n_tiles + 1) * sizeof(int32_t),
                     hipMemcpyDeviceToDevice, s) != hipSuccess)
    return TG_ERR_HIP;
  if (sorted && n_keys > 0 &&
      hipMemcpyAsync(sorted, f->sorted, (size_t)n_keys * sizeof(int32_t), hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    return TG_ERR_HIP;
  return TG_OK;
}

tg_status tg_frame_pixel_state(tg_frame* f, float* T_final, int32_t* last, void* stream) {
  if (!f || !f->rendered) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  size_t o = 0;
  for (int v = 0; v < f->n_views; ++v) {
    const tg::CamArgs& c = f->n_views > 1 ? f->views[v].cam : f->cam;
    const size_t npix = (size_t)c.W * c.H, src = (size_t)v * f->view_pixels;
    if (T_final && hipMemcpyAsync(T_final + o, f->T_final + src, npix * sizeof(float), hipMemcpyDeviceToDevice,
                                  s) != hipSuccess)
      return TG_ERR_HIP;
    if (last && hipMemcpyAsync(last + o, f->last + src, npix * sizeof(int32_t), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
      return TG_ERR_HIP;
    o += npix;
  }
  return TG_OK;
}

tg_status tg_project_views(tg_frame* f, const tg_gaussians* g, const tg_camera* cams, int32_t n_views,
                           void* stream) {
  if (!f || !cams || n_views < 1 || n_views > f->max_views) return TG_ERR_INVALID;
  if (n_views == 1) return tg_project(f, g, cams, stream);
  tg_status st = check_gaussians(f, g, false);
  if (st != TG_OK) return st;
  for (int v = 0; v < n_views; ++v)
    if (cams[v].width <= 0 || cams[v].height <= 0 || cams[v].width > f->max_w || cams[v].height > f->max_h)
      return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  const int64_t pn = tg::padded(g->n);
  int32_t tiles = 0, most = 0;
  for (int v = 0; v < n_views; ++v) {
    tg::ReqDev& q = f->views[v];
    q = tg::ReqDev{};
    q.mean = g->mean; q.scale = g->scale; q.quat = g->quat; q.opacity = g->opacity; q.feat = g->feat;
    q.T_final = f->T_final + v * f->view_pixels;
    q.last = f->last + v * f->view_pixels;
    q.n = g->n;
    q.g_off = v * pn;
    q.s_off = q.g_off;
    q.tile_off = tiles;
    q.cam = cam_args(&cams[v]);
    q.extra_views = v == 0 ? n_views - 1 : 0;
    q.covered = v > 0 ? 1 : 0;
    const int32_t t = q.cam.tiles_x * q.cam.tiles_y;
    tiles += t;
    most = t > most ? t : most;
  }
  f->cam = f->views[0].cam;
  f->n = g->n;
  f->n_views = n_views;
  f->n_tiles = tiles;
  f->max_req_tiles = most;
  f->g_end = n_views * pn;
  f->binned = f->rendered = false;
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  if (upload_views(f, s) != hipSuccess) return TG_ERR_HIP;
  return tg::launch_project(frame_args(f), f->g_end, s) == hipSuccess ? TG_OK : TG_ERR_HIP;
}

tg_status tg_render_fwd_views(tg_frame* f, const tg_gaussians* g, const float* bg, float* const* out_feat,
                              float* const* out_alpha, void* stream) {
  if (!f || !out_feat) return TG_ERR_INVALID;
  if (f->n_views == 1) return tg_render_fwd(f, g, bg, out_feat[0], out_alpha ? out_alpha[0] : nullptr, stream);
  if (!f->binned) return TG_ERR_INVALID;
  tg_status st = check_gaussians(f, g, true);
  if (st != TG_OK) return st;
  if (g->n != f->n) return TG_ERR_INVALID;
  for (int v = 0; v < f->n_views; ++v)
    if (!out_feat[v]) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  for (int v = 0; v < f->n_views; ++v) {
    tg::ReqDev& q = f->views[v];
    q.feat = g->feat;
    q.bg = bg;
    q.out_feat = out_feat[v];
    q.out_alpha = out_alpha ? out_alpha[v] : nullptr;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  f->c = g->c;
  if (upload_views(f, s) != hipSuccess) return TG_ERR_HIP;
  if (tg::launch_render_fwd(frame_args(f), g->c, f->n_tiles, s, false) != hipSuccess) return TG_ERR_HIP;
  f->rendered = true;
  return TG_OK;
}

tg_status tg_render_bwd_views(tg_frame* f, const tg_gaussians* g, const float* bg, const float* const* d_feat,
                              const float* const* d_alpha, const tg_grads* out, void* stream) {
  if (!f || !d_feat || !out) return TG_ERR_INVALID;
  if (f->n_views == 1) return tg_render_bwd(f, g, bg, d_feat[0], d_alpha ? d_alpha[0] : nullptr, out, stream);
  if (!f->rendered) return TG_ERR_INVALID;
  tg_status st = check_gaussians(f, g, true);
  if (st != TG_OK) return st;
  if (g->n != f->n || g->c != f->c) return TG_ERR_INVALID;
  if (g->n > 0 && !out->d_feat) return TG_ERR_INVALID;
  for (int v = 0; v < f->n_views; ++v)
    if (!d_feat[v]) return TG_ERR_INVALID;
  DeviceGuard guard(f->device);
  for (int v = 0; v < f->n_views; ++v) {
    tg::ReqDev& q = f->views[v];
    q.feat = g->feat;
    q.bg = bg;
    q.d_img = d_feat[v];
    q.d_alpha = d_alpha ? d_alpha[v] : nullptr;
    q.d_mean = out->d_mean;
    q.d_log_scale = out->d_log_scale;
    q.d_quat = out->d_quat;
    q.d_logit = out->d_opacity_logit;
    q.d_feat = out->d_feat;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  f->last_stream = s;
  if (upload_views(f, s) != hipSuccess) return TG_ERR_HIP;
  if (tg::launch_render_bwd(frame_args(f), g->c, f->g_end, f->n_tiles, s) != hipSuccess) return TG_ERR_HIP;
  return TG_OK;
}

}  // extern "C"
