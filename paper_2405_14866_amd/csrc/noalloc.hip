// noalloc.hip -- tg_render_noalloc: the render sequence (projection,
// binning + sort, blend) of include/tg.h with its workspace in a static
// device array instead of a tg_frame, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The workspace is one file-scope __device__ array, `scratch`, sized for the
// largest render it accepts (the TG_NOALLOC_MAX_* limits of include/tg.h:
// 524,288 Gaussians, 2,097,152 (tile, Gaussian) keys, 1,048,576 pixels,
// 8,192 tiles; 150 MiB).  Each device the library runs on holds its own copy
// for the life of the process.  Host code never names the array except to
// ask for its device address: tg_ctx_create calls noalloc_setup with the
// context's device current, which resolves the address once per device
// with hipGetSymbolAddress and keeps it; kernels receive that address (as
// the sub-buffers carved from it), like a frame's workspace.
//
// Every call shares its device's array, so calls that overlap on one device
// race; a call leaves the array holding its own state.  What the kernels
// accumulate into or read before writing (the device counters and flags) is
// cleared at the start of every call by a one-lane kernel, not by a memset
// node (the sequence may be captured into a graph).
#include <mutex>

#include "../../include/tg.h"
#include "tg_internal.h"

namespace tg {
namespace {

constexpr int64_t NA_MAX_N = TG_NOALLOC_MAX_N;
constexpr int64_t NA_MAX_KEYS = TG_NOALLOC_MAX_KEYS;
constexpr int64_t NA_MAX_PIXELS = TG_NOALLOC_MAX_PIXELS;
constexpr int64_t NA_MAX_TILES = TG_NOALLOC_MAX_TILES;

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Sub-buffer offsets inside the array (bytes, each 256-aligned).
struct Layout {
  size_t xy, conic_o, wq, ext, rect, depth;
  size_t tile_count, tile_start, tile_cursor, tile_order;
  size_t keys, keys_tmp, sorted, qlist, qcount, qcut;
  size_t T_final, last, dev, total;
};

constexpr Layout make_layout() {
  Layout l{};
  size_t o = 0;
  l.xy = o;          o += align256(NA_MAX_N * sizeof(double2));
  l.conic_o = o;     o += align256(NA_MAX_N * sizeof(float4));
  l.wq = o;          o += align256(NA_MAX_N * sizeof(float4));
  l.ext = o;         o += align256(NA_MAX_N * sizeof(float4));
  l.rect = o;        o += align256(NA_MAX_N * sizeof(uint2));
  l.depth = o;       o += align256(NA_MAX_N * sizeof(uint32_t));
  l.tile_count = o;  o += align256(NA_MAX_TILES * sizeof(int32_t));
  l.tile_start = o;  o += align256((NA_MAX_TILES + 1) * sizeof(int32_t));
  l.tile_cursor = o; o += align256(NA_MAX_TILES * sizeof(int32_t));
  l.tile_order = o;  o += align256(NA_MAX_TILES * sizeof(int32_t));
  l.keys = o;        o += align256(NA_MAX_KEYS * sizeof(uint64_t));
  l.keys_tmp = o;    o += align256(NA_MAX_KEYS * sizeof(uint64_t));
  l.sorted = o;      o += align256(NA_MAX_KEYS * sizeof(int32_t));
  l.qlist = o;       o += align256(4 * NA_MAX_KEYS * sizeof(int2));
  l.qcount = o;      o += align256(4 * NA_MAX_TILES * sizeof(int32_t));
  l.qcut = o;        o += align256(4 * NA_MAX_TILES * sizeof(int32_t));
  l.T_final = o;     o += align256(NA_MAX_PIXELS * sizeof(float));
  l.last = o;        o += align256(NA_MAX_PIXELS * sizeof(int32_t));
  l.dev = o;         o += align256(sizeof(FrameDev));
  l.total = o;
  return l;
}

constexpr Layout LAYOUT = make_layout();
static_assert(LAYOUT.total == TG_NOALLOC_SCRATCH_BYTES, "the header states the array's size");
static_assert(NA_MAX_N <= MAX_GAUSS_SPACE, "Gaussian indices fit the binning's keys");

// The workspace.  In host code this name is only a handle for
// hipGetSymbolAddress; its device address is looked up per device.
static __device__ __align__(256) unsigned char scratch[LAYOUT.total];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};    // device address of `scratch` on each device

// Clear the device counters and flags of the workspace.
__global__ void k_noalloc_reset(FrameDev* d) {
  *d = FrameDev{};
}

// The outcome of the binning for the caller: TG_ERR_CAPACITY when the keys
// did not fit (the later kernels skipped the frame), else TG_OK.
__global__ void k_noalloc_status(const FrameDev* d, int32_t* status) {
  *status = d->overflow ? (int32_t)TG_ERR_CAPACITY : (int32_t)TG_OK;
}

template <class T>
T* at(unsigned char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

}  // namespace

// Resolve the array's address on `device`, which must be current.  Called
// by tg_ctx_create; the first call per device does the lookup.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_scratch[device];
}

}  // namespace tg

namespace tg {
int ctx_device(const tg_ctx* c);
}

extern "C" tg_status tg_render_noalloc(tg_ctx* ctx, const tg_gaussians* g, const tg_camera* cam,
                                       const float* bg, float* out_feat, float* out_alpha,
                                       int32_t* status, void* stream) {
  using namespace tg;
  if (!ctx || !g || !cam || !out_feat) return TG_ERR_INVALID;
  if (g->n < 0 || (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->feat)))
    return TG_ERR_INVALID;
  if (!(g->c == 8 || g->c == 16 || g->c == 32 || g->c == 64)) return TG_ERR_UNSUPPORTED;
  if (cam->width <= 0 || cam->height <= 0 || cam->width > 65535 * TILE || cam->height > 65535 * TILE)
    return TG_ERR_INVALID;
  const int64_t tiles_x = (cam->width + TILE - 1) / TILE, tiles_y = (cam->height + TILE - 1) / TILE;
  // sizes beyond the array's capacity are refused before anything is enqueued
  if (padded(g->n) > NA_MAX_N || (int64_t)cam->width * cam->height > NA_MAX_PIXELS ||
      tiles_x * tiles_y > NA_MAX_TILES)
    return TG_ERR_CAPACITY;
  const int device = ctx_device(ctx);
  unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(device));
  if (!base) return TG_ERR_HIP;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return TG_ERR_HIP;
  if (prev != device && hipSetDevice(device) != hipSuccess) return TG_ERR_HIP;

  CamArgs c;
  for (int i = 0; i < 9; ++i) c.R[i] = cam->R[i];
  for (int i = 0; i < 3; ++i) c.t[i] = cam->t[i];
  c.fx = cam->fx; c.fy = cam->fy; c.cx = cam->cx; c.cy = cam->cy; c.znear = cam->znear;
  c.W = cam->width; c.H = cam->height;
  c.tiles_x = (int32_t)tiles_x;
  c.tiles_y = (int32_t)tiles_y;

  BatchArgs a{};
  a.table = nullptr;
  a.hdr_dev = nullptr;
  ReqDev& q = a.one;
  q.mean = g->mean; q.scale = g->scale; q.quat = g->quat; q.opacity = g->opacity; q.feat = g->feat;
  q.bg = bg;
  q.out_feat = out_feat;
  q.out_alpha = out_alpha;
  q.T_final = at<float>(base, LAYOUT.T_final);
  q.last = at<int32_t>(base, LAYOUT.last);
  q.n = g->n;
  q.g_off = 0;
  q.tile_off = 0;
  q.cam = c;
  a.hdr.n_req = 1;
  a.hdr.n_tiles = (int32_t)(tiles_x * tiles_y);
  a.hdr.g_end = padded(g->n);
  a.xy = at<double2>(base, LAYOUT.xy);
  a.conic_o = at<float4>(base, LAYOUT.conic_o);
  a.wq = at<float4>(base, LAYOUT.wq);
  a.ext = at<float4>(base, LAYOUT.ext);
  a.rect = at<uint2>(base, LAYOUT.rect);
  a.depth = at<uint32_t>(base, LAYOUT.depth);
  a.tile_count = at<int32_t>(base, LAYOUT.tile_count);
  a.tile_start = at<int32_t>(base, LAYOUT.tile_start);
  a.tile_cursor = at<int32_t>(base, LAYOUT.tile_cursor);
  a.tile_order = at<int32_t>(base, LAYOUT.tile_order);
  a.keys = at<uint64_t>(base, LAYOUT.keys);
  a.keys_tmp = at<uint64_t>(base, LAYOUT.keys_tmp);
  a.sorted = at<int32_t>(base, LAYOUT.sorted);
  a.qlist = at<int2>(base, LAYOUT.qlist);
  a.qcount = at<int32_t>(base, LAYOUT.qcount);
  a.qcut = at<int32_t>(base, LAYOUT.qcut);
  a.g2d = nullptr;                       // forward only: no adjoint accumulators
  a.g_cap = NA_MAX_N;
  a.key_cap = NA_MAX_KEYS;
  a.dev = at<FrameDev>(base, LAYOUT.dev);

  hipStream_t s = static_cast<hipStream_t>(stream);
  tg_status st = TG_OK;
  hipLaunchKernelGGL(k_noalloc_reset, dim3(1), dim3(1), 0, s, a.dev);
  if (hipGetLastError() != hipSuccess) st = TG_ERR_HIP;
  if (st == TG_OK && launch_project(a, padded(g->n), s) != hipSuccess) st = TG_ERR_HIP;
  if (st == TG_OK && launch_bin_sort(a, padded(g->n), a.hdr.n_tiles, a.hdr.n_tiles, s) != hipSuccess)
    st = TG_ERR_HIP;
  if (st == TG_OK && launch_render_fwd(a, g->c, a.hdr.n_tiles, s) != hipSuccess) st = TG_ERR_HIP;
  if (st == TG_OK && status) {
    hipLaunchKernelGGL(k_noalloc_status, dim3(1), dim3(1), 0, s, (const FrameDev*)a.dev, status);
    if (hipGetLastError() != hipSuccess) st = TG_ERR_HIP;
  }
  if (prev != device) (void)hipSetDevice(prev);
  return st;
}
