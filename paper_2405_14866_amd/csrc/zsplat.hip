// zsplat.hip -- z-buffer point splat of the cascaded disparity
// initialisation (gfx950).
//
// §4.1 estimates disparity in cascade: the point cloud lifted from cam0's
// depth is rasterized into the viewpoints of cam2 and cam3, the z-buffers
// are extracted and converted to disparity maps (Eq. 2-3: they initialise
// the stereo matching of the other pairs).  The paper gives no splat size;
// the reading here is a one-pixel splat: a point lands in the pixel
// (floor(u), floor(v)) that contains its projection and keeps the nearest
// view depth there.  Points with view depth <= znear, or whose pixel lies
// outside the image, land nowhere.
//
// The landing pixel and the depth are discrete decisions, so they come from
// a fixed float32 operation sequence (the same as the rasterizer's binning
// spec for the view transform and the projection; the file is built with
// -ffp-contract=off and gfx950's float division is correctly rounded):
//   t_k = ((R_k0 x + R_k1 y) + R_k2 z) + t_k,  u = (fx t_x) / t_z + cx,
//   v = (fy t_y) / t_z + cy,  pixel = (floor(u), floor(v)).
// The nearest depth is an atomic minimum on the float32 bit pattern: the
// depths are positive (t_z > znear >= 0), and positive IEEE floats order
// like their bit patterns as unsigned integers, so the result does not
// depend on the order in which points arrive.  disparity = fx B / z in FP64,
// rounded to float32; 0 where no point landed.
//
// One launch projects every point into every target view (up to
// TG_ZSPLAT_MAX_VIEWS; a point's 12 bytes are read once).  HBM traffic:
// 12 B per point, 4 B per (point, view) atomic, 4 B per pixel to clear the
// z-buffer, 8 B per pixel for the disparity.
#include "../../include/tg.h"
#include "tg_internal.h"

namespace tg {
namespace {

struct ZView {
  float R[9], t[3];
  float fx, fy, cx, cy, znear, baseline;
  int32_t W, H;
  int64_t off;          // first pixel of this view's planes
};

struct ZArgs {
  ZView v[TG_ZSPLAT_MAX_VIEWS];
  int32_t n_views, pad;
  int64_t n, total_pixels;
  const float* mean;    // [3][n]
  uint32_t* zbuf;       // float32 bits, [total_pixels]
  float* disp;          // [total_pixels] or null
};

constexpr uint32_t INF_BITS = 0x7f800000u;

__global__ void __launch_bounds__(256) k_zsplat_clear(ZArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < a.total_pixels; p += (int64_t)gridDim.x * 256)
    a.zbuf[p] = INF_BITS;
}

__global__ void __launch_bounds__(256) k_zsplat(ZArgs a) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  const float x = a.mean[k], y = a.mean[a.n + k], z = a.mean[2 * a.n + k];
#pragma unroll
  for (int q = 0; q < TG_ZSPLAT_MAX_VIEWS; ++q) {
    if (q >= a.n_views) break;
    const ZView& c = a.v[q];
    const float tx = ((c.R[0] * x + c.R[1] * y) + c.R[2] * z) + c.t[0];
    const float ty = ((c.R[3] * x + c.R[4] * y) + c.R[5] * z) + c.t[1];
    const float tz = ((c.R[6] * x + c.R[7] * y) + c.R[8] * z) + c.t[2];
    if (!(tz > c.znear)) continue;
    const float u = (c.fx * tx) / tz + c.cx;
    const float v = (c.fy * ty) / tz + c.cy;
    const float fi = floorf(u), fj = floorf(v);
    if (!(fi >= 0.0f && fi < (float)c.W && fj >= 0.0f && fj < (float)c.H)) continue;
    const int64_t p = c.off + (int64_t)fj * c.W + (int64_t)fi;
    atomicMin(&a.zbuf[p], __float_as_uint(tz));
  }
}

__global__ void __launch_bounds__(256) k_zsplat_disp(ZArgs a) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < a.total_pixels; p += (int64_t)gridDim.x * 256) {
    int q = 0;
#pragma unroll
    for (int r = 1; r < TG_ZSPLAT_MAX_VIEWS; ++r)
      if (r < a.n_views && p >= a.v[r].off) q = r;
    const uint32_t b = a.zbuf[p];
    const double fb = (double)a.v[q].fx * (double)a.v[q].baseline;
    a.disp[p] = b == INF_BITS ? 0.0f : (float)(fb / (double)__uint_as_float(b));
  }
}

}  // namespace

int ctx_device(const tg_ctx* c);

}  // namespace tg

extern "C" tg_status tg_zsplat(tg_ctx* ctx, const float* mean, int64_t n, const tg_camera* cams,
                               const float* baselines, int32_t n_views, float* zbuf, float* disparity,
                               void* stream) {
  if (!ctx || !cams || !zbuf || n < 0 || n > ((int64_t)1 << 38) || (n > 0 && !mean) || n_views < 1 || n_views > TG_ZSPLAT_MAX_VIEWS)
    return TG_ERR_INVALID;
  if (disparity && !baselines) return TG_ERR_INVALID;
  tg::ZArgs a{};
  int64_t off = 0;
  for (int q = 0; q < n_views; ++q) {
    const tg_camera& c = cams[q];
    if (c.width <= 0 || c.height <= 0 || !(c.znear >= 0.0f)) return TG_ERR_INVALID;
    tg::ZView& v = a.v[q];
    for (int e = 0; e < 9; ++e) v.R[e] = c.R[e];
    for (int e = 0; e < 3; ++e) v.t[e] = c.t[e];
    v.fx = c.fx; v.fy = c.fy; v.cx = c.cx; v.cy = c.cy; v.znear = c.znear;
    v.baseline = baselines ? baselines[q] : 0.0f;
    v.W = c.width;
    v.H = c.height;
    v.off = off;
    off += (int64_t)c.width * c.height;
  }
  a.n_views = n_views;
  a.n = n;
  a.total_pixels = off;
  a.mean = mean;
  a.zbuf = reinterpret_cast<uint32_t*>(zbuf);
  a.disp = disparity;
  int prev = -1;
  const int dev = tg::ctx_device(ctx);
  const bool switched = hipGetDevice(&prev) == hipSuccess && prev != dev && hipSetDevice(dev) == hipSuccess;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t pb = (off + 255) / 256;
  const int pgrid = (int)(pb < 8192 ? pb : 8192);
  tg_status st = TG_OK;
  hipLaunchKernelGGL(tg::k_zsplat_clear, dim3(pgrid), dim3(256), 0, s, a);
  if (hipGetLastError() != hipSuccess) st = TG_ERR_HIP;
  if (st == TG_OK && n > 0) {
    hipLaunchKernelGGL(tg::k_zsplat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) st = TG_ERR_HIP;
  }
  if (st == TG_OK && disparity) {
    hipLaunchKernelGGL(tg::k_zsplat_disp, dim3(pgrid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) st = TG_ERR_HIP;
  }
  if (switched) (void)hipSetDevice(prev);
  return st;
}
