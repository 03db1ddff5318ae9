// lift.hip -- the step upstream of the rasterizer: the foreground pixels of
// the source views become Gaussians, on the device (gfx950).
//
// §4.1 converts each source view's predicted disparity map to depth (for a
// rectified pair of baseline B, a disparity of d pixels is the depth
// z = f_x B / d); §4.2 unprojects the depth maps with the camera
// parameters, and every foreground pixel becomes one pixel-aligned Gaussian:
// its position is the world point on the ray through the pixel centre at
// depth z, its latent feature, scale and opacity are the encoder's
// per-pixel maps (the heads of Eq. 4), its rotation is the identity.  The
// output is the Gaussian set in the rasterizer's layout (include/tg.h),
// compacted in (view, row-major pixel) order.
//
// A pixel is lifted when its mask byte is non-zero and its disparity (or,
// when no disparity map is given, its depth) is positive; a NaN is not.
//
// Stream compaction in three launches, one 256-lane workgroup per block of
// LIFT_BLOCK = 1024 pixels of one view (lane l of a workgroup takes pixels
// l, l + 256, l + 512, l + 768 of its block, so every load is a unit-stride
// wave access):
//   k_lift_count  the block's number of lifted pixels (wave ballots);
//   k_lift_scan   one workgroup: exclusive scan of the block counts, in
//                 place, so each block knows its first output row; the total
//                 is the Gaussian count n;
//   k_lift_write  the block again: each lifted pixel's rank inside the block
//                 (ballot prefix counts plus the per-wave totals in LDS), its
//                 world position in FP64, its scale, opacity and the identity
//                 quaternion as SoA columns of stride n, and the feature rows
//                 as one cooperative copy of 16-byte words (a lifted pixel's
//                 C features are one contiguous row of the channels-last map,
//                 and the block's output rows are one contiguous run).
// The position is evaluated in FP64 in a fixed operation order:
//   z = (f_x B) / d,   x_c = (((i + 0.5) - c_x) / f_x) z,
//   y_c = (((j + 0.5) - c_y) / f_y) z,   z_c = z,
//   x_w[a] = ((0 + R[0][a] (x_c - t_0)) + R[1][a] (y_c - t_1)) + R[2][a] (z_c - t_2)
// (R^T (x_c - t), the inverse of x_c = R x_w + t), each operation a
// correctly rounded IEEE double operation (no contraction), then rounded
// once to float32.
//
// HBM traffic: 5 B per pixel (mask + disparity) read by the count and again
// by the write, 16 + 4C B per lifted pixel read (scale, opacity, features),
// 44 + 4C B per Gaussian written.
#include <new>

#include "../../include/tg.h"
#include "tg_internal.h"

namespace tg {
namespace {

constexpr int LIFT_BLOCK = 1024;   // pixels per workgroup
constexpr int LIFT_LANES = 256;

struct LiftView {
  const float* zsrc;      // disparity [H][W] (disp = 1) or depth [H][W]
  const uint8_t* mask;    // [H][W]
  const float* feat;      // [H][W][c]
  const float* scale;     // [H][W][3]
  const float* opacity;   // [H][W]
  float R[9], t[3];
  float fx, fy, cx, cy, baseline;
  int32_t W, H, disp;
  int32_t blk0;           // first block of this view
  int64_t npix;
};

struct LiftArgs {
  LiftView v[TG_LIFT_MAX_VIEWS];
  int32_t n_views, c, n_blocks, pad;
  int32_t* blk;           // [n_blocks]: counts, then exclusive offsets
  int64_t* n_out;
  int64_t cap;
  float* mean;            // [3][n]
  float* scale;           // [3][n]
  float* quat;            // [4][n]
  float* opacity;         // [n]
  float* feat;            // [n][c]
};

// The workgroup's view (block b lies in view k when blk0[k] <= b < blk0[k + 1]).
__device__ __forceinline__ int view_of(const LiftArgs& a, int b) {
  int k = 0;
#pragma unroll
  for (int q = 1; q < TG_LIFT_MAX_VIEWS; ++q)
    if (q < a.n_views && b >= a.v[q].blk0) k = q;
  return k;
}

__device__ __forceinline__ bool lifted(const LiftView& V, int64_t p) {
  if (p >= V.npix) return false;
  const uint8_t m = V.mask[p];
  const float z = V.zsrc[p];
  return m != 0 && z > 0.0f;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ void __launch_bounds__(LIFT_LANES) k_lift_count(LiftArgs a) {
  __shared__ int32_t wsum[LIFT_LANES / 64];
  const int b = blockIdx.x;
  if (b >= a.n_blocks) return;
  const LiftView& V = a.v[view_of(a, b)];
  const int64_t p0 = (int64_t)(b - V.blk0) * LIFT_BLOCK;
  const int tid = threadIdx.x;
  bool f[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) f[k] = lifted(V, p0 + k * LIFT_LANES + tid);
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) cnt += __popcll(__ballot(f[k]));
  if ((tid & 63) == 0) wsum[tid >> 6] = cnt;
  __syncthreads();
  if (tid == 0) a.blk[b] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// One workgroup of 1024 lanes; lane l owns the blocks [l per, (l + 1) per).
__global__ void __launch_bounds__(1024) k_lift_scan(LiftArgs a) {
  __shared__ int64_t wsum[16];
  const int nb = a.n_blocks;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  int64_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += a.blk[b];
  int64_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int64_t run = incl - sum, total = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    run += q < wv ? wsum[q] : 0;
    total += wsum[q];
  }
  for (int b = b0; b < b1; ++b) {
    const int32_t c = a.blk[b];
    a.blk[b] = (int32_t)run;
    run += c;
  }
  if (tid == 0) *a.n_out = total;
}

__global__ void __launch_bounds__(LIFT_LANES) k_lift_write(LiftArgs a) {
  __shared__ int32_t rows[LIFT_BLOCK];          // block-local pixel of each output row
  __shared__ int32_t wcnt[4][LIFT_LANES / 64];  // lifted pixels per (quarter, wave)
  const int b = blockIdx.x;
  if (b >= a.n_blocks) return;
  const int64_t n = *a.n_out;
  if (n > a.cap) return;                        // too many for the buffers: nothing is written
  const LiftView& V = a.v[view_of(a, b)];
  const int64_t p0 = (int64_t)(b - V.blk0) * LIFT_BLOCK;
  const int tid = threadIdx.x, w = tid >> 6;
  bool f[4];
  uint64_t bal[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[k] = lifted(V, p0 + k * LIFT_LANES + tid);
    bal[k] = __ballot(f[k]);
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) wcnt[k][w] = __popcll(bal[k]);
  }
  __syncthreads();
  // row of pixel k * 256 + tid: everything lifted in earlier quarters, then
  // in earlier waves of this quarter, then in lower lanes of this wave
  int before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int qsum = 0, wbefore = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      qsum += wcnt[k][q];
      wbefore += q < w ? wcnt[k][q] : 0;
    }
    if (f[k]) rows[before + wbefore + __popcll(bal[k] & lanes_below())] = k * LIFT_LANES + tid;
    before += qsum;
  }
  total = before;
  __syncthreads();
  const int64_t off = a.blk[b];
  const double fx = V.fx, fy = V.fy, cx = V.cx, cy = V.cy, fb = (double)V.fx * (double)V.baseline;
  for (int r = tid; r < total; r += LIFT_LANES) {
    const int64_t p = p0 + rows[r];
    const int64_t i = p % V.W, j = p / V.W;
    const double d = V.zsrc[p];
    const double z = V.disp ? fb / d : d;
    const double xc[3] = {(((double)i + 0.5) - cx) / fx * z, (((double)j + 0.5) - cy) / fy * z, z};
    const int64_t o = off + r;
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) {
      double acc = 0.0;
#pragma unroll
      for (int e = 0; e < 3; ++e) acc = acc + (double)V.R[3 * e + c3] * (xc[e] - (double)V.t[e]);
      a.mean[c3 * n + o] = (float)acc;
      a.scale[c3 * n + o] = V.scale[3 * p + c3];
    }
    a.opacity[o] = V.opacity[p];
    a.quat[o] = 1.0f;
    a.quat[n + o] = 0.0f;
    a.quat[2 * n + o] = 0.0f;
    a.quat[3 * n + o] = 0.0f;
  }
  // feature rows: 16-byte words, q4 per row; four words in flight per lane
  const int q4 = a.c >> 2, sh = __ffs(q4) - 1;
  const int words = total * q4;
  const float4* src = reinterpret_cast<const float4*>(V.feat);
  float4* dst = reinterpret_cast<float4*>(a.feat) + off * q4;
  auto word = [&](int e) { return src[(p0 + rows[e >> sh]) * q4 + (e & (q4 - 1))]; };
  for (int e0 = tid; e0 < words; e0 += 4 * LIFT_LANES) {
    // indices past the end re-read the last word (in bounds) and store nothing
    const int e1 = min(e0 + LIFT_LANES, words - 1), e2 = min(e0 + 2 * LIFT_LANES, words - 1),
              e3 = min(e0 + 3 * LIFT_LANES, words - 1);
    const float4 v0 = word(e0), v1 = word(e1), v2 = word(e2), v3 = word(e3);
    dst[e0] = v0;
    if (e0 + LIFT_LANES < words) dst[e1] = v1;
    if (e0 + 2 * LIFT_LANES < words) dst[e2] = v2;
    if (e0 + 3 * LIFT_LANES < words) dst[e3] = v3;
  }
}

}  // namespace
}  // namespace tg

struct tg_lifter {
  int device = 0;
  int64_t max_pixels = 0;
  int32_t max_blocks = 0;
  int32_t* blk = nullptr;
};

namespace {

struct LiftDeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit LiftDeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~LiftDeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

namespace tg {
int ctx_device(const tg_ctx* c);
}

extern "C" {

tg_status tg_lifter_create(tg_ctx* ctx, int64_t max_pixels, tg_lifter** out) {
  if (!ctx || !out || max_pixels <= 0 || max_pixels > ((int64_t)1 << 34)) return TG_ERR_INVALID;
  *out = nullptr;
  const int dev = tg::ctx_device(ctx);
  LiftDeviceGuard guard(dev);
  tg_lifter* l = new (std::nothrow) tg_lifter;
  if (!l) return TG_ERR_OOM;
  l->device = dev;
  l->max_pixels = max_pixels;
  const int64_t blocks = max_pixels / tg::LIFT_BLOCK + TG_LIFT_MAX_VIEWS;
  if (blocks >= ((int64_t)1 << 31)) {
    delete l;
    return TG_ERR_INVALID;
  }
  l->max_blocks = (int32_t)blocks;
  if (hipMalloc(reinterpret_cast<void**>(&l->blk), (size_t)blocks * sizeof(int32_t)) != hipSuccess) {
    delete l;
    return TG_ERR_OOM;
  }
  *out = l;
  return TG_OK;
}

void tg_lifter_destroy(tg_lifter* l) {
  if (!l) return;
  LiftDeviceGuard guard(l->device);
  (void)hipDeviceSynchronize();
  if (l->blk) (void)hipFree(l->blk);
  delete l;
}

tg_status tg_lift(tg_lifter* l, const tg_source_view* views, int32_t n_views, int32_t c,
                  const tg_gaussian_buffers* out, int64_t* n_out, void* stream) {
  if (!l || !views || !out || !n_out || n_views < 1 || n_views > TG_LIFT_MAX_VIEWS) return TG_ERR_INVALID;
  if (!(c == 8 || c == 16 || c == 32 || c == 64)) return TG_ERR_UNSUPPORTED;
  if (out->cap < 0 || !out->mean || !out->scale || !out->quat || !out->opacity || !out->feat ||
      !aligned16(out->feat))
    return TG_ERR_INVALID;
  tg::LiftArgs a{};
  int64_t pixels = 0, blocks = 0;
  for (int k = 0; k < n_views; ++k) {
    const tg_source_view& s = views[k];
    const float* zsrc = s.disparity ? s.disparity : s.depth;
    if (!zsrc || !s.mask || !s.feat || !s.scale || !s.opacity || !aligned16(s.feat)) return TG_ERR_INVALID;
    if (s.cam.width <= 0 || s.cam.height <= 0) return TG_ERR_INVALID;
    if (s.disparity && !(s.baseline > 0.0f)) return TG_ERR_INVALID;
    const int64_t np = (int64_t)s.cam.width * s.cam.height;
    tg::LiftView& v = a.v[k];
    v.zsrc = zsrc;
    v.mask = s.mask;
    v.feat = s.feat;
    v.scale = s.scale;
    v.opacity = s.opacity;
    for (int e = 0; e < 9; ++e) v.R[e] = s.cam.R[e];
    for (int e = 0; e < 3; ++e) v.t[e] = s.cam.t[e];
    v.fx = s.cam.fx; v.fy = s.cam.fy; v.cx = s.cam.cx; v.cy = s.cam.cy;
    v.baseline = s.baseline;
    v.W = s.cam.width;
    v.H = s.cam.height;
    v.disp = s.disparity ? 1 : 0;
    v.blk0 = (int32_t)blocks;
    v.npix = np;
    pixels += np;
    blocks += (np + tg::LIFT_BLOCK - 1) / tg::LIFT_BLOCK;
  }
  if (pixels > l->max_pixels || blocks > l->max_blocks) return TG_ERR_CAPACITY;
  a.n_views = n_views;
  a.c = c;
  a.n_blocks = (int32_t)blocks;
  a.blk = l->blk;
  a.n_out = n_out;
  a.cap = out->cap;
  a.mean = out->mean;
  a.scale = out->scale;
  a.quat = out->quat;
  a.opacity = out->opacity;
  a.feat = out->feat;
  LiftDeviceGuard guard(l->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = (int)blocks;
  hipLaunchKernelGGL(tg::k_lift_count, dim3(grid), dim3(tg::LIFT_LANES), 0, s, a);
  if (hipGetLastError() != hipSuccess) return TG_ERR_HIP;
  hipLaunchKernelGGL(tg::k_lift_scan, dim3(1), dim3(1024), 0, s, a);
  if (hipGetLastError() != hipSuccess) return TG_ERR_HIP;
  hipLaunchKernelGGL(tg::k_lift_write, dim3(grid), dim3(tg::LIFT_LANES), 0, s, a);
  if (hipGetLastError() != hipSuccess) return TG_ERR_HIP;
  return TG_OK;
}

}  // extern "C"
