// tg_internal.h -- device data layout and kernel launchers of libtg (gfx950).
//
// Frame workspace in HBM (all structure-of-arrays, allocated once per frame):
//   per Gaussian  xy      double2  projected mean (u, v) in pixels, FP64 so
//                                  that the render's pixel offsets are exact
//                 conic_o float4   (A, B, C, opacity); conic = Sigma'^-1
//                 rect    uint2    tile rectangle, x0 | x1 << 16, y0 | y1 << 16
//                                  (empty: x0 > x1)
//                 depth   uint32   IEEE bits of the float32 view depth
//   per tile      count, start[n_tiles + 1], cursor       int32
//   per key       keys    uint64   (depth << 32) | index, grouped by tile
//                 keys_tmp uint64  scratch for segments too long for LDS
//                 sorted  int32    Gaussian index, per tile in (depth, index) order
//   per pixel     T_final float32, last int32 (read by the backward pass)
//   per Gaussian  grad2d  float    [8][n] accumulators of the backward pass
//   device state  FrameDev (overflow flag, key count)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tg {

constexpr int TILE = 16;
constexpr int SORT_LDS_CAP = 4096;     // keys sorted entirely in LDS per tile
constexpr int BIN_LDS_MAX_TILES = 32768;  // per-tile counters kept in LDS (128 KB)
constexpr int BIN_CHUNK = 1024;        // Gaussians per binning workgroup

struct FrameDev {
  int32_t overflow;             // set when the binning needs more keys than the frame holds
  int32_t pad;
  int64_t n_keys;               // keys needed by the last binning
  // work of the last counted render
  unsigned long long n_eval;        // (pixel, Gaussian) pairs the per-pixel walk visits
  unsigned long long n_blend;       // (pixel, Gaussian) pairs blended
  unsigned long long wave_steps;    // wave-level Gaussian steps after quadrant culling
  unsigned long long wave_pass;     // ... in which some lane passes the opacity threshold
  unsigned long long wave_blend;    // ... in which some lane blends
};

struct CamArgs {
  float R[9], t[3];
  float fx, fy, cx, cy, znear;
  int32_t W, H, tiles_x, tiles_y;
};

struct ProjectArgs {
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opacity;
  int64_t n;
  CamArgs cam;
  double2* xy;
  float4* conic_o;
  uint2* rect;
  uint32_t* depth;
  int32_t* tile_count;
  int32_t n_tiles;
};

struct BinArgs {
  const uint2* rect;
  const uint32_t* depth;
  int64_t n;
  int32_t tiles_x, n_tiles;
  int32_t* tile_count;
  int32_t* tile_start;
  int32_t* tile_cursor;
  uint64_t* keys;
  uint64_t* keys_tmp;
  int32_t* sorted;
  int64_t key_cap;
  FrameDev* dev;
};

struct RenderArgs {
  const double2* xy;
  const float4* conic_o;
  const float* feat;     // [n][c]
  const int32_t* tile_start;
  const int32_t* sorted;
  const float* bg;       // [c] or null
  float* out_feat;       // [c][H][W]
  float* out_alpha;      // [H][W]
  float* T_final;        // [H][W]
  int32_t* last;         // [H][W]
  int32_t W, H, tiles_x, n_tiles;
  FrameDev* dev;
};

struct BackwardArgs {
  // forward state
  const double2* xy;
  const float4* conic_o;
  const float* feat;
  const int32_t* tile_start;
  const int32_t* sorted;
  const float* bg;
  const float* T_final;
  const int32_t* last;
  // upstream
  const float* d_img;    // [c][H][W]
  const float* d_alpha;  // [H][W] or null
  // outputs: 2D-state gradients [6][n] (du, dv, dA, dB, dC, dopacity) and features [n][c]
  float* g2d;
  float* g_feat;
  int64_t n;
  int32_t W, H, tiles_x, n_tiles;
  const FrameDev* dev;
};

struct ProjectBwdArgs {
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opacity;
  int64_t n;
  CamArgs cam;
  const uint2* rect;
  const float* g2d;      // [6][n]
  float* d_mean;         // [3][n]
  float* d_log_scale;    // [3][n]
  float* d_quat;         // [4][n]
  float* d_logit;        // [n]
};

// launchers (return hipSuccess or the launch error)
hipError_t launch_project(const ProjectArgs& a, hipStream_t s);
hipError_t launch_bin_sort(const BinArgs& a, hipStream_t s);
hipError_t launch_render_fwd(const RenderArgs& a, int c, hipStream_t s, bool count_work = false);
hipError_t launch_render_bwd(const BackwardArgs& a, int c, hipStream_t s);
hipError_t launch_project_bwd(const ProjectBwdArgs& a, hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);

}  // namespace tg
