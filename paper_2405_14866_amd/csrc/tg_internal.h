// tg_internal.h -- device data layout and kernel launchers of libtg (gfx950).
//
// Every kernel works on a *batch* of render requests (a single render is a
// batch of one).  A batch is one virtual frame:
//   * a global Gaussian index space: request r owns indices
//     [g_off, g_off + n) with g_off a multiple of BIN_CHUNK, so a
//     workgroup that covers an aligned chunk of indices never straddles
//     two requests;
//   * a global tile space: request r owns tiles [tile_off, tile_off +
//     tiles_x * tiles_y) in row-major order of its own image.
// Workspace in HBM (structure of arrays, allocated once per frame / slot):
//   per Gaussian  xy      double2  projected mean (u, v) in pixels, FP64 so
//                                  that the render's pixel offsets are exact
//                 conic_o float4   (A, B, C, opacity); conic = Sigma'^-1
//                 wq      float4   exponent factors (s, s k, r, log2 o): the
//                                  exponent of the opacity-weighted Gaussian
//                                  is log2 o - (s (dx + k dy))^2 - (r dy)^2
//                 ext     float4   (ex, ey, opacity, 0): half-extents of the
//                                  alpha >= 1/255 ellipse (-inf: none)
//                 rect    uint2    tile rectangle, x0 | x1 << 16, y0 | y1 << 16
//                                  (empty: x0 > x1)
//                 depth   uint32   IEEE bits of the float32 view depth
//                 g2d     float    [cap][8] backward accumulators: the six 2D
//                                  gradients of a Gaussian (u, v, conic A, B, C,
//                                  opacity) in one 32-byte row
//   Views of one Gaussian set (extra_views / covered) are requests of their
//   own (own index range, tiles and pixel state) whose Gaussian loads in
//   the projection and its adjoint are shared.
//   A request may share the projection and sorted lists of an earlier
//   request of the same batch whose geometry and camera are byte-identical
//   (src > 0): it keeps its own index range (its adjoint accumulators live
//   there) and its own tiles (its outputs and work items), but reads the 2D
//   state of the source's range (s_off) and a copy of the source's lists.
//   per tile      count, start[n_tiles + 1], cursor       int32
//                 order   int32    tiles by descending key count (the sort,
//                                  blend and adjoint take the longest first)
//   per key       keys    uint64   (depth << 32) | (quadrant mask << 28) |
//                                  global index, grouped by tile
//                 keys_tmp uint64  scratch for segments too long for LDS
//                 sorted  int32    global index, per tile in (depth, index) order
//                 qlist   int2     (global index, position in the tile's list) of the
//                                  entries whose alpha support reaches each 8x8
//                                  quadrant, in list order: tile t with segment
//                                  [s, s + n) keeps quadrant q's list at
//                                  qlist[4 s + q n ...] (room for 4 keys per key),
//                                  its length at qcount[4 t + q]; the forward
//                                  blend writes at qcut[4 t + q] one past the
//                                  list index of the last entry some pixel of
//                                  the quadrant blended (0: none), where the
//                                  adjoint starts its backward walk
//   per pixel     T_final float32, last int32 (read by the backward pass),
//                 one slice per request
//   device state  FrameDev (overflow flag, key count, work counters)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tg {

constexpr int TILE = 16;
constexpr int BIN_LDS_MAX_TILES = 32768;  // per-tile counters kept in LDS (128 KB)
constexpr int BIN_CHUNK = 1024;           // Gaussians per binning workgroup (and index alignment)
constexpr int MAX_BATCH = 64;             // requests per batch
// Gaussian indices of a frame or batch (the padded index space) stay below
// this: the binning packs a 4-bit quadrant mask above the index in a key.
constexpr int64_t MAX_GAUSS_SPACE = (int64_t)1 << 28;

struct FrameDev {
  int32_t overflow;             // set when the binning needs more keys than the frame holds
  int32_t pad;
  int64_t n_keys;               // keys needed by the last binning
  unsigned long long geom_mismatch;  // bit r: request r shares a source whose geometry differs
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

// One render request of a batch.
struct ReqDev {
  const float* mean;     // [3][n]
  const float* scale;    // [3][n]
  const float* quat;     // [4][n]
  const float* opacity;  // [n]
  const float* feat;     // [n][c]
  const float* bg;       // [c] or null
  float* out_feat;       // [c][H][W]
  float* out_alpha;      // [H][W] or null
  float* T_final;        // [H][W] (workspace slice)
  int32_t* last;         // [H][W] (workspace slice)
  // backward
  const float* d_img;    // [c][H][W]
  const float* d_alpha;  // [H][W] or null
  float* d_mean;         // [3][n] or null
  float* d_log_scale;    // [3][n] or null
  float* d_quat;         // [4][n] or null
  float* d_logit;        // [n] or null
  float* d_feat;         // [n][c]
  int64_t n;
  int64_t g_off;         // first global Gaussian index (multiple of BIN_CHUNK)
  int64_t s_off;         // first global index of the 2D state it reads (g_off, or its source's)
  int32_t tile_off;      // first global tile
  int32_t src;           // 0, or 1 + the batch index of the request whose projection and lists it shares
  // Several target views of one Gaussian set (a stereo pair): the views are
  // consecutive requests with the same Gaussian pointers; the first one's
  // projection (and projection adjoint) workgroups read each Gaussian once
  // and serve all of them, the others are marked covered.
  int32_t extra_views;   // the next extra_views requests are further views of this one's Gaussians
  int32_t covered;       // 1: an earlier request projects this one (and chains its adjoint)
  CamArgs cam;
};

// Totals of a batch (device copy for replayed launches, inline otherwise).
struct BatchHdr {
  int32_t n_req;
  int32_t n_tiles;       // sum of the requests' tiles
  int64_t g_end;         // end of the padded global Gaussian index space
  int32_t n_shared;      // requests that share an earlier request's projection and lists
  int32_t pad;
};

// Kernel arguments shared by every step.  A single render passes its
// request inline (table == nullptr); a replayed batch reads the request
// table and the header from device memory.
struct BatchArgs {
  const ReqDev* table;
  const BatchHdr* hdr_dev;
  ReqDev one;
  BatchHdr hdr;
  // workspace
  double2* xy;
  float4* conic_o;
  float4* wq;
  float4* ext;
  uint2* rect;
  uint32_t* depth;
  int32_t* tile_count;
  int32_t* tile_start;
  int32_t* tile_cursor;
  int32_t* tile_order;
  uint64_t* keys;
  uint64_t* keys_tmp;
  int32_t* sorted;
  int2* qlist;           // [4 key_cap] quadrant lists
  int32_t* qcount;       // [4 tiles] quadrant list lengths
  int32_t* qcut;         // [4 tiles] end of the quadrant lists' blended part
  float* g2d;            // [g_cap][8]
  int64_t g_cap;         // capacity of the global Gaussian index space
  int64_t key_cap;
  FrameDev* dev;
};

__device__ __forceinline__ BatchHdr batch_hdr(const BatchArgs& a) {
  return a.table ? *a.hdr_dev : a.hdr;
}

__device__ __forceinline__ const ReqDev& batch_req(const BatchArgs& a, int r) {
  return a.table ? a.table[r] : a.one;
}

// request that owns global Gaussian index g of the padded space, or -1
__device__ __forceinline__ int req_of_gauss(const BatchArgs& a, const BatchHdr& h, int64_t g) {
  if (g >= h.g_end) return -1;
  if (!a.table) return 0;
  for (int r = h.n_req - 1; r >= 0; --r)
    if (g >= a.table[r].g_off) return r;
  return -1;
}

// request that owns global tile t, or -1
__device__ __forceinline__ int req_of_tile(const BatchArgs& a, const BatchHdr& h, int t) {
  if (t >= h.n_tiles) return -1;
  if (!a.table) return 0;
  for (int r = h.n_req - 1; r >= 0; --r)
    if (t >= a.table[r].tile_off) return r;
  return -1;
}

__host__ __device__ inline int64_t padded(int64_t n) {
  return (n + BIN_CHUNK - 1) / BIN_CHUNK * BIN_CHUNK;
}

// Launchers; they return hipSuccess or the launch error.  Grids are sized
// from grid_gauss (padded Gaussian capacity) and grid_tiles (tile
// capacity): exact for a single render, the slot capacity for a replayed
// batch (workgroups beyond the batch's totals return at once).
hipError_t launch_project(const BatchArgs& a, int64_t grid_gauss, hipStream_t s);
hipError_t launch_bin_sort(const BatchArgs& a, int64_t grid_gauss, int32_t grid_tiles,
                           int32_t max_tiles_per_req, hipStream_t s);
hipError_t launch_render_fwd(const BatchArgs& a, int c, int32_t grid_tiles, hipStream_t s,
                             bool count_work = false);
hipError_t launch_render_bwd(const BatchArgs& a, int c, int64_t grid_gauss, int32_t grid_tiles,
                             hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t bin_set_attributes();

}  // namespace tg
