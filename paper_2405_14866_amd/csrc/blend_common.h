// blend_common.h -- per-(tile, Gaussian) state shared by the forward blend
// and its adjoint (gfx950).  Both kernels stage a Gaussian with make_state
// and evaluate its alpha with blend_alpha(exponent()), so the adjoint
// re-takes every skip / blend decision of the forward bit for bit.
#pragma once

#include "tg_internal.h"

namespace tg {

constexpr float CULL_MARGIN = 0.0625f;   // px added to the alpha-support box
constexpr float ALPHA_MIN = 1.f / 255.f;

typedef float f4v __attribute__((ext_vector_type(4)));

// Tile-dependent part of one staged Gaussian.  The projection stores the
// exponent factors wq = (s, s k, r, log2 o) of the Gaussian (see the
// projection kernel); relative to a tile origin the exponent of pixel
// centre p (tile-local) is
//   log2 o - z1^2 - z2^2,  z1 = s px + s k py + c1,  z2 = r py + c2,
// with c1 = -s (u + k v) and c2 = -r v for the tile-relative mean (u, v),
// formed here in FP64 from the FP64 mean.  mask: bit q set when the
// alpha >= 1/255 ellipse (half-extents ext.xy, widened by CULL_MARGIN so no
// pixel that could pass is culled) reaches the 8x8 quadrant q of the tile.
// The binning applies the same test when it splits each tile's sorted list
// into the four quadrant lists the forward blend walks.
struct TileState {
  float c1, c2;
  float u, v;                 // tile-relative mean (the adjoint's moments)
  uint32_t mask;
};

// Quadrants of the tile at (ox, oy) that the alpha >= 1/255 ellipse of a
// Gaussian (FP64 mean xy, half-extents ext.xy) can reach, from the
// tile-relative mean (u, v) rounded to float32.
__device__ __forceinline__ uint32_t quadrant_mask(float u, float v, float4 ext) {
  const float ex = ext.x + CULL_MARGIN, ey = ext.y + CULL_MARGIN;   // -inf: no support
  uint32_t mask = 0;
#pragma unroll
  for (int qd = 0; qd < 4; ++qd) {
    const float x0 = (float)((qd & 1) * 8) + 0.5f, y0 = (float)((qd >> 1) * 8) + 0.5f;
    const bool hit = (u + ex >= x0) && (u - ex <= x0 + 7.f) && (v + ey >= y0) && (v - ey <= y0 + 7.f);
    mask |= hit ? (1u << qd) : 0u;
  }
  return mask;
}

__device__ __forceinline__ uint32_t quadrant_mask(double2 xy, float4 ext, double ox, double oy) {
  return quadrant_mask((float)(xy.x - ox), (float)(xy.y - oy), ext);
}

__device__ __forceinline__ TileState make_state(double2 xy, float4 wq, float4 ext, double ox, double oy) {
  TileState t;
  const double du = xy.x - ox, dv = xy.y - oy;
  t.c1 = (float)(-((double)wq.x * du + (double)wq.y * dv));
  t.c2 = (float)(-(double)wq.z * dv);
  t.u = (float)du;
  t.v = (float)dv;
  t.mask = quadrant_mask(t.u, t.v, ext);
  return t;
}

// c1, c2 of make_state alone (the quadrant lists are already culled)
__device__ __forceinline__ float2 exponent_offsets(double2 xy, float4 wq, double ox, double oy) {
  const double du = xy.x - ox, dv = xy.y - oy;
  return make_float2((float)(-((double)wq.x * du + (double)wq.y * dv)), (float)(-(double)wq.z * dv));
}

// log2 of the opacity-weighted Gaussian at tile-local pixel centre
// (fpx, fpy): log2 o - z1^2 - z2^2.  The Gaussian factor is <= 1 by
// construction (both squares are subtracted), so the method's rule that a
// positive exponent is skipped never fires.
__device__ __forceinline__ float exponent(float4 wq, float c1, float c2, float fpx, float fpy) {
  const float z1 = __builtin_fmaf(wq.x, fpx, __builtin_fmaf(wq.y, fpy, c1));
  const float z2 = __builtin_fmaf(wq.z, fpy, c2);
  return __builtin_fmaf(-z1, z1, __builtin_fmaf(-z2, z2, wq.w));
}

// alpha = min(0.99, o G); the caller compares it with ALPHA_MIN
__device__ __forceinline__ float blend_alpha(float P) {
  return fminf(0.99f, __builtin_amdgcn_exp2f(P));
}

}  // namespace tg
