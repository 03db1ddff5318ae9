// blend_common.h -- per-(tile, Gaussian) state shared by the forward blend
// and its adjoint (gfx950).  Both kernels stage a Gaussian with make_state
// and evaluate its exponent with exponent(), so the adjoint re-takes every
// skip / blend decision of the forward bit for bit.
#pragma once

#include "tg_internal.h"

namespace tg {

constexpr float LOG2E = 1.4426950408889634f;
constexpr float CULL_MARGIN = 0.0625f;   // px added to the alpha-support box

typedef float f4v __attribute__((ext_vector_type(4)));

// 2D state of one staged Gaussian, from the projection: st = (u, v) relative
// to the tile origin (converted from the FP64 projection), opacity, exponent
// threshold thr = -log2(255 o); cq = conic scaled by -log2(e)/2 (so that
// exp2 of the exponent is the Gaussian) and, as bits, the 4-bit mask of the
// 8x8 quadrants its alpha >= 1/255 ellipse can reach (bounding box widened
// by CULL_MARGIN, so no pixel that could pass the threshold is culled).
__device__ __forceinline__ void make_state(double2 xy, float4 co, double ox, double oy,
                                           float4& st, float4& cq) {
  const float u = (float)(xy.x - ox), v = (float)(xy.y - oy);
  const float o = co.w;
  float thr = INFINITY;
  uint32_t mask = 0;
  if (o * 255.f >= 1.f) {
    thr = -log2f(255.f * o);
    // alpha >= 1/255  <=>  d^T Q d <= rho = 2 ln(255 o); box of that ellipse
    const float rho = 2.f * logf(255.f * o);
    const float det = co.x * co.z - co.y * co.y;
    const float ex = sqrtf(fmaxf(rho * co.z / det, 0.f)) + CULL_MARGIN;
    const float ey = sqrtf(fmaxf(rho * co.x / det, 0.f)) + CULL_MARGIN;
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const float x0 = (float)((qd & 1) * 8) + 0.5f, y0 = (float)((qd >> 1) * 8) + 0.5f;
      const bool hit = (u + ex >= x0) && (u - ex <= x0 + 7.f) && (v + ey >= y0) && (v - ey <= y0 + 7.f);
      mask |= hit ? (1u << qd) : 0u;
    }
  }
  st = make_float4(u, v, o, thr);
  cq = make_float4(-0.5f * LOG2E * co.x, -LOG2E * co.y, -0.5f * LOG2E * co.z, __uint_as_float(mask));
}

// log2 of the Gaussian at tile-local pixel centre (fpx, fpy):
// -(A dx^2 + C dy^2)/2 - B dx dy in units of log2(e)
__device__ __forceinline__ float exponent(float4 st, float4 cq, float fpx, float fpy) {
  const float dx = fpx - st.x, dy = fpy - st.y;
  return __builtin_fmaf(dx, __builtin_fmaf(cq.x, dx, cq.y * dy), cq.z * dy * dy);
}

// thr <= P <= 0 as one median (thr is finite for every Gaussian a quadrant walks)
__device__ __forceinline__ bool passes(float P, float thr) {
  return __builtin_amdgcn_fmed3f(P, thr, 0.f) == P;
}

__device__ __forceinline__ float blend_alpha(float o, float P) {
  return fminf(0.99f, o * __builtin_amdgcn_exp2f(P));
}

}  // namespace tg
