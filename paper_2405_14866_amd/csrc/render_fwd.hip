// render_fwd.hip -- step 3 of the rasterizer: per-tile front-to-back blend
// of C-channel latent features (gfx950).
//
// One 256-lane workgroup (4 wave64) per 16x16 tile, one pixel per lane; wave
// w owns the 8x8 quadrant (w & 1, w >> 1) of the tile.  The tile's sorted
// Gaussian list is consumed in batches of B entries, double-buffered in LDS:
//   * while batch b is blended, batch b+1 is fetched: its feature rows go
//     straight from HBM into LDS with global_load_lds_dwordx4 (no VGPRs, no
//     wait until the end of the batch), its 2D state is loaded into
//     registers and written to LDS after the blend, and the list indices of
//     batch b+2 are loaded the same way;
//   * per staged Gaussian the state is two float4: (u, v) relative to the
//     tile origin (converted from the FP64 projection, so pixel offsets are
//     accurate to ~1e-7 px), opacity, the exponent threshold
//     log2(1/(255 o)); the conic pre-scaled by -log2(e)/2, and a 4-bit mask
//     of the quadrants its alpha >= 1/255 ellipse can reach (bounding box
//     widened by 1/16 px, so no pixel that could pass the threshold is ever
//     culled and the blend's decisions are those of the plain walk);
//   * each wave ballots the quadrant bits of the batch and walks only the
//     Gaussians that reach its quadrant, in list order (s_ff1 over the
//     ballot mask), so Gaussians that only touch the other quadrants cost
//     it nothing;
//   * the per-Gaussian body has a single wave-uniform branch for the
//     exponential and one for the C-channel FMAs; the rest are selects.
// Per pixel: P = -d^T conic d / 2; skip when P > 0 or when P is below the
// opacity threshold (alpha < 1/255); alpha = min(0.99, o e^P); a Gaussian
// that would take T below 1e-4 ends the pixel without being blended.
// Features accumulate in registers (C VGPRs per lane).
#include "tg_internal.h"

namespace tg {
namespace {

constexpr float LOG2E = 1.4426950408889634f;
constexpr float CULL_MARGIN = 0.0625f;   // px added to the alpha-support box

typedef __attribute__((address_space(3))) void lds_void;

// Gather feature rows [r0, r0 + B) of the list into LDS (row-major, C
// floats each) with one 16-byte LDS-DMA load per lane per instruction.
template <int C, int B>
__device__ __forceinline__ void dma_features(const float* __restrict__ feat, const int32_t* sidx,
                                             float* dst, int nb, int w, int lane) {
  constexpr int CHUNKS = C / 4;              // 16-byte chunks per row
  constexpr int INSTR = B * CHUNKS / 64;     // wave-wide loads per batch
#pragma unroll
  for (int k = w; k < INSTR; k += 4) {
    const int q = k * 64 + lane;
    const int r = q / CHUNKS, p = q % CHUNKS;
    const int g = sidx[r < nb ? r : 0];
    const float* src = feat + (size_t)g * C + 4 * p;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(dst + k * 256), 16, 0, 0);
  }
}

// 2D state of one staged Gaussian, from the projection of step 1.
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

template <int C, int B, bool COUNT>
__global__ void __launch_bounds__(256) k_render(RenderArgs a) {
  static_assert(B % 64 == 0 && (B * C / 4) % 64 == 0, "batch shape");
  if (a.dev->overflow) return;
  const int tile = blockIdx.x;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int lx = ((w & 1) << 3) | (lane & 7);
  const int ly = ((w >> 1) << 3) | (lane >> 3);
  const int px = tx * TILE + lx, py = ty * TILE + ly;
  const bool inside = px < a.W && py < a.H;
  const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;
  const double ox = (double)(tx * TILE), oy = (double)(ty * TILE);
  const int s = a.tile_start[tile], e = a.tile_start[tile + 1];
  const int len = e - s;
  const uint32_t qbit = 1u << w;

  __shared__ float4 st[2][B];
  __shared__ float4 cq[2][B];
  __shared__ int32_t sidx[2][B];
  __shared__ __align__(16) float fe[2][B * C];

  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.f;
  float T = 1.f;
  int last = -1;
  bool done = !inside;
  int stop_pos = -1;                  // list position that ended the pixel (COUNT only)
  uint32_t n_blend = 0, steps = 0, steps_pass = 0, steps_blend = 0;

  const int nbatch = (len + B - 1) / B;
  // prologue: indices of batches 0 and 1, then batch 0 staged
  if (tid < B) {
    sidx[0][tid] = tid < len ? a.sorted[s + tid] : 0;
    sidx[1][tid] = B + tid < len ? a.sorted[s + B + tid] : 0;
  }
  __syncthreads();
  if (nbatch > 0) {
    dma_features<C, B>(a.feat, sidx[0], fe[0], min(B, len), w, lane);
    if (tid < B && tid < len) {
      const int g = sidx[0][tid];
      float4 s0, s1;
      make_state(a.xy[g], a.conic_o[g], ox, oy, s0, s1);
      st[0][tid] = s0;
      cq[0][tid] = s1;
    }
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();

  for (int b = 0; b < nbatch; ++b) {
    const int cur = b & 1, nxt = cur ^ 1;
    const int b0 = b * B;
    const int nb = min(B, len - b0);
    // ---- prefetch batch b+1 (features by DMA, state and next indices into registers)
    const bool more = b + 1 < nbatch;
    const int nb1 = more ? min(B, len - b0 - B) : 0;
    double2 pxy = make_double2(0.0, 0.0);
    float4 pco = make_float4(0.f, 0.f, 0.f, 0.f);
    int pidx = 0;
    if (more) {
      dma_features<C, B>(a.feat, sidx[nxt], fe[nxt], nb1, w, lane);
      if (tid < nb1) {
        const int g = sidx[nxt][tid];
        pxy = a.xy[g];
        pco = a.conic_o[g];
      }
      if (tid < B && b0 + 2 * B + tid < len) pidx = a.sorted[s + b0 + 2 * B + tid];
    }
    // ---- blend batch b: walk the Gaussians that reach this wave's quadrant
    const float4* stc = st[cur];
    const float4* cqc = cq[cur];
    const float* fec = fe[cur];
    for (int m0 = 0; m0 < nb; m0 += 64) {
      const int jj = m0 + lane;
      const bool reach = jj < nb && (__float_as_uint(cqc[jj].w) & qbit) != 0;
      uint64_t mask = __ballot(reach);
      while (mask) {
        if (__ballot(!done) == 0) break;
        const int j = m0 + (int)__builtin_ctzll(mask);
        mask &= mask - 1;
        const float4 gs = stc[j];
        const float4 q = cqc[j];
        const float dx = fpx - gs.x, dy = fpy - gs.y;
        const float P = __builtin_fmaf(dx, __builtin_fmaf(q.x, dx, q.y * dy), q.z * dy * dy);
        const bool pass = !done && P <= 0.f && P >= gs.w;
        if (COUNT) ++steps;
        if (__ballot(pass) == 0) continue;
        if (COUNT) ++steps_pass;
        const float al = fminf(0.99f, gs.z * __builtin_amdgcn_exp2f(P));
        const bool ok = pass && al >= 1.f / 255.f;
        const float Tn = T * (1.f - al);
        const bool stop = ok && Tn < 1e-4f;
        const bool blend = ok && !stop;
        if (COUNT && stop) stop_pos = b0 + j;
        done = done || stop;
        const float wgt = blend ? al * T : 0.f;
        T = blend ? Tn : T;
        last = blend ? b0 + j : last;
        if (COUNT && blend) ++n_blend;
        if (__ballot(blend) != 0) {
          if (COUNT) ++steps_blend;
          const float* f = fec + j * C;
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] = __builtin_fmaf(wgt, f[c], acc[c]);
        }
      }
    }
    // ---- finish staging batch b+1
    if (more) {
      if (tid < nb1) {
        float4 s0, s1;
        make_state(pxy, pco, ox, oy, s0, s1);
        st[nxt][tid] = s0;
        cq[nxt][tid] = s1;
      }
      if (tid < B) sidx[cur][tid] = pidx;
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (__syncthreads_count(!done) == 0) break;
  }
  if (inside) {
    const size_t HW = (size_t)a.W * a.H;
    const size_t pix = (size_t)py * a.W + px;
#pragma unroll
    for (int c = 0; c < C; ++c) a.out_feat[c * HW + pix] = acc[c] + T * (a.bg ? a.bg[c] : 0.f);
    if (a.out_alpha) a.out_alpha[pix] = 1.f - T;
    a.T_final[pix] = T;
    a.last[pix] = last;
  }
  if (COUNT) {
    // evaluated pairs of the plain walk: every list position up to the stop
    const uint32_t n_eval = !inside ? 0u : (stop_pos >= 0 ? (uint32_t)(stop_pos + 1) : (uint32_t)len);
    __shared__ unsigned long long cnt[5];
    if (tid < 5) cnt[tid] = 0;
    __syncthreads();
    atomicAdd(&cnt[0], (unsigned long long)n_eval);
    atomicAdd(&cnt[1], (unsigned long long)n_blend);
    if (lane == 0) {
      atomicAdd(&cnt[2], (unsigned long long)steps);
      atomicAdd(&cnt[3], (unsigned long long)steps_pass);
      atomicAdd(&cnt[4], (unsigned long long)steps_blend);
    }
    __syncthreads();
    if (tid == 0) {
      atomicAdd(&a.dev->n_eval, cnt[0]);
      atomicAdd(&a.dev->n_blend, cnt[1]);
      atomicAdd(&a.dev->wave_steps, cnt[2]);
      atomicAdd(&a.dev->wave_pass, cnt[3]);
      atomicAdd(&a.dev->wave_blend, cnt[4]);
    }
  }
}

__global__ void k_zero_work(FrameDev* d) {
  d->n_eval = 0;
  d->n_blend = 0;
  d->wave_steps = 0;
  d->wave_pass = 0;
  d->wave_blend = 0;
}

template <int C>
hipError_t launch_c(const RenderArgs& a, hipStream_t s, bool count) {
  constexpr int B = 64;
  if (count) {
    hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(1), 0, s, a.dev);
    hipLaunchKernelGGL((k_render<C, B, true>), dim3(a.n_tiles), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_render<C, B, false>), dim3(a.n_tiles), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

__global__ void k_fill_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

}  // namespace

hipError_t launch_render_fwd(const RenderArgs& a, int c, hipStream_t s, bool count_work) {
  switch (c) {
    case 8: return launch_c<8>(a, s, count_work);
    case 16: return launch_c<16>(a, s, count_work);
    case 32: return launch_c<32>(a, s, count_work);
    case 64: return launch_c<64>(a, s, count_work);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_zero, dim3((int)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace tg
