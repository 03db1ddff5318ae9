// render_fwd.hip -- step 3 of the rasterizer: per-tile front-to-back blend
// of C-channel latent features (gfx950).
//
// Persistent workgroups of 256 lanes (4 wave64) take tiles of the batch's
// global tile space from a device work queue, longest tiles first; one
// pixel per lane, wave w owns the 8x8 quadrant (w & 1, w >> 1) of the tile.
// The tile's sorted Gaussian list is consumed in batches of B entries,
// double-buffered in LDS:
//   * while batch b is blended, batch b+1 is fetched by LDS DMA
//     (global_load_lds_dwordx4): its feature rows as 16-byte chunks over
//     the four waves, its FP64 mean, exponent factors and support extents
//     (one 16-byte load per entry each), straight into the other buffer
//     without passing through VGPRs; the list indices of batch b+2 come
//     into a register.  The two buffers are separate LDS objects and the
//     batch loop is unrolled by two, so the compiler can tell the DMA target
//     from the buffer being walked and the walk never waits for the DMA;
//     each wave waits for its own DMA before the barrier that ends the batch;
//   * the kernel asks for five waves per SIMD: latency, not issue, bounds
//     the walk, and the registers of five waves leave room to fetch both
//     entries' feature slices at the top of a walk iteration, so that their
//     LDS latency overlaps the exponents and decisions;
//   * per staged Gaussian the walk reads the projection's exponent factors
//     (s, s k, r, log2 o) and the tile-dependent offsets (c1, c2), formed in
//     FP64 from the FP64 mean relative to the tile origin (so pixel offsets
//     are accurate to ~1e-7 px); log2 of the opacity-weighted Gaussian at a
//     pixel is then log2 o - z1^2 - z2^2 with z1, z2 affine in the pixel
//     centre: five FMAs and one v_exp_f32 give o G.  make_state also forms a
//     4-bit mask of the quadrants its alpha >= 1/255 ellipse can reach
//     (bounding box widened by 1/16 px, so no pixel that could pass the
//     threshold is ever culled and the blend's decisions are those of the
//     plain walk);
//   * each wave ballots the quadrant bits of the batch and walks only the
//     Gaussians that reach its quadrant, in list order (s_ff1 over the
//     ballot mask), so Gaussians that only touch the other quadrants cost
//     it nothing; a wave whose pixels have all ended walks nothing more;
//   * the walk takes two reaching Gaussians per iteration: their alphas are
//     independent and overlap, then their decisions and feature
//     accumulations run in list order.  A pixel's threshold test is one
//     compare against its own minimum alpha (1/255 while it runs, 2 once it
//     has ended, so an ended pixel fails every later test); the state
//     updates of a blend and its feature accumulation sit behind a
//     wave-uniform branch, since many steps blend in few pixels;
//   * the feature accumulation of a step is the rank-1 update F += w f^T of
//     the wave's 64 pixels x C channels (w: each lane's blend weight, 0 where
//     it does not blend).  It runs on the matrix cores as C/4
//     v_mfma_f32_4x4x1_16b_f32: block b of lanes 4b..4b+3 (four consecutive
//     pixels of a row) takes the lanes' own weights as A, and instruction m
//     covers channels m + (C/4) q, q = lane & 3, so each lane's B operands
//     are one contiguous C/4-float slice of the feature row (C/16
//     ds_read_b128 per lane instead of C/4 full-row broadcasts).  This moves
//     the C FMAs per step off the VALU and cuts the LDS bytes of a step
//     four-fold; the background enters as one last update with weight T.
// Per pixel: alpha = min(0.99, o G); skip when alpha < 1/255; a Gaussian
// that would take T below 1e-4 ends the pixel without being blended.
#include "blend_common.h"

namespace tg {
namespace {

constexpr int RENDER_B = 64;             // Gaussians per staged batch
constexpr int PERSISTENT_WG = 256 * 8;   // persistent workgroups (>= resident capacity)


// this lane's C/4 contiguous features of a row (LDS), for the MFMA B
// operands; volatile LDS reads, so that they issue where they are written
// and are not sunk into the branches that consume them
template <int NM>
__device__ __forceinline__ void load_slice(const float* p, float (&fl)[NM]) {
  if constexpr (NM % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NM / 4; ++k) {
      const f4v v = ((const volatile __attribute__((address_space(3))) f4v*)p)[k];
      fl[4 * k] = v.x; fl[4 * k + 1] = v.y; fl[4 * k + 2] = v.z; fl[4 * k + 3] = v.w;
    }
  } else {
    const float2 v = *reinterpret_cast<const float2*>(p);
    fl[0] = v.x; fl[1] = v.y;
  }
}

struct WorkCount {
  uint32_t n_eval = 0, n_blend = 0, steps = 0, steps_pass = 0, steps_blend = 0;
};

typedef __attribute__((address_space(3))) void lds_void;

// LDS of one staged batch (one of two, each a separate __shared__ object so
// that the compiler can tell the DMA into one from the walk over the other)
template <int C, int B>
struct BatchLDS {
  float4 wq[B];                     // exponent factors, DMA target (walked as they are)
  double2 xy[B];                    // FP64 mean, DMA target
  float4 ext[B];                    // support half-extents, DMA target
  float4 st[B];                     // (c1, c2, quadrant mask bits, -) from make_state
  int32_t ix[B];                    // Gaussian indices
  __align__(16) float fe[B * C];    // feature rows, DMA target
};

// Issue the DMA of batch entries [0, nb) (indices in L.ix): feature rows
// as 16-byte chunks spread over the four waves; the mean by wave 0, the
// exponent factors by wave 1 and the extents by wave 2 (one 16-byte load
// per lane each).
template <int C, int B>
__device__ __forceinline__ void dma_batch(const BatchArgs& a, const float* __restrict__ feat, int64_t g_off,
                                          BatchLDS<C, B>& L, int nb, int w, int lane) {
  constexpr int CHUNKS = C / 4;
  constexpr int INSTR = B * CHUNKS / 64;     // wave-wide feature loads per batch
  constexpr int PER = (INSTR + 3) / 4;       // ... per wave
  // all index reads first: an LDS read after a DMA into the same object
  // would have to wait for the DMA
  const int g0 = L.ix[lane < nb ? lane : 0];
  int gi[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int q = (w + 4 * i) * 64 + lane;
    const int r = q / CHUNKS;
    gi[i] = L.ix[r < nb ? r : 0];
  }
  if (w == 0) __builtin_amdgcn_global_load_lds((const void*)(a.xy + g0), (lds_void*)L.xy, 16, 0, 0);
  if (w == 1) __builtin_amdgcn_global_load_lds((const void*)(a.wq + g0), (lds_void*)L.wq, 16, 0, 0);
  if (w == 2) __builtin_amdgcn_global_load_lds((const void*)(a.ext + g0), (lds_void*)L.ext, 16, 0, 0);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int k = w + 4 * i;
    if (k < INSTR) {
      const int p = ((k * 64 + lane) % CHUNKS);
      __builtin_amdgcn_global_load_lds((const void*)(feat + (int64_t)(gi[i] - g_off) * C + 4 * p),
                                       (lds_void*)(L.fe + k * 256), 16, 0, 0);
    }
  }
}

// tile-dependent state of entry t of a staged batch
template <int C, int B>
__device__ __forceinline__ void stage_state(BatchLDS<C, B>& L, int t, double ox, double oy) {
  const TileState ts = make_state(L.xy[t], L.wq[t], L.ext[t], ox, oy);
  L.st[t] = make_float4(ts.c1, ts.c2, __uint_as_float(ts.mask), 0.f);
}

// Blend one tile (tile-local coordinates tx, ty of request q).
template <int C, int B, bool COUNT>
__device__ __forceinline__ void render_tile(const BatchArgs& a, const ReqDev& q, int gtile, int tx,
                                            int ty, BatchLDS<C, B>& L0, BatchLDS<C, B>& L1, WorkCount& wc) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int W = q.cam.W, H = q.cam.H;
  const int lx = ((w & 1) << 3) | (lane & 7);
  const int ly = ((w >> 1) << 3) | (lane >> 3);
  const int px = tx * TILE + lx, py = ty * TILE + ly;
  const bool inside = px < W && py < H;
  const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;
  const double ox = (double)(tx * TILE), oy = (double)(ty * TILE);
  const int s = a.tile_start[gtile], e = a.tile_start[gtile + 1];
  const int len = e - s;
  const uint32_t qbit = 1u << w;
  const float* feat = q.feat;
  const int64_t g_off = q.s_off;      // the list holds indices of this 2D-state range

  constexpr int NM = C / 4;           // MFMA updates per blend step
  const int q4 = lane & 3;
  f4v acc[NM];                        // acc[m][r]: channel m + NM q4, pixel (lane & ~3) + r
#pragma unroll
  for (int m = 0; m < NM; ++m) acc[m] = f4v{0.f, 0.f, 0.f, 0.f};
  float T = 1.f;
  int last = -1;
  // smallest alpha the pixel still takes: 1/255 while it runs, 2 (above any
  // alpha) once it has ended or when it lies outside the image
  float amin = inside ? ALPHA_MIN : 2.f;
  int stop_pos = -1;                  // list position that ended the pixel (COUNT only)

  const int nbatch = (len + B - 1) / B;
  // prologue: indices of batches 0 and 1, batch 0 fetched and staged
  if (tid < B) {
    L0.ix[tid] = tid < len ? a.sorted[s + tid] : 0;
    L1.ix[tid] = B + tid < len ? a.sorted[s + B + tid] : 0;
  }
  __syncthreads();
  if (nbatch > 0) {
    dma_batch<C, B>(a, feat, g_off, L0, min(B, len), w, lane);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  if (tid < B && tid < len) stage_state<C, B>(L0, tid, ox, oy);
  __syncthreads();

  // One list entry (position pos) against this wave's pixels, given its
  // alpha and feature slice: the stop / blend decisions, then the state
  // updates and the feature accumulation behind a wave-uniform branch
  // (most steps blend in only some of the pixels).
  auto visit = [&](const float (&fl)[NM], int pos, float al, bool valid) {
    const bool ok = valid & (al >= amin);
    const float Tn = __builtin_fmaf(-al, T, T);
    const bool stop = ok & (Tn < 1e-4f);
    if (COUNT && __builtin_amdgcn_ballot_w64(ok) != 0) ++wc.steps_pass;
    amin = stop ? 2.f : amin;
    if (COUNT && stop) stop_pos = pos;
    const bool blend = ok & !stop;
    if (__builtin_amdgcn_ballot_w64(blend) != 0) {
      if (COUNT) ++wc.steps_blend;
      if (COUNT && blend) ++wc.n_blend;
      const float wgt = blend ? al * T : 0.f;
      T = blend ? Tn : T;
      last = blend ? pos : last;
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[m] = __builtin_amdgcn_mfma_f32_4x4x1f32(wgt, fl[m], acc[m], 0, 0, 0);
    }
  };

  auto step = [&](BatchLDS<C, B>& cur, BatchLDS<C, B>& nxt, int b) -> bool {
    const int b0 = b * B;
    const int nb = min(B, len - b0);
    const bool more = b + 1 < nbatch;
    const int nb1 = more ? min(B, len - b0 - B) : 0;
    // ---- batch b+1 on its way into LDS; indices of batch b+2 into a register
    if (more) dma_batch<C, B>(a, feat, g_off, nxt, nb1, w, lane);
    int pidx = 0;
    if (more && tid < B && b0 + 2 * B + tid < len) pidx = a.sorted[s + b0 + 2 * B + tid];
    // ---- blend batch b: walk the Gaussians that reach this wave's quadrant
    // (none once every pixel of the wave has ended)
    {
      const bool live = __builtin_amdgcn_ballot_w64(amin < 1.f) != 0;
      const bool reach = live && lane < nb && (__float_as_uint(cur.st[lane].z) & qbit) != 0;
      uint64_t mask = __builtin_amdgcn_ballot_w64(reach);
      // two reaching Gaussians per iteration: their alphas are independent
      // and overlap; the decisions and accumulations then run in list order
      while (mask) {
        const int j1 = (int)__builtin_ctzll(mask);
        mask &= mask - 1;
        const bool has2 = mask != 0;
        const int j2 = has2 ? (int)__builtin_ctzll(mask) : j1;
        if (has2) mask &= mask - 1;
        // feature slices of both entries first (see load_slice)
        float fl1[NM], fl2[NM];
        load_slice<NM>(cur.fe + j1 * C + NM * q4, fl1);
        load_slice<NM>(cur.fe + j2 * C + NM * q4, fl2);
        const float4 w1 = cur.wq[j1], w2 = cur.wq[j2];
        const float2 c1 = *reinterpret_cast<const float2*>(&cur.st[j1]);
        const float2 c2 = *reinterpret_cast<const float2*>(&cur.st[j2]);
        const float al1 = blend_alpha(exponent(w1, c1.x, c1.y, fpx, fpy));
        const float al2 = blend_alpha(exponent(w2, c2.x, c2.y, fpx, fpy));
        if (COUNT) wc.steps += has2 ? 2 : 1;
        visit(fl1, b0 + j1, al1, true);
        visit(fl2, b0 + j2, al2, has2);
      }
    }
    // ---- finish batch b+1: every wave's DMA complete, then its 2D state
    __builtin_amdgcn_s_waitcnt(0);
    const int alive = __syncthreads_count(amin < 1.f);
    if (more) {
      if (tid < nb1) stage_state<C, B>(nxt, tid, ox, oy);
      if (tid < B) cur.ix[tid] = pidx;
    }
    __syncthreads();
    return alive != 0;
  };
  for (int b = 0; b < nbatch; b += 2) {
    if (!step(L0, L1, b)) break;
    if (b + 1 >= nbatch) break;
    if (!step(L1, L0, b + 1)) break;
  }
  if (q.bg) {                         // F += T_final bg, as one more rank-1 update
    float bl[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) bl[m] = q.bg[m + NM * q4];
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m] = __builtin_amdgcn_mfma_f32_4x4x1f32(T, bl[m], acc[m], 0, 0, 0);
  }
  if (inside) {
    const size_t pix = (size_t)py * W + px;
    if (q.out_alpha) q.out_alpha[pix] = 1.f - T;
    q.T_final[pix] = T;
    q.last[pix] = last;
  }
  {
    // lane 4b + q4 holds channels m + NM q4 of the four pixels of block b,
    // which are consecutive in one row of the quadrant
    const size_t HW = (size_t)W * H;
    const int b4 = lane & ~3;
    const int px0 = tx * TILE + ((w & 1) << 3) + (b4 & 7);
    const int py0 = ty * TILE + ((w >> 1) << 3) + (b4 >> 3);
    if (py0 < H) {
      float* base = q.out_feat + (size_t)py0 * W + px0;
      if (px0 + 3 < W && (W & 3) == 0) {
#pragma unroll
        for (int m = 0; m < NM; ++m)
          *reinterpret_cast<float4*>(base + (size_t)(m + NM * q4) * HW) =
              make_float4(acc[m][0], acc[m][1], acc[m][2], acc[m][3]);
      } else {
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (px0 + r < W) base[(size_t)(m + NM * q4) * HW + r] = acc[m][r];
      }
    }
  }
  if (COUNT && inside) {
    // evaluated pairs of the plain walk: every list position up to the stop
    wc.n_eval += stop_pos >= 0 ? (uint32_t)(stop_pos + 1) : (uint32_t)len;
  }
  __syncthreads();                    // LDS buffers are reused by the next tile
}

// TABLE: the batch's requests come from the device table (a replayed
// serving batch) rather than inline (a single render); the two are separate
// instantiations so that each keeps its own launch statistics.
template <int C, int B, bool COUNT, bool TABLE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) k_render(BatchArgs a) {
  if (a.dev->overflow) return;
  if (!TABLE) a.table = nullptr;
  const BatchHdr h = batch_hdr(a);
  __shared__ BatchLDS<C, B> L0;
  __shared__ BatchLDS<C, B> L1;
  __shared__ int s_tile;
  const int tid = threadIdx.x;
  WorkCount wc;
  for (;;) {
    if (tid == 0) {                  // queue position -> tile, longest tiles first
      const int k = atomicAdd(&a.dev->tile_queue, 1);
      s_tile = k < h.n_tiles ? a.tile_order[k] : -1;
    }
    __syncthreads();
    const int t = s_tile;
    __syncthreads();
    if (t < 0) break;
    const int r = req_of_tile(a, h, t);
    if (r < 0) break;
    const ReqDev& q = batch_req(a, r);
    const int lt = t - q.tile_off;
    render_tile<C, B, COUNT>(a, q, t, lt % q.cam.tiles_x, lt / q.cam.tiles_x, L0, L1, wc);
  }
  if (COUNT) {
    __shared__ unsigned long long cnt[5];
    if (tid < 5) cnt[tid] = 0;
    __syncthreads();
    atomicAdd(&cnt[0], (unsigned long long)wc.n_eval);
    atomicAdd(&cnt[1], (unsigned long long)wc.n_blend);
    if ((tid & 63) == 0) {
      atomicAdd(&cnt[2], (unsigned long long)wc.steps);
      atomicAdd(&cnt[3], (unsigned long long)wc.steps_pass);
      atomicAdd(&cnt[4], (unsigned long long)wc.steps_blend);
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
  // the last workgroup out re-arms the queue for the next launch
  if (tid == 0 && atomicAdd(&a.dev->tile_done, 1) == (int)gridDim.x - 1) {
    atomicExch(&a.dev->tile_queue, 0);
    atomicExch(&a.dev->tile_done, 0);
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
hipError_t launch_c(const BatchArgs& a, int32_t grid_tiles, hipStream_t s, bool count) {
  const int grid = grid_tiles < PERSISTENT_WG ? (grid_tiles > 0 ? grid_tiles : 1) : PERSISTENT_WG;
  if (count) {                        // work counts: single renders only
    if (a.table) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(1), 0, s, a.dev);
    hipLaunchKernelGGL((k_render<C, RENDER_B, true, false>), dim3(grid), dim3(256), 0, s, a);
  } else {
    if (a.table) hipLaunchKernelGGL((k_render<C, RENDER_B, false, true>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_render<C, RENDER_B, false, false>), dim3(grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

__global__ void k_fill_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

}  // namespace

hipError_t launch_render_fwd(const BatchArgs& a, int c, int32_t grid_tiles, hipStream_t s,
                             bool count_work) {
  switch (c) {
    case 8: return launch_c<8>(a, grid_tiles, s, count_work);
    case 16: return launch_c<16>(a, grid_tiles, s, count_work);
    case 32: return launch_c<32>(a, grid_tiles, s, count_work);
    case 64: return launch_c<64>(a, grid_tiles, s, count_work);
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
