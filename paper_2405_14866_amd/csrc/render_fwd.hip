// render_fwd.hip -- step 3 of the rasterizer: per-tile front-to-back blend
// of C-channel latent features (gfx950).
//
// Work item = one 8x8 quadrant of a 16x16 tile, one wave64 per item, one
// pixel per lane.  The binning leaves, for every quadrant, the sub-list of
// its tile's sorted list whose alpha >= 1/255 support can reach the
// quadrant (a conservative bounding-box test widened by 1/16 px), in list
// order, as (Gaussian index, tile-list position); walking that sub-list
// gives exactly the pixels' walk over the whole tile list, because every
// entry left out is skipped by all 64 pixels.  The waves of a workgroup are
// independent: each takes its items from a fixed assignment over the tile
// order (tiles longest first; see k_render) and never waits for another
// wave, so a quadrant with a long list holds up nobody.
//   * the quadrant list is consumed in batches of B entries (B = 24 at
//     C = 32: two 3 KB feature buffers per wave, five 4-wave workgroups per
//     CU): while batch b is walked, batch b+1's feature rows arrive in the
//     wave's other LDS buffer and its FP64 means and exponent factors in the
//     wave's raw slots, all by LDS DMA (global_load_lds_dwordx4, C/4 lanes
//     per feature row), so no register is held for them across the walk;
//     the entries of batch b+2 load into a register.  After the walk the
//     wave waits for its own DMA, forms batch b+1's tile-dependent offsets
//     and stages them;
//   * the work item, and so the tile, its request and its lists, is
//     wave-uniform and kept in scalar registers;
//   * per staged Gaussian the walk reads the projection's exponent factors
//     (s, s k, r, log2 o) and the tile-dependent offsets (c1, c2), formed in
//     FP64 from the FP64 mean relative to the tile origin (so pixel offsets
//     are accurate to ~1e-7 px); log2 of the opacity-weighted Gaussian at a
//     pixel is then log2 o - z1^2 - z2^2 with z1, z2 affine in the pixel
//     centre: five FMAs and one v_exp_f32 give o G;
//   * the walk takes two entries per iteration, read at fixed LDS offsets
//     (the second slot is always inside the batch buffers; past the batch's
//     end it is masked): their alphas are independent and overlap, then
//     their decisions and feature accumulations run in list order.  A pixel's threshold test is one
//     compare against its own minimum alpha (1/255 while it runs, 2 once it
//     has ended, so an ended pixel fails every later test); the state
//     updates of a blend and its feature accumulation sit behind a
//     wave-uniform branch, since many steps blend in few pixels; a wave whose
//     pixels have all ended stops;
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
// that would take T below 1e-4 ends the pixel without being blended.  The
// last blended Gaussian's position in the tile's list is kept for the
// adjoint.
#include "blend_common.h"

namespace tg {
namespace {



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

// One wave's LDS: the feature rows of two batches (the one being walked
// and the next, arriving by LDS DMA) and the staged state of the batch being
// walked.  Four waves of a workgroup hold four of these and share nothing.
template <int C, int B>
struct WaveLDS {
  __align__(16) float fe[2][B * C];  // feature rows, DMA targets
  float4 wq[B];                      // exponent factors
  float4 st[B];                      // (c1, c2, tile-list position as bits, -)
  double2 rxy[B];                    // next batch's FP64 means, DMA target
  float4 rwq[B];                     // next batch's exponent factors, DMA target
};

// Entries per batch: two feature buffers of 3 KB (C >= 16), so that five
// workgroups of four waves fit a CU's LDS.
template <int C>
constexpr int wave_batch() { return C >= 64 ? 12 : (C == 32 ? 24 : (C == 16 ? 48 : 64)); }

// Issue the LDS DMA of the feature rows of a batch (entries [0, nb); lane j
// holds entry j's global index gi) into buffer dst: 16-byte chunks, C / 4
// lanes per row, 64 / (C / 4) rows per instruction.  Rows past nb read row
// 0's address (in bounds) and are never walked.
template <int C, int B>
__device__ __forceinline__ void dma_rows(const float* __restrict__ feat, int64_t g_off, float* dst, int gi, int nb,
                                         int lane) {
  constexpr int LPR = C / 4;
  constexpr int RPI = 64 / LPR;
  static_assert(B % RPI == 0, "a batch is a whole number of DMA instructions");
#pragma unroll
  for (int k = 0; k < B / RPI; ++k) {
    const int row = k * RPI + lane / LPR;
    const int g = __shfl(gi, row < nb ? row : 0, 64);
    if (k * RPI < nb)
      __builtin_amdgcn_global_load_lds((const void*)(feat + (g - g_off) * C + 4 * (lane % LPR)),
                                       (lds_void*)(dst + k * 256), 16, 0, 0);
  }
}

// Blend the 8x8 quadrant qd of one tile (tile-local coordinates tx, ty of
// request q) with one wave, walking the quadrant's list.
template <int C, int B, bool COUNT>
__device__ __forceinline__ void render_quadrant(const BatchArgs& a, const ReqDev& q, int gtile, int tx, int ty,
                                                int qd, WaveLDS<C, B>& L, WorkCount& wc) {
  const int lane = threadIdx.x & 63;
  const int W = q.cam.W, H = q.cam.H;
  const int lx = ((qd & 1) << 3) | (lane & 7);
  const int ly = ((qd >> 1) << 3) | (lane >> 3);
  const int px = tx * TILE + lx, py = ty * TILE + ly;
  const bool inside = px < W && py < H;
  const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;
  const double ox = (double)(tx * TILE), oy = (double)(ty * TILE);
  const int s = a.tile_start[gtile], len = a.tile_start[gtile + 1] - s;
  const int qn = a.qcount[4 * gtile + qd];
  const int2* ql = a.qlist + 4 * (int64_t)s + (int64_t)qd * len;
  const float* feat = q.feat;
  const int64_t g_off = q.s_off;      // the lists hold indices of this 2D-state range

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

  // One list entry (tile-list position pos) against this wave's pixels,
  // given its alpha and feature slice: the stop / blend decisions, then the
  // state updates and the feature accumulation behind a wave-uniform branch.
  int qlast = -1;                     // quadrant-list index of the last entry some pixel blended
  auto visit = [&](const float (&fl)[NM], int pos, int k, float al, bool valid) {
    const bool ok = valid & (al >= amin);
    const float Tn = __builtin_fmaf(-al, T, T);
    const bool stop = ok & (Tn < 1e-4f);
    if (COUNT && __builtin_amdgcn_ballot_w64(ok) != 0) ++wc.steps_pass;
    amin = stop ? 2.f : amin;
    if (COUNT && stop) stop_pos = pos;
    const bool blend = ok & !stop;
    if (__builtin_amdgcn_ballot_w64(blend) != 0) {
      qlast = k;
      if (COUNT) ++wc.steps_blend;
      if (COUNT && blend) ++wc.n_blend;
      const float wgt = blend ? al * T : 0.f;
      T = blend ? Tn : T;
      last = blend ? pos : last;
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[m] = __builtin_amdgcn_mfma_f32_4x4x1f32(wgt, fl[m], acc[m], 0, 0, 0);
    }
  };

  const int nbatch = (qn + B - 1) / B;
  // prologue: batch 0's rows on their way, its state staged; batch 1's entries in a register
  int2 e = lane < B && lane < qn ? ql[lane] : make_int2(0, 0);
  int2 en = lane < B && B + lane < qn ? ql[B + lane] : make_int2(0, 0);
  if (nbatch > 0) {
    dma_rows<C, B>(feat, g_off, L.fe[0], e.x, min(B, qn), lane);
    if (lane < B && lane < qn) {
      const double2 xy = a.xy[e.x];
      const float4 wq = a.wq[e.x];
      const float2 cc = exponent_offsets(xy, wq, ox, oy);
      L.wq[lane] = wq;
      L.st[lane] = make_float4(cc.x, cc.y, __int_as_float(e.y), 0.f);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  for (int b = 0; b < nbatch; ++b) {
    const int b0 = b * B;
    const int nb = min(B, qn - b0);
    const bool more = b + 1 < nbatch;
    const int nb1 = more ? min(B, qn - b0 - B) : 0;
    float* cur = L.fe[b & 1];
    // ---- batch b+1: its rows into the other buffer and its FP64 means and
    // exponent factors into the wave's raw slots, all by LDS DMA (nothing
    // held in registers across the walk); the entries of batch b+2 into a
    // register
    int2 en2 = make_int2(0, 0);
    if (more) {
      dma_rows<C, B>(feat, g_off, L.fe[(b + 1) & 1], en.x, nb1, lane);
      if (lane < nb1) {
        __builtin_amdgcn_global_load_lds((const void*)(a.xy + en.x), (lds_void*)L.rxy, 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void*)(a.wq + en.x), (lds_void*)L.rwq, 16, 0, 0);
      }
      if (lane < B && b0 + 2 * B + lane < qn) en2 = ql[b0 + 2 * B + lane];
    }
    // ---- walk batch b, two entries per iteration: their alphas are
    // independent and overlap; the decisions and accumulations run in list
    // order.  Slot j + 1 is always inside the batch buffers (B is even), so
    // both entries are read at fixed offsets with no clamp; past the end of
    // the batch its contents are stale and has2 keeps them out.
    static_assert(B % 2 == 0, "entry pairs stay inside the batch buffers");
    for (int j = 0; j < nb; j += 2) {
      const bool has2 = j + 1 < nb;
      float fl1[NM], fl2[NM];
      load_slice<NM>(cur + j * C + NM * q4, fl1);
      load_slice<NM>(cur + (j + 1) * C + NM * q4, fl2);
      const float4 w1 = L.wq[j], w2 = L.wq[j + 1];
      const float4 s1 = L.st[j], s2 = L.st[j + 1];
      const float al1 = blend_alpha(exponent(w1, s1.x, s1.y, fpx, fpy));
      const float al2 = blend_alpha(exponent(w2, s2.x, s2.y, fpx, fpy));
      if (COUNT) wc.steps += has2 ? 2 : 1;
      visit(fl1, __float_as_int(s1.z), b0 + j, al1, true);
      visit(fl2, __float_as_int(s2.z), b0 + j + 1, al2, has2);
    }
    const bool live = __builtin_amdgcn_ballot_w64(amin < 1.f) != 0;
    // ---- batch b+1 has landed; stage its state (batch b's is no longer read)
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (more && lane < nb1) {
      const double2 nxy = L.rxy[lane];
      const float4 nwq = L.rwq[lane];
      const float2 cc = exponent_offsets(nxy, nwq, ox, oy);
      L.wq[lane] = nwq;
      L.st[lane] = make_float4(cc.x, cc.y, __int_as_float(en.y), 0.f);
    }
    en = en2;
    __builtin_amdgcn_wave_barrier();
    if (!live) break;                 // every pixel of the quadrant has ended
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
    const int px0 = tx * TILE + ((qd & 1) << 3) + (b4 & 7);
    const int py0 = ty * TILE + ((qd >> 1) << 3) + (b4 >> 3);
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
  if (lane == 0) a.qcut[4 * gtile + qd] = qlast + 1;   // where the adjoint's backward walk starts
  if (COUNT && inside) {
    // evaluated pairs of the plain walk over the tile's list: every list
    // position up to the stop
    wc.n_eval += stop_pos >= 0 ? (uint32_t)(stop_pos + 1) : (uint32_t)len;
  }
}

// Workgroups of four independent waves, one per tile slot of the batch.
// Work item i is quadrant i & 3 of the tile at position i >> 2 of the tile
// order (longest tiles first); wave w of workgroup b takes item 4 b + w
// (and 4 (b + G) + w, ... if a grid of G workgroups were smaller than the
// tile count), so the four waves of a workgroup blend the four quadrants of
// one tile (sharing its Gaussians in the CU's cache) and each blends alone,
// without a workgroup barrier.  The hardware starts workgroups in index
// order as compute units free up, which makes the schedule a greedy
// longest-first one: measured against 2,048 persistent workgroups that
// each walked two fixed positions of the order, 6.5 % less time on the
// realistic frame.  A device-wide atomic counter handing out items
// serialises at that counter instead (measured: it doubled the blend's
// time).  TABLE: the batch's requests come from the device table (a
// replayed serving batch) rather than inline (a single render); the two
// are separate instantiations so that each keeps its own launch
// statistics.
template <int C, bool COUNT, bool TABLE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_render(BatchArgs a) {
  if (!TABLE) a.table = nullptr;
  // both reads in flight before the first branch: most workgroups of a
  // serving slot's launch lie past the batch's tiles and leave here
  const int overflow = a.dev->overflow;
  const BatchHdr h = batch_hdr(a);
  if (overflow != 0 || (int)blockIdx.x >= h.n_tiles) return;
  constexpr int B = wave_batch<C>();
  __shared__ WaveLDS<C, B> LW[4];
  const int lane = threadIdx.x & 63;
  // the wave's index, as a wave-uniform (scalar) value: everything derived
  // from the work item (tile, request, list bounds) then stays in scalar
  // registers and scalar arithmetic
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  WaveLDS<C, B>& L = LW[wv];
  WorkCount wc;
  const int n_items = 4 * h.n_tiles;
  for (int item = 4 * (int)blockIdx.x + wv; item < n_items; item += 4 * (int)gridDim.x) {
    const int t = a.tile_order[item >> 2];
    const int r = req_of_tile(a, h, t);
    if (r < 0) break;
    const ReqDev& q = batch_req(a, r);
    const int lt = t - q.tile_off;
    render_quadrant<C, B, COUNT>(a, q, t, lt % q.cam.tiles_x, lt / q.cam.tiles_x, item & 3, L, wc);
  }
  if (COUNT) {
    // wave sums of the lane counts, then one atomic per wave and count
    unsigned long long v[5] = {wc.n_eval, wc.n_blend, wc.steps, wc.steps_pass, wc.steps_blend};
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if (lane == 0) {
      atomicAdd(&a.dev->n_eval, v[0]);
      atomicAdd(&a.dev->n_blend, v[1]);
      atomicAdd(&a.dev->wave_steps, v[2]);
      atomicAdd(&a.dev->wave_pass, v[3]);
      atomicAdd(&a.dev->wave_blend, v[4]);
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
hipError_t launch_c(const BatchArgs& a, int32_t grid_tiles, hipStream_t s, bool count) {
  const int grid = grid_tiles > 0 ? grid_tiles : 1;   // one workgroup per tile slot
  if (count) {                        // work counts: single renders only
    if (a.table) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(1), 0, s, a.dev);
    hipLaunchKernelGGL((k_render<C, true, false>), dim3(grid), dim3(256), 0, s, a);
  } else {
    if (a.table) hipLaunchKernelGGL((k_render<C, false, true>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_render<C, false, false>), dim3(grid), dim3(256), 0, s, a);
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
