// render_bwd.hip -- adjoint of the rasterizer (gfx950).  §4.2 trains the
// encoder and decoder through R_G, so R_G must be differentiable.
//
// k_render_bwd: one wave64 per (tile, 8x8 quadrant) work item, the
// forward's pixel layout and work assignment, walking the quadrant's own
// list (from the sort) backwards from the end the forward recorded for it
// (one past the last entry some pixel of the quadrant blended), one wave
// per workgroup.  Each group of 16 entries arrives by LDS DMA (feature
// rows, FP64 means, exponent factors, conics) while the previous group's
// sums run.  Nothing per (pixel, Gaussian) is stored by the
// forward: each pixel starts from its final transmittance T_final and the
// list position of its last blended Gaussian and walks its list backwards,
// re-deciding skip / blend with the forward's own float operations (shared
// code) and recovering T_i = T_{i+1} / (1 - alpha_i).  With
// S_i = sum_{j>i} alpha_j T_j f_j + T_final bg (kept as <g, S_i>, g = dL/dF
// of the pixel):
//   dL/dalpha_i = T_i <g, f_i> - (<g, S_i> - dL/dA_out T_final) / (1 - alpha_i)
//   dL/df_i    += w_i g,  w_i = alpha_i T_i
//   dL/dP_i     = alpha_i dL/dalpha_i (0 where alpha is clamped at 0.99)
// and the 2D gradients of (u, v, conic A, B, C, opacity) follow from dL/dP
// and the pixel offset d = p - (u, v).
//
// The per-Gaussian sums over a wave's 64 pixels are dense contractions and
// run on the matrix cores.  Each wave walks the Gaussians of its quadrant
// list in groups of 16; the walk writes each pixel's w_i and dL/dP_i into
// LDS, then
//   dL/df[i][c]  = sum_p w_i(p) g(p)[c]            (16 x C x 64)
//   M[i][k]      = sum_p dL/dP_i(p) phi_k(p)         (16 x 6 x 64)
// are v_mfma_f32_16x16x4_f32 products with the pixels as the reduction
// index; phi = (1, x, y, x^2, xy, y^2) of the pixel centre relative to the
// wave's quadrant centre, from which the six 2D gradient sums are assembled
// exactly (sum dP dx = M_x - u M_1, ...).  Each wave adds its group's sums to the
// per-Gaussian accumulators with one float atomic per value.
//
// k_project_bwd: one lane per Gaussian, FP64 chain rule from the 2D
// gradients to the raw parameters (mean, log-scale, unnormalised
// quaternion, opacity logit) through the EWA projection.
#include "blend_common.h"

namespace tg {
namespace {

constexpr int GROUP = 16;      // Gaussians per staged group and per matrix-core reduction
// LDS row of one group Gaussian's 64 pixel values, padded by 4 floats: the
// matrix-core operand reads take one row per lane column (16 rows at once),
// and an unpadded 64-float stride would put all of them on the same banks
constexpr int ROW = 68;

// One wave's LDS (one per workgroup of one wave): the feature rows of
// the group being walked (LDS DMA target, refilled with the next group's
// while this group's sums run), the next group's raw FP64 means, exponent
// factors and conics (DMA targets), this group's staged state in walk order,
// and the pixel values of the matrix-core sums.  The DMA targets are the
// wave's rows of LDS arrays of their own, so the compiler can tell them from
// what the sums and the atomics read: those never wait for the DMA.
struct BwdBufs {
  float* fe;                   // [GROUP * C] feature rows
  double2* rxy;                // [GROUP] raw FP64 means
  float4* rwq;                 // [GROUP] raw exponent factors
  float4* rcn;                 // [GROUP] raw conics and opacities
};

template <int C>
struct BwdWork {
  float4 wq[GROUP];            // exponent factors, as in the forward
  float4 st[GROUP];            // (c1, c2, u, v): tile offsets and tile-relative mean
  float4 cn[GROUP];            // unscaled conic A, B, C and opacity
  int2 ent[GROUP];             // (global index, tile-list position)
  // row i of the group: pixel values in k-block order, p = 4 kb + q stored at
  // q * 16 + kb (so one lane's 16 A operands are contiguous)
  __align__(16) float wa[GROUP * ROW];
  __align__(16) float dp[GROUP * ROW];
  float mom[GROUP][9];         // 9: rows on distinct banks for the per-row reads
};

__device__ __forceinline__ int perm64(int p) { return (p & 3) * 16 + (p >> 2); }

typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(3))) void lds_void;

// float atomic add on a global-memory address (no-return form; the generic
// form would be a flat atomic that also counts against the LDS counter)
__device__ __forceinline__ void atomic_add_global(float* p, float v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f32((gfloat*)p, v);
}

// LDS DMA of a group's feature rows (lane j < n holds entry j's global index
// gi) and raw state into the wave's buffers: 16-byte chunks, C / 4 lanes per
// row; lanes past the group's GROUP rows stay idle, rows past n read row 0's
// address (in bounds) and are never walked.
template <int C>
__device__ __forceinline__ void dma_group(const BatchArgs& a, const float* __restrict__ feat, int64_t g_off,
                                          const BwdBufs& B, int gi, int n, int lane) {
  constexpr int LPR = C / 4;
  constexpr int RPI = 64 / LPR;
  constexpr int NI = (GROUP + RPI - 1) / RPI;
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int row = k * RPI + lane / LPR;
    const int g = __shfl(gi, row < n ? row : 0, 64);
    if (k * RPI < n && row < GROUP)
      __builtin_amdgcn_global_load_lds((const void*)(feat + (g - g_off) * C + 4 * (lane % LPR)),
                                       (lds_void*)(B.fe + k * RPI * C), 16, 0, 0);
  }
  if (lane < n) {
    __builtin_amdgcn_global_load_lds((const void*)(a.xy + gi), (lds_void*)B.rxy, 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(a.wq + gi), (lds_void*)B.rwq, 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(a.conic_o + gi), (lds_void*)B.rcn, 16, 0, 0);
  }
}

// Staged state of group entry j (after its DMA landed): the forward's
// tile-dependent exponent offsets (the same operations) and the
// tile-relative mean for the 2D gradient moments.
template <int C>
__device__ __forceinline__ void stage_entry(const BwdBufs& B, BwdWork<C>& L, int j, int2 e, double ox, double oy) {
  const double2 xy = B.rxy[j];
  const float4 wq = B.rwq[j];
  const float2 cc = exponent_offsets(xy, wq, ox, oy);
  L.wq[j] = wq;
  L.st[j] = make_float4(cc.x, cc.y, (float)(xy.x - ox), (float)(xy.y - oy));
  L.cn[j] = B.rcn[j];
  L.ent[j] = e;
}

// The adjoint of the 8x8 quadrant qd of one tile (tile-local coordinates
// tx, ty of request q) by one wave: the quadrant's list backwards from the
// last entry the forward blended in it, in groups of GROUP.
template <int C>
__device__ __forceinline__ void bwd_quadrant(const BatchArgs& a, const ReqDev& q, int gtile, int tx, int ty, int qd,
                                             const BwdBufs& B, BwdWork<C>& L) {
  const int kend = a.qcut[4 * gtile + qd];
  if (kend == 0) return;                      // no pixel of the quadrant blended anything
  constexpr int NB = (C + 15) / 16;           // 16-channel blocks of dL/df
  const int lane = threadIdx.x & 63;
  const int ql4 = lane >> 4, l16 = lane & 15; // MFMA operand row / column of this lane
  const int qx0 = (qd & 1) << 3, qy0 = (qd >> 1) << 3;
  const int lx = qx0 | (lane & 7), ly = qy0 | (lane >> 3);
  const int W = q.cam.W, H = q.cam.H;
  const int px = tx * TILE + lx, py = ty * TILE + ly;
  const bool inside = px < W && py < H;
  const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;
  const double ox = (double)(tx * TILE), oy = (double)(ty * TILE);
  const int s = a.tile_start[gtile], len = a.tile_start[gtile + 1] - s;
  const int2* qlst = a.qlist + 4 * (int64_t)s + (int64_t)qd * len;
  const size_t HW = (size_t)W * H;
  const float* feat = q.feat;
  float* const d_feat = q.d_feat;
  const int64_t g_off = q.s_off;              // the lists hold indices of this 2D-state range
  const int64_t acc_off = q.g_off - q.s_off;  // ... the adjoint accumulates in the request's own range

  // group 0 (the last GROUP entries) on its way while the pixel state loads
  int n = min(GROUP, kend);
  int2 e = lane < n ? qlst[kend - 1 - lane] : make_int2(0, 0);
  dma_group<C>(a, feat, g_off, B, e.x, n, lane);

  // ---- per-pixel state
  float g[C];
  float T = 1.f, sgS = 0.f, gAT = 0.f;
  int last = -1;
  if (inside) {
    const size_t pix = (size_t)py * W + px;
    const float Tfin = q.T_final[pix];
    T = Tfin;
    last = q.last[pix];
    gAT = (q.d_alpha ? q.d_alpha[pix] : 0.f) * Tfin;
    float gb = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      g[c] = q.d_img[c * HW + pix];
      gb = __builtin_fmaf(g[c], q.bg ? q.bg[c] : 0.f, gb);
    }
    sgS = Tfin * gb;
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = 0.f;
  }
  // ---- matrix-core operands fixed for the quadrant.  B of the dL/df
  // product: lane (ql4, l16) of k-block kb holds g[c = 16 nb + l16] of wave
  // pixel p = 4 kb + ql4; B of the moment product holds phi_l16 of that pixel.
  float gB[NB][16], phB[16];
#pragma unroll
  for (int kb = 0; kb < 16; ++kb) {
    const int p = 4 * kb + ql4;
    const int plx = qx0 | (p & 7), ply = qy0 | (p >> 3);
    const int ppx = tx * TILE + plx, ppy = ty * TILE + ply;
    const bool pin = ppx < W && ppy < H;
    const size_t ppix = pin ? (size_t)ppy * W + ppx : 0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = 16 * nb + l16;
      gB[nb][kb] = (pin && c < C) ? q.d_img[c * HW + ppix] : 0.f;
    }
    const float x = (float)(plx - qx0) - 3.5f, y = (float)(ply - qy0) - 3.5f;
    float ph = 0.f;
    ph = l16 == 0 ? 1.f : ph;
    ph = l16 == 1 ? x : ph;
    ph = l16 == 2 ? y : ph;
    ph = l16 == 3 ? x * x : ph;
    ph = l16 == 4 ? x * y : ph;
    ph = l16 == 5 ? y * y : ph;
    phB[kb] = ph;
  }
  __builtin_amdgcn_s_waitcnt(0);              // group 0 has landed
  __builtin_amdgcn_wave_barrier();
  if (lane < n) stage_entry<C>(B, L, lane, e, ox, oy);
  __builtin_amdgcn_wave_barrier();

  for (int k1 = kend; k1 > 0; k1 -= GROUP) {
    n = min(GROUP, k1);
    const int nn = min(GROUP, k1 - GROUP);    // the next group's size (<= 0: none)
    int2 en = make_int2(0, 0);
    if (lane < nn) en = qlst[k1 - GROUP - 1 - lane];
    // ---- walk the group, last entry first: row i is list entry k1 - 1 - i
    uint32_t cmask = 0;                       // rows of the group some pixel blends
    for (int i = 0; i < n; ++i) {
      const int pos = L.ent[i].y;
      const float4 wq = L.wq[i], st = L.st[i];
      const float oG = __builtin_amdgcn_exp2f(exponent(wq, st.x, st.y, fpx, fpy));
      const float al = fminf(0.99f, oG);
      const bool contrib = pos <= last && al >= ALPHA_MIN;
      float wv = 0.f, dv = 0.f;
      if (__builtin_amdgcn_ballot_w64(contrib) != 0) {
        cmask |= 1u << i;
        const float* fr = B.fe + i * C;
        float fg = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) fg = __builtin_fmaf(fr[c], g[c], fg);
        // T_i = T_{i+1} / (1 - alpha_i) with a correctly rounded division:
        // the recursion runs over the whole list, an approximate
        // reciprocal would let its error grow with the list length
        const float oma = 1.f - al;
        const float Ti = T / oma;
        const float dLda = Ti * fg + (gAT - sgS) * __builtin_amdgcn_rcpf(oma);
        const float wgt = al * Ti;
        wv = contrib ? wgt : 0.f;
        dv = contrib && oG <= 0.99f ? dLda * al : 0.f;
        sgS = contrib ? __builtin_fmaf(wgt, fg, sgS) : sgS;
        T = contrib ? Ti : T;
      }
      L.wa[i * ROW + perm64(lane)] = wv;
      L.dp[i * ROW + perm64(lane)] = dv;
    }
    __builtin_amdgcn_wave_barrier();
    // ---- the feature rows are read: the next group's rows and raw state
    // arrive by DMA while this group's sums run
    if (nn > 0) dma_group<C>(a, feat, g_off, B, en.x, nn, lane);
    if (cmask != 0) {
      // sums over the wave's pixels on the matrix cores
      f4v accF[NB], accM = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int nb2 = 0; nb2 < NB; ++nb2) accF[nb2] = f4v{0.f, 0.f, 0.f, 0.f};
      const f4v* wrow = reinterpret_cast<const f4v*>(&L.wa[l16 * ROW + ql4 * 16]);
      const f4v* drow = reinterpret_cast<const f4v*>(&L.dp[l16 * ROW + ql4 * 16]);
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        const f4v av = wrow[k4], dvv = drow[k4];
#pragma unroll
        for (int ee = 0; ee < 4; ++ee) {
          const int kb = 4 * k4 + ee;
#pragma unroll
          for (int nb2 = 0; nb2 < NB; ++nb2)
            accF[nb2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ee], gB[nb2][kb], accF[nb2], 0, 0, 0);
          accM = __builtin_amdgcn_mfma_f32_16x16x4f32(dvv[ee], phB[kb], accM, 0, 0, 0);
        }
      }
      // accF[nb][r] = dL/df[row 4 ql4 + r][16 nb + l16]; accM[r] = M[row 4 ql4 + r][l16]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * ql4 + r;
        if (l16 < 6) L.mom[i][l16] = accM[r];
        if (i < n && ((cmask >> i) & 1u)) {
          float* dst = d_feat + (size_t)(L.ent[i].x - g_off) * C;
#pragma unroll
          for (int nb2 = 0; nb2 < NB; ++nb2) {
            const int c = 16 * nb2 + l16;
            if (c < C) atomic_add_global(dst + c, accF[nb2][r]);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      const int gi = L.ent[lane & (GROUP - 1)].x;
      const float4 st = L.st[lane & (GROUP - 1)], cn = L.cn[lane & (GROUP - 1)];
      // 2D gradients from the moments: lane j < n forms entry j's six
      // values; they go out as two instructions of 8 entries x 8 lanes,
      // each entry's six values one 32-byte row of g2d (six scattered
      // single-float atomics per entry cost twice as much)
      float v6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (lane < n && ((cmask >> lane) & 1u)) {
        const float* m = L.mom[lane];
        // pixel offsets d = p - (u, v) with p and (u, v) relative to the quadrant centre
        const float u = st.z - (float)(qx0 + 4), v = st.w - (float)(qy0 + 4);
        const float m1 = m[0], mx = m[1], my = m[2], mxx = m[3], mxy = m[4], myy = m[5];
        const float sdx = mx - u * m1, sdy = my - v * m1;
        const float sdxx = mxx - 2.f * u * mx + u * u * m1;
        const float sdxy = mxy - u * my - v * mx + u * v * m1;
        const float sdyy = myy - 2.f * v * my + v * v * m1;
        v6[0] = cn.x * sdx + cn.y * sdy;
        v6[1] = cn.z * sdy + cn.y * sdx;
        v6[2] = -0.5f * sdxx;
        v6[3] = -sdxy;
        v6[4] = -0.5f * sdyy;
        v6[5] = m1 / cn.w;
      }
      const int k = lane & 7;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = 8 * h + (lane >> 3);
        float vk = 0.f;
#pragma unroll
        for (int kk = 0; kk < 6; ++kk) {
          const float t = __shfl(v6[kk], e, 64);
          vk = k == kk ? t : vk;
        }
        const int egi = __shfl(gi, e, 64);
        if (k < 6 && e < n && ((cmask >> e) & 1u)) atomic_add_global(a.g2d + (egi + acc_off) * 8 + k, vk);
      }
    }
    // ---- the next group has landed: stage it (this group's state is no longer read)
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (lane < nn) stage_entry<C>(B, L, lane, en, ox, oy);
    __builtin_amdgcn_wave_barrier();
  }
}

// One wave per workgroup and (tile, quadrant) work item.  Item i is
// quadrant i & 3 of the tile at position i >> 2 of the tile order (longest
// tiles first).  The hardware starts workgroups in index order as compute
// units free up, one XCD after the other in turn, so workgroup b takes
// tile 8 (b / 32) + b % 8 and quadrant (b / 8) % 4: the four quadrants of
// a tile run on one XCD (sharing its Gaussians in that XCD's L2), the
// order stays longest first in steps of eight tiles, and a wave that ends
// frees its slot and its LDS for the next item at once.  Measured on the
// realistic frame: 1,536 persistent four-wave workgroups striding over the
// items 0.513 ms, one four-wave workgroup per tile 0.474 ms, one wave per
// item 0.455 ms.
template <int C>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) k_render_bwd(BatchArgs a) {
  // both reads in flight before the first branch: most workgroups of a
  // serving slot's launch lie past the batch's tiles and leave here
  const int overflow = a.dev->overflow;
  const BatchHdr h = batch_hdr(a);
  __shared__ __align__(16) float FE[GROUP * C];
  __shared__ double2 RXY[GROUP];
  __shared__ float4 RWQ[GROUP];
  __shared__ float4 RCN[GROUP];
  __shared__ BwdWork<C> L;
  const BwdBufs B{FE, RXY, RWQ, RCN};
  const int n_items = 4 * h.n_tiles;
  const int b = (int)blockIdx.x;
  const int item = 4 * (8 * (b >> 5) + (b & 7)) + ((b >> 3) & 3);
  if (overflow != 0 || item >= n_items) return;
  const int t = a.tile_order[item >> 2];
  const int r = req_of_tile(a, h, t);
  if (r < 0) return;
  const ReqDev& q = batch_req(a, r);
  if (!q.d_img) return;            // a forward-only request of a mixed batch
  const int lt = t - q.tile_off;
  bwd_quadrant<C>(a, q, t, lt % q.cam.tiles_x, lt / q.cam.tiles_x, item & 3, B, L);
}

// zero the 2D accumulators of the batch's index range and the feature
// gradient of each request that asks for an adjoint
__global__ void k_bwd_zero(BatchArgs a, int c) {
  const BatchHdr h = batch_hdr(a);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float4* g2 = reinterpret_cast<float4*>(a.g2d);
  for (int64_t i = i0; i < 2 * h.g_end; i += stride) g2[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int r = 0; r < h.n_req; ++r) {
    const ReqDev& q = batch_req(a, r);
    if (!q.d_img || !q.d_feat) continue;
    for (int64_t i = i0; i < q.n * c; i += stride) q.d_feat[i] = 0.f;
  }
}

template <int C>
hipError_t launch_bwd_c(const BatchArgs& a, int32_t grid_tiles, hipStream_t s) {
  // one workgroup per (tile slot, quadrant), in whole groups of 32
  const int grid = ((4 * (grid_tiles > 0 ? grid_tiles : 1) + 31) / 32) * 32;
  hipLaunchKernelGGL((k_render_bwd<C>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------- project backward
// Raw-parameter gradients of one Gaussian, accumulated in FP64.
struct RawGrad {
  double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dlg = 0;
};

// Add the chain rule of Gaussian i of request qr (read through a reference
// whose address space the caller fixes, so its fields are wave-uniform
// scalar loads; its 2D gradients sit at global index gi) to g.
__device__ __forceinline__ void project_bwd_add(const BatchArgs& a, const ReqDev& qr, int64_t i, int64_t gi,
                                                RawGrad& g) {
  const int64_t n = qr.n;
  double* dmu = g.dmu;
  double* dls = g.dls;
  double* dq = g.dq;
  const uint2 r = a.rect[qr.s_off + i];       // the projection this request's render used
  const bool live = (r.x & 0xffffu) <= (r.x >> 16);
  if (live) {
    const CamArgs& c = qr.cam;
    double W[9];
    for (int k = 0; k < 9; ++k) W[k] = c.R[k];
    const double X = qr.mean[i], Y = qr.mean[n + i], Z = qr.mean[2 * n + i];
    const double tx = W[0] * X + W[1] * Y + W[2] * Z + (double)c.t[0];
    const double ty = W[3] * X + W[4] * Y + W[5] * Z + (double)c.t[1];
    const double tz = W[6] * X + W[7] * Y + W[8] * Z + (double)c.t[2];
    const double fx = c.fx, fy = c.fy;
    const double s3[3] = {qr.scale[i], qr.scale[n + i], qr.scale[2 * n + i]};
    const double q0[4] = {qr.quat[i], qr.quat[n + i], qr.quat[2 * n + i], qr.quat[3 * n + i]};
    const double nq = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
    const double qw = q0[0] / nq, qx = q0[1] / nq, qy = q0[2] / nq, qz = q0[3] / nq;
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                         2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                         2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double M[9];   // R diag(s)
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k) M[3 * p + k] = R[3 * p + k] * s3[k];
    double S[9];   // Sigma3D = M M^T
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k)
        S[3 * p + k] = M[3 * p] * M[3 * k] + M[3 * p + 1] * M[3 * k + 1] + M[3 * p + 2] * M[3 * k + 2];
    const double iz = 1.0 / tz, iz2 = iz * iz, iz3 = iz2 * iz;
    const double J[6] = {fx * iz, 0.0, -fx * tx * iz2, 0.0, fy * iz, -fy * ty * iz2};
    double A[6];   // J W
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 3; ++k) A[3 * p + k] = J[3 * p] * W[k] + J[3 * p + 1] * W[3 + k] + J[3 * p + 2] * W[6 + k];
    double AS[6];
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 3; ++k) AS[3 * p + k] = A[3 * p] * S[k] + A[3 * p + 1] * S[3 + k] + A[3 * p + 2] * S[6 + k];
    const double sa = AS[0] * A[0] + AS[1] * A[1] + AS[2] * A[2] + 0.3;
    const double sb = AS[0] * A[3] + AS[1] * A[4] + AS[2] * A[5];
    const double sc = AS[3] * A[3] + AS[4] * A[4] + AS[5] * A[5] + 0.3;
    const double det = sa * sc - sb * sb;
    const double cA = sc / det, cB = -sb / det, cC = sa / det;
    const float4 g2a = reinterpret_cast<const float4*>(a.g2d)[2 * gi];
    const float4 g2b = reinterpret_cast<const float4*>(a.g2d)[2 * gi + 1];
    const double gu = g2a.x, gv = g2a.y;
    const double gA = g2a.z, gB = g2a.w, gC = g2b.x;
    const double gO = g2b.y;
    // conic = inverse(Sigma'): G_Sigma = -Q G_Q Q with G_Q = [[gA, gB/2], [gB/2, gC]]
    const double Q[4] = {cA, cB, cB, cC};
    const double GQ[4] = {gA, 0.5 * gB, 0.5 * gB, gC};
    double T1[4], GS[4];
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 2; ++k) T1[2 * p + k] = Q[2 * p] * GQ[k] + Q[2 * p + 1] * GQ[2 + k];
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 2; ++k) GS[2 * p + k] = -(T1[2 * p] * Q[k] + T1[2 * p + 1] * Q[2 + k]);
    // Sigma2D = A Sigma3D A^T
    double G3[9];
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int x = 0; x < 2; ++x)
          for (int y = 0; y < 2; ++y) acc += A[3 * x + p] * GS[2 * x + y] * A[3 * y + k];
        G3[3 * p + k] = acc;
      }
    double GA[6];   // 2 G_S A Sigma3D
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int y = 0; y < 2; ++y)
          for (int l = 0; l < 3; ++l) acc += GS[2 * p + y] * A[3 * y + l] * S[3 * l + k];
        GA[3 * p + k] = 2.0 * acc;
      }
    double GJ[6];   // dL/dJ = dL/dA W^T
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 3; ++k) GJ[3 * p + k] = GA[3 * p] * W[3 * k] + GA[3 * p + 1] * W[3 * k + 1] + GA[3 * p + 2] * W[3 * k + 2];
    double gt[3];
    gt[0] = gu * fx * iz - GJ[2] * fx * iz2;
    gt[1] = gv * fy * iz - GJ[5] * fy * iz2;
    gt[2] = -gu * fx * tx * iz2 - gv * fy * ty * iz2 - GJ[0] * fx * iz2 + GJ[2] * 2.0 * fx * tx * iz3 -
            GJ[4] * fy * iz2 + GJ[5] * 2.0 * fy * ty * iz3;
    for (int k = 0; k < 3; ++k) dmu[k] += W[k] * gt[0] + W[3 + k] * gt[1] + W[6 + k] * gt[2];
    // Sigma3D = M M^T, M = R diag(s)
    double GM[9];
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k)
        GM[3 * p + k] = 2.0 * (G3[3 * p] * M[k] + G3[3 * p + 1] * M[3 + k] + G3[3 * p + 2] * M[6 + k]);
    double GR[9];
    for (int k = 0; k < 3; ++k) {
      double ds = 0;
      for (int p = 0; p < 3; ++p) {
        GR[3 * p + k] = GM[3 * p + k] * s3[k];
        ds += GM[3 * p + k] * R[3 * p + k];
      }
      dls[k] += ds * s3[k];
    }
    double gq[4];
    gq[0] = 2 * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
    gq[1] = 2 * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2 * qx * GR[4] - qw * GR[5] + qz * GR[6] + qw * GR[7] -
                 2 * qx * GR[8]);
    gq[2] = 2 * (-2 * qy * GR[0] + qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] + qz * GR[7] -
                 2 * qy * GR[8]);
    gq[3] = 2 * (-2 * qz * GR[0] - qw * GR[1] + qx * GR[2] + qw * GR[3] - 2 * qz * GR[4] + qy * GR[5] + qx * GR[6] +
                 qy * GR[7]);
    const double dot = qw * gq[0] + qx * gq[1] + qy * gq[2] + qz * gq[3];
    const double qh[4] = {qw, qx, qy, qz};
    for (int k = 0; k < 4; ++k) dq[k] += (gq[k] - qh[k] * dot) / nq;
    const double o = qr.opacity[i];
    g.dlg += o * (1.0 - o) * gO;
  }
}

// Write the accumulated gradients of Gaussian i of request qr.
__device__ __forceinline__ void project_bwd_write(const ReqDev& qr, int64_t i, const RawGrad& g) {
  const int64_t n = qr.n;
  const double* dmu = g.dmu;
  const double* dls = g.dls;
  const double* dq = g.dq;
  const double dlg = g.dlg;
  if (qr.d_mean)
    for (int k = 0; k < 3; ++k) qr.d_mean[k * n + i] = (float)dmu[k];
  if (qr.d_log_scale)
    for (int k = 0; k < 3; ++k) qr.d_log_scale[k * n + i] = (float)dls[k];
  if (qr.d_quat)
    for (int k = 0; k < 4; ++k) qr.d_quat[k * n + i] = (float)dq[k];
  if (qr.d_logit) qr.d_logit[i] = (float)dlg;
}

template <bool TABLE>
__global__ void __launch_bounds__(256) k_project_bwd(BatchArgs a) {
  const BatchHdr h = TABLE ? *a.hdr_dev : a.hdr;
  const int64_t g0 = (int64_t)blockIdx.x * 256;
  if (g0 >= h.g_end) return;
  const int64_t gi = g0 + threadIdx.x;
  RawGrad g;
  if (TABLE) {                                   // a batch's table in global memory
    const int rq = req_of_gauss(a, h, g0);
    if (rq < 0) return;
    const ReqDev& q = a.table[rq];
    if (q.covered) return;                       // chained by the first view of its set
    const int64_t i = gi - q.g_off;
    if (i >= q.n || !q.d_img) return;            // no adjoint asked for this request
    const int nv = q.extra_views;
    for (int v = 0; v <= nv; ++v) {              // every view of the set: summed
      const ReqDev& qv = a.table[rq + v];
      project_bwd_add(a, qv, i, qv.g_off + i, g);
    }
    project_bwd_write(q, i, g);
  } else {                                       // one request in the kernel arguments
    const int64_t i = gi - a.one.g_off;
    if (i >= a.one.n || !a.one.d_img) return;
    project_bwd_add(a, a.one, i, gi, g);
    project_bwd_write(a.one, i, g);
  }
}

}  // namespace

hipError_t launch_render_bwd(const BatchArgs& a, int c, int64_t grid_gauss, int32_t grid_tiles,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_zero, dim3(1024), dim3(256), 0, s, a, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (c) {
    case 8: e = launch_bwd_c<8>(a, grid_tiles, s); break;
    case 16: e = launch_bwd_c<16>(a, grid_tiles, s); break;
    case 32: e = launch_bwd_c<32>(a, grid_tiles, s); break;
    case 64: e = launch_bwd_c<64>(a, grid_tiles, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int64_t blocks = (grid_gauss + 255) / 256;
  if (a.table) hipLaunchKernelGGL(k_project_bwd<true>, dim3((int)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_project_bwd<false>, dim3((int)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tg
