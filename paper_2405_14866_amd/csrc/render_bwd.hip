// render_bwd.hip -- adjoint of the rasterizer (gfx950).  §4.2 trains the
// encoder and decoder through R_G, so R_G must be differentiable.
//
// k_render_bwd: one 256-lane workgroup per 16x16 tile (same pixel layout as
// the forward).  Nothing per (pixel, Gaussian) is stored by the forward;
// each pixel starts from its final transmittance T_final and the list
// position of its last blended Gaussian, and walks its list backwards,
// re-deciding skip / blend with exactly the forward's float operations and
// recovering T_i = T_{i+1} / (1 - alpha_i).  With S_i = sum_{j>i} alpha_j
// T_j f_j + T_final bg (tracked as the scalar <dL/dF, S_i>):
//   dL/dalpha_i = T_i <g, f_i> - <g, S_i> / (1 - alpha_i)
//                 + dL/dA_out T_final / (1 - alpha_i)
//   dL/df_i    += alpha_i T_i g
// and, unless alpha was clamped at 0.99, dL/dP = alpha dL/dalpha with
// P = -(A dx^2 + C dy^2)/2 - B dx dy, giving the 2D gradients (u, v, A, B,
// C, opacity).  Per Gaussian the 64 lanes' contributions are summed by a
// transposing butterfly (each exchange halves the values a lane holds, so
// V values cost about V shuffles instead of 6 V), the 4 waves are summed in
// LDS and the tile's total is added to the per-Gaussian accumulators with
// one float atomic per value.
//
// k_project_bwd: one lane per Gaussian, FP64 chain rule from the 2D
// gradients to the raw parameters (mean, log-scale, unnormalised
// quaternion, opacity logit) through the EWA projection.
#include "tg_internal.h"

namespace tg {
namespace {

constexpr float LOG2E = 1.4426950408889634f;

// Sum V values over the 64 lanes.  On return v[0] of every lane holds the
// full sum of value index reduce_index<V>(lane).
template <int V>
__device__ __forceinline__ void transpose_reduce(float (&v)[V], int lane) {
  int o = 32;
#pragma unroll
  for (int half = V / 2; half >= 1; half >>= 1) {
    if (o >= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const float send = up ? v[i] : v[i + half];
        const float keep = up ? v[i + half] : v[i];
        v[i] = keep + __shfl_xor(send, o, 64);
      }
      o >>= 1;
    }
  }
  for (; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o, 64);
}

template <int V>
__device__ __forceinline__ int reduce_index(int lane) {
  int idx = 0, o = 32;
  for (int half = V / 2; half >= 1 && o >= 1; half >>= 1, o >>= 1)
    if (lane & o) idx += half;
  return idx;
}

// lanes whose bits below the butterfly's split bits are zero hold unique results
template <int V>
__device__ __forceinline__ bool reduce_writer(int lane) {
  int bits = 0;
  for (int x = V; x > 1; x >>= 1) ++bits;
  if (bits >= 6) return true;
  const int low = (1 << (6 - bits)) - 1;
  return (lane & low) == 0;
}

template <int C, int BATCH>
struct BwdShared {
  float4 sg[BATCH];     // u, v (tile-local), opacity, log2 threshold
  float4 sq[BATCH];     // scaled conic (as in the forward)
  float4 sc[BATCH];     // unscaled conic A, B, C
  int32_t sidx[BATCH];
  __align__(16) float sf[BATCH][C + 4];
  float r2d[4][BATCH][8];
  float rft[4][BATCH][C];
  int32_t rflag[4][BATCH];
  int32_t smax;
};

template <int C, int BATCH>
__device__ __forceinline__ void bwd_tile(const BatchArgs& a, const ReqDev& q, int gtile, int tx, int ty,
                                         BwdShared<C, BATCH>& sh) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int lx = ((w & 1) << 3) | (lane & 7);
  const int ly = ((w >> 1) << 3) | (lane >> 3);
  const int W = q.cam.W, H = q.cam.H;
  const int px = tx * TILE + lx, py = ty * TILE + ly;
  const bool inside = px < W && py < H;
  const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;
  const double ox = (double)(tx * TILE), oy = (double)(ty * TILE);
  const int s = a.tile_start[gtile];
  auto& sg = sh.sg; auto& sq = sh.sq; auto& sc = sh.sc; auto& sidx = sh.sidx; auto& sf = sh.sf;
  auto& r2d = sh.r2d; auto& rft = sh.rft; auto& rflag = sh.rflag; auto& smax = sh.smax;

  const size_t HW = (size_t)W * H;
  const size_t pix = inside ? (size_t)py * W + px : 0;
  float g[C];
  float T = 1.f, gA = 0.f, sgS = 0.f, Tfin = 1.f;
  int last = -1;
  if (inside) {
    Tfin = q.T_final[pix];
    T = Tfin;
    last = q.last[pix];
    gA = q.d_alpha ? q.d_alpha[pix] : 0.f;
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
  if (tid == 0) smax = -1;
  for (int k = tid; k < 4 * BATCH; k += 256) (&rflag[0][0])[k] = 0;
  __syncthreads();
  if (last >= 0) atomicMax(&smax, last);
  __syncthreads();
  const int maxlast = smax;
  if (maxlast < 0) {
    __syncthreads();                 // smax is rewritten by the next tile
    return;
  }
  const float gAT = gA * Tfin;

  for (int b = maxlast / BATCH; b >= 0; --b) {
    const int b0 = b * BATCH;
    const int nb = min(BATCH, maxlast + 1 - b0);
    if (tid < nb) {
      const int gi = a.sorted[s + b0 + tid];
      const double2 xy = a.xy[gi];
      const float4 co = a.conic_o[gi];
      const float o = co.w;
      const float thr = o > 0.f ? -log2f(255.f * o) : INFINITY;
      sg[tid] = make_float4((float)(xy.x - ox), (float)(xy.y - oy), o, thr);
      sq[tid] = make_float4(-0.5f * LOG2E * co.x, -LOG2E * co.y, -0.5f * LOG2E * co.z, 0.f);
      sc[tid] = make_float4(co.x, co.y, co.z, 0.f);
      sidx[tid] = gi;
      const float4* fr = reinterpret_cast<const float4*>(q.feat + (size_t)(gi - q.g_off) * C);
#pragma unroll
      for (int q = 0; q < C / 4; ++q) *reinterpret_cast<float4*>(&sf[tid][4 * q]) = fr[q];
    }
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      const int pos = b0 + j;
      const float4 gs = sg[j];
      const float4 q = sq[j];
      const float dx = fpx - gs.x, dy = fpy - gs.y;
      const float P = __builtin_fmaf(dx, __builtin_fmaf(q.x, dx, q.y * dy), q.z * dy * dy);
      bool contrib = false;
      float al = 0.f, G = 0.f;
      if (pos <= last && P <= 0.f && P >= gs.w) {
        G = __builtin_amdgcn_exp2f(P);
        al = fminf(0.99f, gs.z * G);
        contrib = al >= 1.f / 255.f;
      }
      if (__ballot(contrib) == 0) continue;
      float v2[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float vf[C];
      if (contrib) {
        const float oma = 1.f - al;
        const float Ti = T / oma;
        float fg = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) fg = __builtin_fmaf(sf[j][c], g[c], fg);
        const float dLda = Ti * fg + (gAT - sgS) / oma;
        const float wgt = al * Ti;
        sgS = __builtin_fmaf(wgt, fg, sgS);
#pragma unroll
        for (int c = 0; c < C; ++c) vf[c] = wgt * g[c];
        if (gs.z * G <= 0.99f) {
          const float4 cn = sc[j];
          // dx, dy here are pixel - mean; P = -(A dx^2 + C dy^2)/2 - B dx dy
          const float dP = dLda * al;
          v2[0] = dP * (cn.x * dx + cn.y * dy);
          v2[1] = dP * (cn.z * dy + cn.y * dx);
          v2[2] = -0.5f * dP * dx * dx;
          v2[3] = -dP * dx * dy;
          v2[4] = -0.5f * dP * dy * dy;
          v2[5] = dLda * G;
        }
        T = Ti;
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) vf[c] = 0.f;
      }
      transpose_reduce<8>(v2, lane);
      transpose_reduce<C>(vf, lane);
      if (reduce_writer<8>(lane)) r2d[w][j][reduce_index<8>(lane)] = v2[0];
      if (reduce_writer<C>(lane)) rft[w][j][reduce_index<C>(lane)] = vf[0];
      if (lane == 0) rflag[w][j] = 1;
    }
    __syncthreads();
    // sum the waves and add the tile's share to the per-Gaussian totals
    for (int k = tid; k < nb * (6 + C); k += 256) {
      const int j = k / (6 + C), v = k % (6 + C);
      float sum = 0.f;
      bool any = false;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        if (rflag[ww][j]) {
          any = true;
          sum += v < 6 ? r2d[ww][j][v] : rft[ww][j][v - 6];
        }
      }
      if (any) {
        const int gi = sidx[j];
        if (v < 6) atomicAdd(&a.g2d[(int64_t)v * a.g_cap + gi], sum);
        else atomicAdd(&q.d_feat[(size_t)(gi - q.g_off) * C + (v - 6)], sum);
      }
    }
    __syncthreads();
    for (int k = tid; k < 4 * BATCH; k += 256) (&rflag[0][0])[k] = 0;
    __syncthreads();
  }
}

template <int C, int BATCH>
__global__ void __launch_bounds__(256) k_render_bwd(BatchArgs a) {
  if (a.dev->overflow) return;
  const BatchHdr h = batch_hdr(a);
  __shared__ BwdShared<C, BATCH> sh;
  __shared__ int s_tile;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {                  // queue position -> tile, longest tiles first
      const int k = atomicAdd(&a.dev->bwd_queue, 1);
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
    bwd_tile<C, BATCH>(a, q, t, lt % q.cam.tiles_x, lt / q.cam.tiles_x, sh);
  }
  if (tid == 0 && atomicAdd(&a.dev->bwd_done, 1) == (int)gridDim.x - 1) {
    atomicExch(&a.dev->bwd_queue, 0);
    atomicExch(&a.dev->bwd_done, 0);
  }
}

// zero the 2D accumulators of the batch and each request's feature gradient
__global__ void k_bwd_zero(BatchArgs a, int c) {
  const BatchHdr h = batch_hdr(a);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < 6 * a.g_cap; i += stride) a.g2d[i] = 0.f;
  for (int r = 0; r < h.n_req; ++r) {
    const ReqDev& q = batch_req(a, r);
    for (int64_t i = i0; i < q.n * c; i += stride) q.d_feat[i] = 0.f;
  }
}

constexpr int BWD_PERSISTENT_WG = 256 * 6;

template <int C>
hipError_t launch_bwd_c(const BatchArgs& a, int32_t grid_tiles, hipStream_t s) {
  constexpr int BATCH = 32;
  const int grid = grid_tiles < BWD_PERSISTENT_WG ? (grid_tiles > 0 ? grid_tiles : 1) : BWD_PERSISTENT_WG;
  hipLaunchKernelGGL((k_render_bwd<C, BATCH>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------- project backward
__global__ void __launch_bounds__(256) k_project_bwd(BatchArgs a) {
  const BatchHdr h = batch_hdr(a);
  const int64_t g0 = (int64_t)blockIdx.x * 256;
  const int rq = req_of_gauss(a, h, g0);
  if (rq < 0) return;
  const ReqDev& qr = batch_req(a, rq);
  const int64_t gi = g0 + threadIdx.x;
  const int64_t i = gi - qr.g_off;
  const int64_t n = qr.n;
  if (i >= n) return;
  const int64_t gc = a.g_cap;
  double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dlg = 0;
  const uint2 r = a.rect[gi];
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
    const double gu = a.g2d[gi], gv = a.g2d[gc + gi];
    const double gA = a.g2d[2 * gc + gi], gB = a.g2d[3 * gc + gi], gC = a.g2d[4 * gc + gi];
    const double gO = a.g2d[5 * gc + gi];
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
    for (int k = 0; k < 3; ++k) dmu[k] = W[k] * gt[0] + W[3 + k] * gt[1] + W[6 + k] * gt[2];
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
      dls[k] = ds * s3[k];
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
    for (int k = 0; k < 4; ++k) dq[k] = (gq[k] - qh[k] * dot) / nq;
    const double o = qr.opacity[i];
    dlg = o * (1.0 - o) * gO;
  }
  if (qr.d_mean)
    for (int k = 0; k < 3; ++k) qr.d_mean[k * n + i] = (float)dmu[k];
  if (qr.d_log_scale)
    for (int k = 0; k < 3; ++k) qr.d_log_scale[k * n + i] = (float)dls[k];
  if (qr.d_quat)
    for (int k = 0; k < 4; ++k) qr.d_quat[k * n + i] = (float)dq[k];
  if (qr.d_logit) qr.d_logit[i] = (float)dlg;
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
  hipLaunchKernelGGL(k_project_bwd, dim3((int)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tg
