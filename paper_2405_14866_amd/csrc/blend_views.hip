// blend_views.hip -- occlusion-aware blending of the source views into the
// novel view, and the depth-map normals it weighs with (gfx950).
//
// §4.3 feeds the refiner a high-resolution image I_blend blended from the
// source views (Eq. 6-10).  Per novel pixel (u, v) with fused depth z:
//   X   = Pi_novel^-1(u + 0.5, v + 0.5, z)                      (Eq. 6)
//   per source view i: x_i = Pi_i(X) (camera point and pixel coordinates),
//   c_i, z_i, M_i, n_i = bilinear samples of colour, depth, mask and normal
//   map at x_i's pixel coordinates                               (Eq. 7)
//   w_i = M_i Occ_i max(0, -<r, n_i / |n_i|>) / |x_i^cam|         (Eq. 8)
//   Occ_i = 1 iff |x_i.z - z_i| < delta                          (Eq. 9)
//   I_blend = sum_i w_i c_i / sum_i w_i, 0 where the sum is 0    (Eq. 10)
// with r the unit ray of the novel pixel.  Bilinear sampling is between the
// four pixel centres around the point (top-left clamped to keep all four
// inside the view) and only for points inside the rectangle of the view's
// pixel centres; colours are 8-bit RGBA over 255.  The normal map of a view
// (k_normals) is the cross product of the central differences of the
// unprojected pixel centres, turned toward the view's camera, in the world
// frame; 0 on the border and where a depth of the stencil is not positive.
//
// Both kernels evaluate every quantity in FP64 in one fixed operation order
// (built with -ffp-contract=off; FP64 division and square root are
// correctly rounded), so any IEEE implementation of the same sequence gives
// the same float32 outputs bit for bit.  The cost is a few hundred FP64
// operations per (pixel, view): at CDNA4's vector FP64 rate this stays
// below the time of the gathers.
//
// Layout: one lane per novel pixel, 16x16 pixels per 256-lane workgroup
// (wave w takes rows 4w..4w+3, 64-byte row segments).  Neighbouring novel
// tiles fetch from overlapping source neighbourhoods, so the tile order is
// made XCD-aware: the hardware deals workgroups round-robin over the eight
// XCDs, and the kernel maps workgroup b to tile (b mod 8) * (G / 8) + b / 8,
// which gives every XCD (and its L2) one contiguous band of tiles instead of
// every eighth tile.
#include "../../include/tg.h"
#include "tg_internal.h"

namespace tg {
namespace {

constexpr int NXCD = 8;

struct BView {
  const uint8_t* rgba;     // [H][W][4]
  const float* depth;      // [H][W]
  const uint8_t* mask;     // [H][W]
  const float* normal;     // [H][W][3]
  float R[9], t[3];
  float fx, fy, cx, cy, znear;
  int32_t W, H;
};

struct BlendArgs {
  BView v[TG_BLEND_MAX_VIEWS];
  int32_t n_views;
  float delta;
  float R[9], t[3];          // novel camera
  float fx, fy, cx, cy;
  int32_t W, H, tiles_x, n_tiles;
  const float* z_fused;      // [H][W]
  float* rgb;                // [3][H][W]
  float* wsum;               // [H][W]
};

// XCD-aware tile of workgroup b (the grid is a multiple of NXCD)
__device__ __forceinline__ int xcd_tile(int b, int grid) {
  return (b % NXCD) * (grid / NXCD) + b / NXCD;
}

__global__ void __launch_bounds__(256) k_blend_views(BlendArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= a.n_tiles) return;
  const int tid = threadIdx.x;
  const int i = (tile % a.tiles_x) * 16 + (tid & 15);
  const int j = (tile / a.tiles_x) * 16 + (tid >> 4);
  if (i >= a.W || j >= a.H) return;
  const int64_t P = (int64_t)a.W * a.H;
  const int64_t p = (int64_t)j * a.W + i;
  const double z = (double)a.z_fused[p];
  double out0 = 0.0, out1 = 0.0, out2 = 0.0, ws = 0.0;
  if (z > 0.0 && !isinf(z)) {
    // Eq. 6: the novel pixel's point and ray in the world frame
    const double pn0 = (((double)i + 0.5) - (double)a.cx) / (double)a.fx * z;
    const double pn1 = (((double)j + 0.5) - (double)a.cy) / (double)a.fy * z;
    const double pn2 = z;
    const double pl = sqrt((pn0 * pn0 + pn1 * pn1) + pn2 * pn2);
    const double rc0 = pn0 / pl, rc1 = pn1 / pl, rc2 = pn2 / pl;
    const double tn0 = a.t[0], tn1 = a.t[1], tn2 = a.t[2];
    double X[3], r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double R0 = a.R[c], R1 = a.R[3 + c], R2 = a.R[6 + c];
      double acc = 0.0;
      acc = acc + R0 * (pn0 - tn0);
      acc = acc + R1 * (pn1 - tn1);
      acc = acc + R2 * (pn2 - tn2);
      X[c] = acc;
      double ra = 0.0;
      ra = ra + R0 * rc0;
      ra = ra + R1 * rc1;
      ra = ra + R2 * rc2;
      r[c] = ra;
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (int k = 0; k < a.n_views; ++k) {
      const BView& V = a.v[k];
      double xc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        xc[c] = (((double)V.R[3 * c] * X[0] + (double)V.R[3 * c + 1] * X[1]) + (double)V.R[3 * c + 2] * X[2]) +
                (double)V.t[c];
      if (!(xc[2] > (double)V.znear)) continue;
      const double u = ((double)V.fx * xc[0]) / xc[2] + (double)V.cx;
      const double w = ((double)V.fy * xc[1]) / xc[2] + (double)V.cy;
      // Eq. 7: bilinear taps between the pixel centres around (u, w)
      const double su = u - 0.5, sw = w - 0.5;
      const double Wm1 = (double)V.W - 1.0, Hm1 = (double)V.H - 1.0;
      if (!(su >= 0.0 && su <= Wm1 && sw >= 0.0 && sw <= Hm1)) continue;
      const double fu = fmin(floor(su), fmax((double)V.W - 2.0, 0.0));
      const double fw = fmin(floor(sw), fmax((double)V.H - 2.0, 0.0));
      const int i0 = (int)fu, j0 = (int)fw;
      const int i1 = min(i0 + 1, V.W - 1), j1 = min(j0 + 1, V.H - 1);
      const double ta = su - fu, tb = sw - fw;
      const double w00 = (1.0 - ta) * (1.0 - tb), w10 = ta * (1.0 - tb), w01 = (1.0 - ta) * tb, w11 = ta * tb;
      const int64_t p00 = (int64_t)j0 * V.W + i0, p10 = (int64_t)j0 * V.W + i1;
      const int64_t p01 = (int64_t)j1 * V.W + i0, p11 = (int64_t)j1 * V.W + i1;
      auto interp = [&](double f00, double f10, double f01, double f11) {
        return ((w00 * f00 + w10 * f10) + w01 * f01) + w11 * f11;
      };
      const double m = interp(V.mask[p00] ? 1.0 : 0.0, V.mask[p10] ? 1.0 : 0.0, V.mask[p01] ? 1.0 : 0.0,
                              V.mask[p11] ? 1.0 : 0.0);
      if (!(m > 0.0)) continue;
      const double zi = interp(V.depth[p00], V.depth[p10], V.depth[p01], V.depth[p11]);
      // Eq. 9
      if (!(fabs(xc[2] - zi) < (double)a.delta)) continue;
      double n[3];
#pragma unroll
      for (int q = 0; q < 3; ++q)
        n[q] = interp(V.normal[3 * p00 + q], V.normal[3 * p10 + q], V.normal[3 * p01 + q], V.normal[3 * p11 + q]);
      const double nl = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
      if (!(nl > 0.0)) continue;
      const double cosv = -((r[0] * n[0] + r[1] * n[1]) + r[2] * n[2]) / nl;
      if (!(cosv > 0.0)) continue;
      const double dist = sqrt((xc[0] * xc[0] + xc[1] * xc[1]) + xc[2] * xc[2]);
      // Eq. 8
      const double wt = (m * cosv) / dist;
      const uchar4 c00 = *reinterpret_cast<const uchar4*>(V.rgba + 4 * p00);
      const uchar4 c10 = *reinterpret_cast<const uchar4*>(V.rgba + 4 * p10);
      const uchar4 c01 = *reinterpret_cast<const uchar4*>(V.rgba + 4 * p01);
      const uchar4 c11 = *reinterpret_cast<const uchar4*>(V.rgba + 4 * p11);
      acc0 = acc0 + wt * (interp(c00.x, c10.x, c01.x, c11.x) / 255.0);
      acc1 = acc1 + wt * (interp(c00.y, c10.y, c01.y, c11.y) / 255.0);
      acc2 = acc2 + wt * (interp(c00.z, c10.z, c01.z, c11.z) / 255.0);
      ws = ws + wt;
    }
    if (ws > 0.0) {
      // Eq. 10
      out0 = acc0 / ws;
      out1 = acc1 / ws;
      out2 = acc2 / ws;
    } else {
      ws = 0.0;
    }
  }
  a.rgb[p] = (float)out0;
  a.rgb[P + p] = (float)out1;
  a.rgb[2 * P + p] = (float)out2;
  a.wsum[p] = (float)ws;
}

struct NormalArgs {
  float R[9];
  float fx, fy, cx, cy;
  int32_t W, H, tiles_x, n_tiles;
  const float* depth;
  float* normal;
};

__global__ void __launch_bounds__(256) k_normals(NormalArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= a.n_tiles) return;
  const int tid = threadIdx.x;
  const int i = (tile % a.tiles_x) * 16 + (tid & 15);
  const int j = (tile / a.tiles_x) * 16 + (tid >> 4);
  if (i >= a.W || j >= a.H) return;
  const int64_t p = (int64_t)j * a.W + i;
  double o0 = 0.0, o1 = 0.0, o2 = 0.0;
  if (i >= 1 && j >= 1 && i <= a.W - 2 && j <= a.H - 2) {
    const double zc = a.depth[p], zl = a.depth[p - 1], zr = a.depth[p + 1], zu = a.depth[p - a.W],
                 zd = a.depth[p + a.W];
    if (zc > 0.0 && zl > 0.0 && zr > 0.0 && zu > 0.0 && zd > 0.0) {
      const double fx = a.fx, fy = a.fy, cx = a.cx, cy = a.cy;
      auto px = [&](int c, double zz) { return (((double)c + 0.5) - cx) / fx * zz; };
      auto py = [&](int c, double zz) { return (((double)c + 0.5) - cy) / fy * zz; };
      const double pc0 = px(i, zc), pc1 = py(j, zc), pc2 = zc;
      const double dx0 = px(i + 1, zr) - px(i - 1, zl);
      const double dx1 = py(j, zr) - py(j, zl);
      const double dx2 = zr - zl;
      const double dy0 = px(i, zd) - px(i, zu);
      const double dy1 = py(j + 1, zd) - py(j - 1, zu);
      const double dy2 = zd - zu;
      const double c0 = dx1 * dy2 - dx2 * dy1, c1 = dx2 * dy0 - dx0 * dy2, c2 = dx0 * dy1 - dx1 * dy0;
      const double len = sqrt((c0 * c0 + c1 * c1) + c2 * c2);
      if (len > 0.0) {
        const double side = (c0 * pc0 + c1 * pc1) + c2 * pc2;
        const double sgn = side > 0.0 ? -1.0 : 1.0;
        const double n0 = sgn * c0 / len, n1 = sgn * c1 / len, n2 = sgn * c2 / len;
        double acc;
        acc = 0.0; acc = acc + (double)a.R[0] * n0; acc = acc + (double)a.R[3] * n1; acc = acc + (double)a.R[6] * n2;
        o0 = acc;
        acc = 0.0; acc = acc + (double)a.R[1] * n0; acc = acc + (double)a.R[4] * n1; acc = acc + (double)a.R[7] * n2;
        o1 = acc;
        acc = 0.0; acc = acc + (double)a.R[2] * n0; acc = acc + (double)a.R[5] * n1; acc = acc + (double)a.R[8] * n2;
        o2 = acc;
      }
    }
  }
  a.normal[3 * p] = (float)o0;
  a.normal[3 * p + 1] = (float)o1;
  a.normal[3 * p + 2] = (float)o2;
}

int grid_of(int n_tiles) { return (n_tiles + NXCD - 1) / NXCD * NXCD; }

struct DevGuard {
  int prev = -1;
  bool changed = false;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~DevGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

}  // namespace

int ctx_device(const tg_ctx* c);

}  // namespace tg

extern "C" {

tg_status tg_depth_normals(tg_ctx* ctx, const tg_camera* cam, const float* depth, float* normal, void* stream) {
  if (!ctx || !cam || !depth || !normal || cam->width <= 0 || cam->height <= 0) return TG_ERR_INVALID;
  tg::NormalArgs a{};
  for (int e = 0; e < 9; ++e) a.R[e] = cam->R[e];
  a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy;
  a.W = cam->width;
  a.H = cam->height;
  a.tiles_x = (a.W + 15) / 16;
  const int64_t nt = (int64_t)a.tiles_x * ((a.H + 15) / 16);
  if (nt >= ((int64_t)1 << 30)) return TG_ERR_INVALID;
  a.n_tiles = (int32_t)nt;
  a.depth = depth;
  a.normal = normal;
  tg::DevGuard guard(tg::ctx_device(ctx));
  hipLaunchKernelGGL(tg::k_normals, dim3(tg::grid_of(a.n_tiles)), dim3(256), 0, static_cast<hipStream_t>(stream), a);
  return hipGetLastError() == hipSuccess ? TG_OK : TG_ERR_HIP;
}

tg_status tg_blend_views(tg_ctx* ctx, const tg_blend_view* views, int32_t n_views, const tg_camera* novel,
                         const float* z_fused, float delta, float* out_rgb, float* out_wsum, void* stream) {
  if (!ctx || !views || !novel || !z_fused || !out_rgb || !out_wsum || n_views < 0 ||
      n_views > TG_BLEND_MAX_VIEWS || novel->width <= 0 || novel->height <= 0 || !(delta > 0.0f))
    return TG_ERR_INVALID;
  tg::BlendArgs a{};
  for (int k = 0; k < n_views; ++k) {
    const tg_blend_view& s = views[k];
    if (!s.rgba || !s.depth || !s.mask || !s.normal || s.cam.width <= 0 || s.cam.height <= 0) return TG_ERR_INVALID;
    if ((reinterpret_cast<uintptr_t>(s.rgba) & 3u) != 0) return TG_ERR_INVALID;
    tg::BView& v = a.v[k];
    v.rgba = s.rgba;
    v.depth = s.depth;
    v.mask = s.mask;
    v.normal = s.normal;
    for (int e = 0; e < 9; ++e) v.R[e] = s.cam.R[e];
    for (int e = 0; e < 3; ++e) v.t[e] = s.cam.t[e];
    v.fx = s.cam.fx; v.fy = s.cam.fy; v.cx = s.cam.cx; v.cy = s.cam.cy; v.znear = s.cam.znear;
    v.W = s.cam.width;
    v.H = s.cam.height;
  }
  a.n_views = n_views;
  a.delta = delta;
  for (int e = 0; e < 9; ++e) a.R[e] = novel->R[e];
  for (int e = 0; e < 3; ++e) a.t[e] = novel->t[e];
  a.fx = novel->fx; a.fy = novel->fy; a.cx = novel->cx; a.cy = novel->cy;
  a.W = novel->width;
  a.H = novel->height;
  a.tiles_x = (a.W + 15) / 16;
  const int64_t nt = (int64_t)a.tiles_x * ((a.H + 15) / 16);
  if (nt >= ((int64_t)1 << 30)) return TG_ERR_INVALID;
  a.n_tiles = (int32_t)nt;
  a.z_fused = z_fused;
  a.rgb = out_rgb;
  a.wsum = out_wsum;
  tg::DevGuard guard(tg::ctx_device(ctx));
  hipLaunchKernelGGL(tg::k_blend_views, dim3(tg::grid_of(a.n_tiles)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     a);
  return hipGetLastError() == hipSuccess ? TG_OK : TG_ERR_HIP;
}

}  // extern "C"
