// project.hip -- step 1 of the rasterizer: per-Gaussian projection (gfx950).
//
// One lane per Gaussian, structure-of-arrays loads (each of the 11 input
// streams is read with unit stride, so every wave issues fully coalesced
// 256-byte reads); a workgroup covers 256 aligned indices of the batch's
// padded Gaussian index space, hence one request.  The kernel does two
// things per Gaussian:
//
//  * the float32 "binning spec": view transform, quaternion rotation,
//    Sigma3D, EWA Sigma2D = (J W) Sigma3D (J W)^T, the 0.3 px^2 dilation,
//    largest eigenvalue, r = ceil(3 sqrt(lambda)), tile rectangle and depth
//    key.  Every operation is a separately rounded IEEE single operation in
//    a fixed order (the file is built with -ffp-contract=off; division and
//    sqrt are correctly rounded on gfx950), so culling, rectangles and keys
//    are reproducible bit for bit by any IEEE implementation of the same
//    sequence;
//  * the continuous 2D state in FP64: the mean (u, v), the conic, and the
//    tile-independent factors of the blend's exponent.  With Sigma' the
//    dilated 2D covariance (entries a, b, c) the quadratic form completes to
//      d^T Sigma'^-1 d = (c / det) (dx - (b / c) dy)^2 + dy^2 / c,
//    so that, in units of log2(e), the exponent is -(z1^2 + z2^2) with
//    z1 = s (dx + k dy), z2 = r dy, s = sqrt(log2(e) c / (2 det)),
//    k = -b / c, r = sqrt(log2(e) / (2 c)); the factors come straight from
//    Sigma' (no cancellation in det(Sigma'^-1) for elongated Gaussians).
//    The alpha >= 1/255 ellipse d^T Sigma'^-1 d <= 2 ln(255 o) has the
//    half-extents sqrt(2 ln(255 o) a) and sqrt(2 ln(255 o) c).  The render
//    forms pixel offsets relative to its tile from the FP64 mean, which keeps
//    them accurate to ~1e-7 px at any image size.  The kernel is HBM-bound,
//    so the FP64 arithmetic (full rate on CDNA4's vector FP64 units) is free.
#include "tg_internal.h"

namespace tg {
namespace {

struct Rect { int x0, y0, x1, y1; bool ok; uint32_t key; };

// float32 binning spec (see header comment); returns ok = false when culled
__device__ __forceinline__ Rect spec_f32(const CamArgs& c, float mx, float my, float mz,
                                         float sx, float sy, float sz,
                                         float qw, float qx, float qy, float qz) {
  Rect out{0, 0, -1, -1, false, 0u};
  const float vx = ((c.R[0] * mx + c.R[1] * my) + c.R[2] * mz) + c.t[0];
  const float vy = ((c.R[3] * mx + c.R[4] * my) + c.R[5] * mz) + c.t[1];
  const float vz = ((c.R[6] * mx + c.R[7] * my) + c.R[8] * mz) + c.t[2];
  if (!(vz > c.znear)) return out;
  const float u = (c.fx * vx) / vz + c.cx;
  const float v = (c.fy * vy) / vz + c.cy;
  const float qn = sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  if (!(qn > 0.0f)) return out;
  const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  // rotation rows of the unit quaternion
  const float r00 = 1.0f - 2.0f * (y * y + z * z), r01 = 2.0f * (x * y - w * z), r02 = 2.0f * (x * z + w * y);
  const float r10 = 2.0f * (x * y + w * z), r11 = 1.0f - 2.0f * (x * x + z * z), r12 = 2.0f * (y * z - w * x);
  const float r20 = 2.0f * (x * z - w * y), r21 = 2.0f * (y * z + w * x), r22 = 1.0f - 2.0f * (x * x + y * y);
  // M = R diag(s)
  const float m00 = r00 * sx, m01 = r01 * sy, m02 = r02 * sz;
  const float m10 = r10 * sx, m11 = r11 * sy, m12 = r12 * sz;
  const float m20 = r20 * sx, m21 = r21 * sy, m22 = r22 * sz;
  // Sigma3D = M M^T (symmetric, entries as rows i, j)
  const float c00 = (m00 * m00 + m01 * m01) + m02 * m02;
  const float c01 = (m00 * m10 + m01 * m11) + m02 * m12;
  const float c02 = (m00 * m20 + m01 * m21) + m02 * m22;
  const float c10 = (m10 * m00 + m11 * m01) + m12 * m02;
  const float c11 = (m10 * m10 + m11 * m11) + m12 * m12;
  const float c12 = (m10 * m20 + m11 * m21) + m12 * m22;
  const float c20 = (m20 * m00 + m21 * m01) + m22 * m02;
  const float c21 = (m20 * m10 + m21 * m11) + m22 * m12;
  const float c22 = (m20 * m20 + m21 * m21) + m22 * m22;
  // perspective Jacobian and A = J W (two rows)
  const float vz2 = vz * vz;
  const float ja = c.fx / vz;
  const float jb = -((c.fx * vx) / vz2);
  const float jc = c.fy / vz;
  const float jd = -((c.fy * vy) / vz2);
  const float a00 = ja * c.R[0] + jb * c.R[6], a01 = ja * c.R[1] + jb * c.R[7], a02 = ja * c.R[2] + jb * c.R[8];
  const float a10 = jc * c.R[3] + jd * c.R[6], a11 = jc * c.R[4] + jd * c.R[7], a12 = jc * c.R[5] + jd * c.R[8];
  // B = A Sigma3D
  const float b00 = (a00 * c00 + a01 * c10) + a02 * c20;
  const float b01 = (a00 * c01 + a01 * c11) + a02 * c21;
  const float b02 = (a00 * c02 + a01 * c12) + a02 * c22;
  const float b10 = (a10 * c00 + a11 * c10) + a12 * c20;
  const float b11 = (a10 * c01 + a11 * c11) + a12 * c21;
  const float b12 = (a10 * c02 + a11 * c12) + a12 * c22;
  // Sigma2D = B A^T, upper triangle; dilation on the diagonal
  const float sa = ((b00 * a00 + b01 * a01) + b02 * a02) + 0.3f;
  const float sb = (b00 * a10 + b01 * a11) + b02 * a12;
  const float sc = ((b10 * a10 + b11 * a11) + b12 * a12) + 0.3f;
  const float det = sa * sc - sb * sb;
  if (!(det > 0.0f)) return out;
  const float mid = 0.5f * (sa + sc);
  const float disc = mid * mid - det;
  const float lam = mid + sqrtf(disc > 0.0f ? disc : 0.0f);
  const float rad = ceilf(3.0f * sqrtf(lam));
  const float lastx = (float)(c.tiles_x - 1), lasty = (float)(c.tiles_y - 1);
  const float fx0 = floorf((u - rad) / 16.0f), fx1 = floorf((u + rad) / 16.0f);
  const float fy0 = floorf((v - rad) / 16.0f), fy1 = floorf((v + rad) / 16.0f);
  if (!(fx1 >= 0.0f && fx0 <= lastx && fy1 >= 0.0f && fy0 <= lasty)) return out;
  out.x0 = (int)fmaxf(fx0, 0.0f);
  out.x1 = (int)fminf(fx1, lastx);
  out.y0 = (int)fmaxf(fy0, 0.0f);
  out.y1 = (int)fminf(fy1, lasty);
  out.key = __float_as_uint(vz);
  out.ok = true;
  return out;
}

// The 11 input values of one Gaussian.
struct GaussIn {
  float mx, my, mz, sx, sy, sz, qw, qx, qy, qz, op;
};

// Gaussian i of request q (read through a reference whose address space the
// caller fixes, so its fields are wave-uniform scalar loads).
__device__ __forceinline__ GaussIn load_gauss(const ReqDev& q, int64_t i) {
  const int64_t n = q.n;
  GaussIn G;
  G.mx = q.mean[i]; G.my = q.mean[n + i]; G.mz = q.mean[2 * n + i];
  G.sx = q.scale[i]; G.sy = q.scale[n + i]; G.sz = q.scale[2 * n + i];
  G.qw = q.quat[i]; G.qx = q.quat[n + i]; G.qy = q.quat[2 * n + i]; G.qz = q.quat[3 * n + i];
  G.op = q.opacity[i];
  return G;
}

// Project one Gaussian into camera c; the state goes to global index gi.
__device__ __forceinline__ void project_store(const BatchArgs& a, const CamArgs& c, const GaussIn& G, int64_t gi) {
  const float mx = G.mx, my = G.my, mz = G.mz, sx = G.sx, sy = G.sy, sz = G.sz;
  const float qw = G.qw, qx = G.qx, qy = G.qy, qz = G.qz, op = G.op;
  const Rect rc = spec_f32(c, mx, my, mz, sx, sy, sz, qw, qx, qy, qz);

  uint2 rect = make_uint2(1u, 0u);   // empty
  double2 xy = make_double2(0.0, 0.0);
  float4 co = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 wq = make_float4(0.f, 0.f, 0.f, -INFINITY);
  float4 ext = make_float4(-INFINITY, -INFINITY, op, 0.f);
  if (rc.ok) {
    // continuous state in FP64
    const double X = mx, Y = my, Z = mz;
    const double tx = (double)c.R[0] * X + (double)c.R[1] * Y + (double)c.R[2] * Z + (double)c.t[0];
    const double ty = (double)c.R[3] * X + (double)c.R[4] * Y + (double)c.R[5] * Z + (double)c.t[1];
    const double tz = (double)c.R[6] * X + (double)c.R[7] * Y + (double)c.R[8] * Z + (double)c.t[2];
    const double fx = c.fx, fy = c.fy;
    const double itz = 1.0 / tz;
    xy.x = fx * tx * itz + (double)c.cx;
    xy.y = fy * ty * itz + (double)c.cy;
    const double dw = qw, dx = qx, dy = qy, dz = qz;
    const double inq = 1.0 / sqrt(dw * dw + dx * dx + dy * dy + dz * dz);
    const double w = dw * inq, x = dx * inq, y = dy * inq, z = dz * inq;
    double Rq[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                       {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                       {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double s2[3] = {(double)sx * sx, (double)sy * sy, (double)sz * sz};
    double S[3][3];
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k)
        S[p][k] = Rq[p][0] * s2[0] * Rq[k][0] + Rq[p][1] * s2[1] * Rq[k][1] + Rq[p][2] * s2[2] * Rq[k][2];
    const double j00 = fx * itz, j02 = -fx * tx * itz * itz, j11 = fy * itz, j12 = -fy * ty * itz * itz;
    double A[2][3];
    for (int k = 0; k < 3; ++k) {
      A[0][k] = j00 * (double)c.R[k] + j02 * (double)c.R[6 + k];
      A[1][k] = j11 * (double)c.R[3 + k] + j12 * (double)c.R[6 + k];
    }
    double AS[2][3];
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 3; ++k) AS[p][k] = A[p][0] * S[0][k] + A[p][1] * S[1][k] + A[p][2] * S[2][k];
    const double sa = AS[0][0] * A[0][0] + AS[0][1] * A[0][1] + AS[0][2] * A[0][2] + 0.3;
    const double sb = AS[0][0] * A[1][0] + AS[0][1] * A[1][1] + AS[0][2] * A[1][2];
    const double sc = AS[1][0] * A[1][0] + AS[1][1] * A[1][1] + AS[1][2] * A[1][2] + 0.3;
    const double det = sa * sc - sb * sb;
    if (det > 0.0) {
      const double idet = 1.0 / det, isc = 1.0 / sc;
      co = make_float4((float)(sc * idet), (float)(-sb * idet), (float)(sa * idet), op);
      constexpr double L2E = 1.4426950408889634;
      const double sw = sqrt(0.5 * L2E * sc * idet);
      wq = make_float4((float)sw, (float)(sw * (-sb * isc)), (float)sqrt(0.5 * L2E * isc), log2f(op));
      if (op * 255.f >= 1.f) {
        const double rho = 2.0 * (double)logf(255.f * op);
        ext.x = (float)sqrt(rho * sa);
        ext.y = (float)sqrt(rho * sc);
      }
      rect = make_uint2((uint32_t)rc.x0 | ((uint32_t)rc.x1 << 16), (uint32_t)rc.y0 | ((uint32_t)rc.y1 << 16));
    }
  }
  a.xy[gi] = xy;
  a.conic_o[gi] = co;
  a.wq[gi] = wq;
  a.ext[gi] = ext;
  a.rect[gi] = rect;
  a.depth[gi] = rc.ok ? rc.key : 0xffffffffu;
}

// TABLE: the requests come from the device table (a serving batch, the
// views of one set); a separate instantiation from the single inline
// request, so that the single render keeps its own register budget.
template <bool TABLE>
__global__ void __launch_bounds__(256) k_project(BatchArgs a) {
  const BatchHdr h = TABLE ? *a.hdr_dev : a.hdr;
  // clear the per-tile key counters that the binning accumulates into
  for (int t = blockIdx.x * 256 + threadIdx.x; t < h.n_tiles; t += gridDim.x * 256) a.tile_count[t] = 0;
  const int64_t g0 = (int64_t)blockIdx.x * 256;       // 256-aligned: one request per workgroup
  const int64_t gi = g0 + threadIdx.x;
  if (TABLE) {                                   // a batch's table in global memory
    const int r = req_of_gauss(a, h, g0);
    if (r < 0) return;
    const ReqDev& q = a.table[r];
    // a sharing request reads its source's state; a covered view is
    // projected by the workgroups of the set's first view
    if (q.src != 0 || q.covered) return;
    const int64_t i = gi - q.g_off;
    if (i >= q.n) return;
    const GaussIn G = load_gauss(q, i);          // read once for every view of the set
    const int nv = q.extra_views;
    for (int v = 0; v <= nv; ++v) {
      const ReqDev& qv = a.table[r + v];
      project_store(a, qv.cam, G, qv.g_off + i);
    }
  } else {                                       // one request in the kernel arguments
    if (g0 >= h.g_end) return;
    const int64_t i = gi - a.one.g_off;
    if (i < a.one.n) project_store(a, a.one.cam, load_gauss(a.one, i), gi);
  }
}

}  // namespace

hipError_t launch_project(const BatchArgs& a, int64_t grid_gauss, hipStream_t s) {
  const int64_t blocks = (grid_gauss + 255) / 256;
  const int grid = (int)(blocks > 0 ? blocks : 1);
  if (a.table) hipLaunchKernelGGL(k_project<true>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_project<false>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tg
