// tgo.cpp -- plain, slow, brute-force CPU oracle for the latent Gaussian
// rasterizer R_G of Tele-Aloha (arXiv 2405.14866, §4.2: per-pixel latent
// Gaussians {x, f, s, alpha} splatted into a novel view, F = R_G({G}, Pi)).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, header, table or constant
// generator with the HIP path.
//
// The paper does not restate how the rasterizer works (§4.2 only cites the
// differentiable 3D Gaussian splatting rasterizer), so the conventions below
// are the project's stated reading of that rasterizer:
//   * EWA splatting: Sigma2D = J W Sigma3D W^T J^T, Sigma3D = R S S^T R^T;
//   * 0.3 px^2 added to the diagonal of Sigma2D ("dilation");
//   * radius r = ceil(3 sqrt(lambda_max)); the 16x16-tile rectangle
//     [floor((u-r)/16), floor((u+r)/16)] (clamped) is the support;
//   * per pixel, Gaussians of the pixel's tile in ascending (view depth,
//     index) order; alpha = min(0.99, o exp(-d^T Sigma'^-1 d / 2));
//     alpha < 1/255 is skipped; a Gaussian that would take the transmittance
//     below 1e-4 is not blended and ends the pixel;
//   * F = sum_i alpha_i T_i f_i + T_final bg, alpha_out = 1 - T_final.
//
// Two precisions:
//   * every discrete decision that the GPU must reproduce bit for bit (cull,
//     tile rectangle, depth key and therefore tile lists and their order) is
//     taken from a float32 "binning spec" with a fixed operation order and no
//     contraction (build with -ffp-contract=off, no fast-math);
//   * every continuous value (2D mean, conic, alpha, T, F, gradients) is FP64.
//
// Near the two thresholds (alpha vs 1/255, T' vs 1e-4) an FP32 renderer may
// legitimately take the other branch.  The oracle flags such decisions and
// can evaluate the pixel under both branches (tgo_pixel_variants), and its
// backward can differentiate a pixel under a chosen branch.
//
// Parity pins: see tests/test_oracle_pins.py (closed forms, invariants,
// brute force on tiny scenes, finite differences for the backward).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

// Mutation hook for the test-suite: building with -DTGO_PLANT=n swaps in a
// deliberately wrong expression at site n, so the tests can show that the
// pins catch it.  The default build (TGO_PLANT = 0) is the oracle.
#ifndef TGO_PLANT
#define TGO_PLANT 0
#endif
#define PLANT(n, good, bad) (TGO_PLANT == (n) ? (bad) : (good))

namespace {

constexpr int TILE = 16;
constexpr double ALPHA_MIN = 1.0 / 255.0;
constexpr double ALPHA_MAX = 0.99;
constexpr double T_MIN = 1e-4;
// Relative half-widths of the bands in which an FP32 renderer may decide a
// threshold differently from FP64 (see the reading of the paper in the docs).
constexpr double ALPHA_BAND = 5e-5;
constexpr double T_BAND = 3e-4;

struct CamD {
  double R[9], t[3], fx, fy, cx, cy, znear;
  int W, H;
};
struct CamF {
  float R[9], t[3], fx, fy, cx, cy, znear;
  int W, H;
};

CamD cam_from(const double* c) {
  CamD k;
  for (int i = 0; i < 9; ++i) k.R[i] = c[i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[9 + i];
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
  k.W = (int)c[16]; k.H = (int)c[17]; k.znear = c[18];
  return k;
}
CamF to_f32(const CamD& d) {
  CamF f;
  for (int i = 0; i < 9; ++i) f.R[i] = (float)d.R[i];
  for (int i = 0; i < 3; ++i) f.t[i] = (float)d.t[i];
  f.fx = (float)d.fx; f.fy = (float)d.fy; f.cx = (float)d.cx; f.cy = (float)d.cy;
  f.znear = (float)d.znear; f.W = d.W; f.H = d.H;
  return f;
}

// ------------------------------------------------------------------ spec32
// The float32 binning spec.  Every line is one IEEE single operation, in the
// order written (the build forbids contraction and fast-math).
struct Spec {
  int culled;
  int x0, y0, x1, y1;
  uint32_t key;
};

Spec spec32(const CamF& c, const float mu[3], const float s[3], const float q[4]) {
  Spec o{1, 0, 0, -1, -1, 0u};
  // (a) camera-space position t = W mu + t_cam
  float tx = ((c.R[0] * mu[0] + c.R[1] * mu[1]) + c.R[2] * mu[2]) + c.t[0];
  float ty = ((c.R[3] * mu[0] + c.R[4] * mu[1]) + c.R[5] * mu[2]) + c.t[1];
  float tz = ((c.R[6] * mu[0] + c.R[7] * mu[1]) + c.R[8] * mu[2]) + c.t[2];
  // (b) near-plane cull
  if (!(tz > c.znear)) return o;
  // (c) pinhole projection of the mean
  float u = (c.fx * tx) / tz + c.cx;
  float v = (c.fy * ty) / tz + c.cy;
  // (d) normalise the quaternion (w, x, y, z)
  float nq = std::sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  if (!(nq > 0.0f)) return o;
  float w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
  // (e) rotation matrix of the unit quaternion
  float r[9];
  r[0] = 1.0f - 2.0f * (y * y + z * z);
  r[1] = 2.0f * (x * y - w * z);
  r[2] = 2.0f * (x * z + w * y);
  r[3] = 2.0f * (x * y + w * z);
  r[4] = 1.0f - 2.0f * (x * x + z * z);
  r[5] = 2.0f * (y * z - w * x);
  r[6] = 2.0f * (x * z - w * y);
  r[7] = 2.0f * (y * z + w * x);
  r[8] = 1.0f - 2.0f * (x * x + y * y);
  // (f) M = R diag(s), Sigma3D = M M^T
  float M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = r[3 * i + j] * s[j];
  float S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = (M[3 * i] * M[3 * j] + M[3 * i + 1] * M[3 * j + 1]) + M[3 * i + 2] * M[3 * j + 2];
  // (g) perspective Jacobian rows and A = J W (2x3)
  float tz2 = tz * tz;
  float j00 = c.fx / tz;
  float j02 = -((c.fx * tx) / tz2);
  float j11 = c.fy / tz;
  float j12 = -((c.fy * ty) / tz2);
  float A[6];
  for (int k = 0; k < 3; ++k) {
    A[k] = j00 * c.R[k] + j02 * c.R[6 + k];
    A[3 + k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
  }
  // Sigma2D = (A Sigma3D) A^T
  float B[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      B[3 * i + j] = (A[3 * i] * S[j] + A[3 * i + 1] * S[3 + j]) + A[3 * i + 2] * S[6 + j];
  float s00 = (B[0] * A[0] + B[1] * A[1]) + B[2] * A[2];
  float s01 = (B[0] * A[3] + B[1] * A[4]) + B[2] * A[5];
  float s11 = (B[3] * A[3] + B[4] * A[4]) + B[5] * A[5];
  // (h) dilation and determinant
  float a = s00 + 0.3f;
  float b = s01;
  float cc = s11 + 0.3f;
  float det = a * cc - b * b;
  if (!(det > 0.0f)) return o;
  // (i) largest eigenvalue and the 3-sigma radius in pixels
  float m = 0.5f * (a + cc);
  float disc = m * m - det;
  float lam = m + std::sqrt(disc > 0.0f ? disc : 0.0f);
  float rad = std::ceil(PLANT(7, 3.0f, 2.0f) * std::sqrt(lam));
  // (j) tile rectangle (inclusive), empty when it misses the image
  const float tmx = (float)((c.W + TILE - 1) / TILE - 1);
  const float tmy = (float)((c.H + TILE - 1) / TILE - 1);
  float fx0 = std::floor((u - rad) / 16.0f);
  float fx1 = std::floor((u + rad) / 16.0f);
  float fy0 = std::floor((v - rad) / 16.0f);
  float fy1 = std::floor((v + rad) / 16.0f);
  if (!(fx1 >= 0.0f && fx0 <= tmx && fy1 >= 0.0f && fy0 <= tmy)) return o;
  o.x0 = (int)std::max(fx0, 0.0f);
  o.x1 = (int)std::min(fx1, tmx);
  o.y0 = (int)std::max(fy0, 0.0f);
  o.y1 = (int)std::min(fy1, tmy);
  // (k) depth key: IEEE bits of the (positive) view depth
  std::memcpy(&o.key, &tz, 4);
  o.culled = 0;
  return o;
}

// ------------------------------------------------------------- FP64 model
struct Proj {          // continuous per-Gaussian 2D state, FP64
  double u, v;         // projected mean, pixels
  double A, B, C;      // conic = inverse of the dilated 2D covariance
  double o;            // opacity
  double tx, ty, tz;   // camera-space mean
};

struct Gauss {         // raw FP64 inputs of one Gaussian
  double mu[3], s[3], q[4], o;
};

// Returns false when the FP64 model itself degenerates (det <= 0 or tz <= 0);
// the float32 spec decides culling, this is only a guard.
bool project64(const CamD& c, const Gauss& g, Proj& p, double Sig3[9], double Amat[6],
               double r[9], double qn[4]) {
  double tx = c.R[0] * g.mu[0] + c.R[1] * g.mu[1] + c.R[2] * g.mu[2] + c.t[0];
  double ty = c.R[3] * g.mu[0] + c.R[4] * g.mu[1] + c.R[5] * g.mu[2] + c.t[1];
  double tz = c.R[6] * g.mu[0] + c.R[7] * g.mu[1] + c.R[8] * g.mu[2] + c.t[2];
  p.tx = tx; p.ty = ty; p.tz = tz;
  if (!(tz > 0.0)) return false;
  p.u = c.fx * tx / tz + c.cx;
  p.v = c.fy * ty / tz + c.cy;
  double nq = std::sqrt(g.q[0] * g.q[0] + g.q[1] * g.q[1] + g.q[2] * g.q[2] + g.q[3] * g.q[3]);
  if (!(nq > 0.0)) return false;
  double w = g.q[0] / nq, x = g.q[1] / nq, y = g.q[2] / nq, z = g.q[3] / nq;
  qn[0] = w; qn[1] = x; qn[2] = y; qn[3] = z;
  r[0] = 1 - 2 * (y * y + z * z); r[1] = PLANT(4, 2 * (x * y - w * z), 2 * (x * y + w * z));     r[2] = 2 * (x * z + w * y);
  r[3] = 2 * (x * y + w * z);     r[4] = 1 - 2 * (x * x + z * z); r[5] = 2 * (y * z - w * x);
  r[6] = 2 * (x * z - w * y);     r[7] = 2 * (y * z + w * x);     r[8] = 1 - 2 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += r[3 * i + k] * g.s[k] * g.s[k] * r[3 * j + k];
      Sig3[3 * i + j] = acc;
    }
  double J[6] = {c.fx / tz, 0.0, -c.fx * tx / (tz * tz), 0.0, c.fy / tz, -c.fy * ty / (tz * tz)};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += J[3 * i + k] * PLANT(3, c.R[3 * k + j], c.R[3 * j + k]);
      Amat[3 * i + j] = acc;
    }
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += Amat[3 * i + k] * Sig3[3 * k + l] * Amat[3 * j + l];
      S2[2 * i + j] = acc;
    }
  double a = S2[0] + PLANT(2, 0.3, 0.0), b = S2[1], cc = S2[3] + PLANT(2, 0.3, 0.0);
  double det = a * cc - b * b;
  if (!(det > 0.0)) return false;
  p.A = cc / det;
  p.B = PLANT(1, -b / det, b / det);
  p.C = a / det;
  p.o = g.o;
  return true;
}

// ----------------------------------------------------------------- context
struct Ctx {
  int64_t n = 0;
  int c = 0;
  CamD cam{};
  CamF camf{};
  int tiles_x = 0, tiles_y = 0;
  std::vector<Gauss> g;
  std::vector<double> feat;      // [n][c]
  std::vector<Spec> spec;
  std::vector<Proj> proj;
  std::vector<int64_t> tile_start;  // [tiles + 1]
  std::vector<int32_t> list;        // [K] Gaussian indices, per tile in (key, index) order
  int nthreads = 1;
};

Spec spec_of(const Ctx& k, const Gauss& g) {
  float mu[3] = {(float)g.mu[0], (float)g.mu[1], (float)g.mu[2]};
  float s[3] = {(float)g.s[0], (float)g.s[1], (float)g.s[2]};
  float q[4] = {(float)g.q[0], (float)g.q[1], (float)g.q[2], (float)g.q[3]};
  return spec32(k.camf, mu, s, q);
}

template <class F>
void parallel_for(int64_t count, int nthreads, F&& fn) {
  if (count <= 0) return;
  int nt = std::max(1, std::min<int>(nthreads, (int)std::min<int64_t>(count, 1 << 20)));
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (;;) {
      int64_t i = next.fetch_add(1);
      if (i >= count) break;
      fn(i);
    }
  };
  if (nt == 1) { work(); return; }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(work);
  for (auto& t : th) t.join();
}

// O3: the tile lists.  For every tile, the Gaussians whose rectangle holds
// it, sorted ascending by (depth key, index).
void build_lists(Ctx& k) {
  const int64_t T = (int64_t)k.tiles_x * k.tiles_y;
  std::vector<std::vector<int32_t>> per(T);
  for (int64_t i = 0; i < k.n; ++i) {
    const Spec& s = k.spec[i];
    if (s.culled) continue;
    for (int ty = s.y0; ty <= s.y1; ++ty)
      for (int tx = s.x0; tx <= s.x1; ++tx) per[(int64_t)ty * k.tiles_x + tx].push_back((int32_t)i);
  }
  parallel_for(T, k.nthreads, [&](int64_t t) {
    std::sort(per[t].begin(), per[t].end(), [&](int32_t a, int32_t b) {
      if (PLANT(8, k.spec[a].key != k.spec[b].key, false)) return k.spec[a].key < k.spec[b].key;
      return a < b;
    });
  });
  k.tile_start.assign(T + 1, 0);
  for (int64_t t = 0; t < T; ++t) k.tile_start[t + 1] = k.tile_start[t] + (int64_t)per[t].size();
  k.list.resize(k.tile_start[T]);
  for (int64_t t = 0; t < T; ++t)
    std::copy(per[t].begin(), per[t].end(), k.list.begin() + k.tile_start[t]);
}

// ------------------------------------------------------------ pixel blend
enum Dec : uint8_t { D_SKIP_P = 1, D_SKIP_A = 2, D_BLEND = 3, D_BLEND_CLAMP = 4, D_STOP = 5 };

struct Flag { int pos; int kind; };  // kind 0: alpha band, 1: T band

struct PixelRun {
  double T = 1.0;
  int last = -1;
  bool stopped = false;
  int64_t n_eval = 0, n_contrib = 0;
  std::vector<Flag> flags;
};

// One blended Gaussian of a pixel: list position, index, alpha, the
// transmittance in front of it, the Gaussian falloff G, clamp state, offset.
struct Contrib { int pos; int32_t gi; double alpha, T, G; bool clamped; double dx, dy; };

struct BlendOpts {
  const std::vector<int>* flip = nullptr;   // list positions whose threshold decision is inverted
  std::vector<uint8_t>* dec = nullptr;      // receives the decision taken at every visited position
  std::vector<Contrib>* contrib = nullptr;  // receives every blended Gaussian
  int32_t swap_gi = -1;                     // Gaussian whose state is replaced by swap_p / swap_f
  const Proj* swap_p = nullptr;
  const double* swap_f = nullptr;
  int64_t start = 0, end = -1;              // walk list positions [start, end)
  double T0 = 1.0;                          // transmittance at `start`
};

// Blend one pixel centred at (px, py) over an ordered candidate list (O5).
// F (c values) is accumulated into, not cleared.
void blend_pixel(const Ctx& k, const Proj* proj, const int32_t* lst, int64_t len, double px,
                 double py, double* F, PixelRun& run, const BlendOpts& op = BlendOpts()) {
  double T = op.T0;
  const int64_t end = op.end < 0 ? len : std::min(len, op.end);
  for (int64_t pos = op.start; pos < end; ++pos) {
    const int32_t gi = lst[pos];
    const bool sw = gi == op.swap_gi;
    const Proj& p = (sw && op.swap_p) ? *op.swap_p : proj[gi];
    ++run.n_eval;
    const double dx = px - p.u, dy = py - p.v;
    const double P = -0.5 * (p.A * dx * dx + p.C * dy * dy) - p.B * dx * dy;
    if (P > 0.0) {
      if (op.dec) op.dec->push_back(D_SKIP_P);
      continue;
    }
    const double G = std::exp(P);
    const double raw = p.o * G;
    const bool clamped = raw > ALPHA_MAX;
    const double alpha = clamped ? ALPHA_MAX : raw;
    bool flipped = false;
    if (op.flip)
      for (int fpos : *op.flip)
        if (fpos == (int)pos) flipped = true;
    bool skip = alpha < ALPHA_MIN;
    if (std::fabs(alpha - ALPHA_MIN) <= ALPHA_BAND * ALPHA_MIN) {
      run.flags.push_back({(int)pos, 0});
      if (flipped) skip = !skip;
    }
    if (skip) {
      if (op.dec) op.dec->push_back(D_SKIP_A);
      continue;
    }
    const double Tn = T * (1.0 - alpha);
    bool stop = PLANT(5, Tn < T_MIN, T < T_MIN);
    if (std::fabs(Tn - T_MIN) <= T_BAND * T_MIN) {
      run.flags.push_back({(int)pos, 1});
      if (flipped) stop = !stop;
    }
    if (stop) {
      if (op.dec) op.dec->push_back(D_STOP);
      run.stopped = true;
      break;
    }
    if (op.dec) op.dec->push_back(clamped ? D_BLEND_CLAMP : D_BLEND);
    const double w = alpha * T;
    const double* f = (sw && op.swap_f) ? op.swap_f : &k.feat[(size_t)gi * k.c];
    for (int ch = 0; ch < k.c; ++ch) F[ch] += w * f[ch];
    if (op.contrib) op.contrib->push_back({(int)pos, gi, alpha, T, G, clamped, dx, dy});
    ++run.n_contrib;
    T = Tn;
    run.last = (int)pos;
  }
  run.T = T;
}

Ctx* make_ctx(int64_t n, int c, const double* mean, const double* scale, const double* quat,
              const double* opac, const double* feat, const double* cam, int nthreads) {
  Ctx* k = new Ctx;
  k->n = n; k->c = c;
  k->cam = cam_from(cam);
  k->camf = to_f32(k->cam);
  k->tiles_x = (k->cam.W + TILE - 1) / TILE;
  k->tiles_y = (k->cam.H + TILE - 1) / TILE;
  k->nthreads = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
  k->g.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    Gauss& g = k->g[i];
    for (int d = 0; d < 3; ++d) { g.mu[d] = mean[d * n + i]; g.s[d] = scale[d * n + i]; }
    for (int d = 0; d < 4; ++d) g.q[d] = quat[d * n + i];
    g.o = opac[i];
  }
  k->feat.assign(feat, feat + (size_t)n * c);
  k->spec.resize(n);
  k->proj.resize(n);
  parallel_for((n + 4095) / 4096, k->nthreads, [&](int64_t b) {
    int64_t e = std::min<int64_t>(n, (b + 1) * 4096);
    double S3[9], Am[6], r[9], qn[4];
    for (int64_t i = b * 4096; i < e; ++i) {
      k->spec[i] = spec_of(*k, k->g[i]);
      if (!k->spec[i].culled) {
        if (!project64(k->cam, k->g[i], k->proj[i], S3, Am, r, qn)) k->spec[i].culled = 1;
      }
    }
  });
  build_lists(*k);
  return k;
}

inline int64_t tile_of(const Ctx& k, int px, int py) {
  return (int64_t)(py / TILE) * k.tiles_x + px / TILE;
}

// ------------------------------------------------------------ backward
// Chain rule from the per-Gaussian 2D gradients (u, v, conic A/B/C,
// opacity) to the raw parameters (mean, log-scale, unnormalised quaternion,
// opacity logit), all FP64.
void chain_to_raw(const CamD& c, const Gauss& g, const double d2[6] /*du dv dA dB dC do*/,
                  double dmu[3], double dls[3], double dq[4], double& dlogit) {
  Proj p; double S3[9], Am[6], r[9], qn[4];
  for (int i = 0; i < 3; ++i) dmu[i] = dls[i] = 0;
  for (int i = 0; i < 4; ++i) dq[i] = 0;
  dlogit = 0;
  if (!project64(c, g, p, S3, Am, r, qn)) return;
  const double tx = p.tx, ty = p.ty, tz = p.tz;
  // conic -> dilated covariance Sigma' = [[a, b], [b, cc]]
  double Q[4] = {p.A, p.B, p.B, p.C};
  double GQ[4] = {d2[2], 0.5 * d2[3], 0.5 * d2[3], d2[4]};  // dL/dQ as a symmetric matrix
  double QG[4], GS[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * GQ[j] + Q[2 * i + 1] * GQ[2 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) GS[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
  // GS = dL/dSigma2D (symmetric gradient; the dilation is a constant shift)
  // dL/dSigma3D = A^T GS A ; dL/dA = 2 GS A Sigma3D
  double G3[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc += Am[3 * a + i] * GS[2 * a + b] * Am[3 * b + j];
      G3[3 * i + j] = acc;
    }
  double dA[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int b = 0; b < 2; ++b)
        for (int l = 0; l < 3; ++l) acc += GS[2 * i + b] * Am[3 * b + l] * S3[3 * l + j];
      dA[3 * i + j] = 2.0 * acc;
    }
  // A = J W  ->  dL/dJ = dL/dA W^T
  double dJ[6];
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 3; ++k) {
      double acc = 0;
      for (int j = 0; j < 3; ++j) acc += dA[3 * i + j] * c.R[3 * k + j];
      dJ[3 * i + k] = acc;
    }
  // J = [[fx/tz, 0, -fx tx/tz^2], [0, fy/tz, -fy ty/tz^2]] and (u, v)
  double dt[3] = {0, 0, 0};
  const double tz2 = tz * tz, tz3 = tz2 * tz;
  dt[0] += d2[0] * c.fx / tz;
  dt[2] += -d2[0] * c.fx * tx / tz2;
  dt[1] += d2[1] * c.fy / tz;
  dt[2] += -d2[1] * c.fy * ty / tz2;
  dt[2] += -dJ[0] * c.fx / tz2;
  dt[0] += -dJ[2] * c.fx / tz2;
  dt[2] += dJ[2] * 2.0 * c.fx * tx / tz3;
  dt[2] += -dJ[4] * c.fy / tz2;
  dt[1] += -dJ[5] * c.fy / tz2;
  dt[2] += dJ[5] * 2.0 * c.fy * ty / tz3;
  // t = W mu + t_cam
  for (int j = 0; j < 3; ++j)
    dmu[j] = PLANT(9, c.R[j] * dt[0] + c.R[3 + j] * dt[1] + c.R[6 + j] * dt[2],
                   c.R[3 * j] * dt[0] + c.R[3 * j + 1] * dt[1] + c.R[3 * j + 2] * dt[2]);
  // Sigma3D = M M^T, M = R diag(s): dL/dM = 2 G3 M
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = r[3 * i + j] * g.s[j];
  double dM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += G3[3 * i + k] * M[3 * k + j];
      dM[3 * i + j] = 2.0 * acc;
    }
  double dR[9];
  for (int j = 0; j < 3; ++j) {
    double ds = 0;
    for (int i = 0; i < 3; ++i) {
      dR[3 * i + j] = dM[3 * i + j] * g.s[j];
      ds += dM[3 * i + j] * r[3 * i + j];
    }
    dls[j] = ds * g.s[j];                    // d/dlog s = s d/ds
  }
  // rotation of the unit quaternion (w, x, y, z)
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  double dqn[4];
  dqn[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dqn[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] +
                w * dR[7] - 2 * x * dR[8]);
  dqn[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                z * dR[7] - 2 * y * dR[8]);
  dqn[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] +
                x * dR[6] + y * dR[7]);
  // normalisation q_hat = q / |q|
  const double nq = std::sqrt(g.q[0] * g.q[0] + g.q[1] * g.q[1] + g.q[2] * g.q[2] + g.q[3] * g.q[3]);
  const double dot = w * dqn[0] + x * dqn[1] + y * dqn[2] + z * dqn[3];
  for (int i = 0; i < 4; ++i) dq[i] = (dqn[i] - qn[i] * dot) / nq;
  // opacity o = sigmoid(logit)
  dlogit = g.o * (1.0 - g.o) * d2[5];
}

// Per-pixel adjoint of the blend (FP64, forward-mode suffix sums): for the
// blended list (alpha_i, T_i), dF/dalpha_i = T_i f_i - S_i / (1 - alpha_i)
// with S_i = sum_{j>i} alpha_j T_j f_j + T_final bg, and
// dA_out/dalpha_i = T_final / (1 - alpha_i).  Accumulates into g2d (6 per
// list position) and gf (c per list position).
void pixel_adjoint(const Ctx& k, const std::vector<Contrib>& cb, double Tfin, const double* g,
                   double gA, const double* bg, const Proj* proj, double* g2d, double* gf) {
  const int C = k.c;
  std::vector<double> S(C);
  for (int ch = 0; ch < C; ++ch) S[ch] = Tfin * bg[ch];
  for (int i = (int)cb.size() - 1; i >= 0; --i) {
    const Contrib& e = cb[i];
    const double* f = &k.feat[(size_t)e.gi * C];
    double dLda = gA * Tfin / (1.0 - e.alpha);
    for (int ch = 0; ch < C; ++ch) dLda += g[ch] * (e.T * f[ch] - PLANT(6, S[ch], 0.0) / (1.0 - e.alpha));
    for (int ch = 0; ch < C; ++ch) gf[(size_t)e.pos * C + ch] += e.alpha * e.T * g[ch];
    for (int ch = 0; ch < C; ++ch) S[ch] += e.alpha * e.T * f[ch];
    if (e.clamped) continue;
    const Proj& p = proj[e.gi];
    const double dLdP = dLda * e.alpha;
    double* q = &g2d[(size_t)e.pos * 6];
    q[0] += dLdP * (p.A * e.dx + p.B * e.dy);
    q[1] += dLdP * (p.C * e.dy + p.B * e.dx);
    q[2] += dLdP * (-0.5 * e.dx * e.dx);
    q[3] += dLdP * (-e.dx * e.dy);
    q[4] += dLdP * (-0.5 * e.dy * e.dy);
    q[5] += dLda * e.G;
  }
}

}  // namespace

// ------------------------------------------------- lifting source views
// The step upstream of the rasterizer (§4.1: each predicted disparity map is
// converted to a depth map; §4.2: given the camera parameters, Gaussian
// positions are unprojected from the depth maps, and the foreground pixels
// of the source views become pixel-aligned Gaussians whose feature, scale
// and opacity are the encoder's per-pixel maps; their rotation is fixed to
// identity).  For a rectified stereo pair the depth of a pixel with
// disparity d is z = f_x B / d (B the baseline); a pixel is lifted when it
// is foreground and its disparity (or depth) is positive.
struct LiftView {
  CamD cam;                 // world -> camera x_c = R x_w + t; fx, fy, cx, cy; W, H
  const double* disparity;  // [H][W] or null (then depth)
  const double* depth;      // [H][W]
  const uint8_t* mask;      // [H][W] foreground != 0
  const double* feat;       // [H][W][c]
  const double* scale;      // [H][W][3]
  const double* opacity;    // [H][W]
  double baseline;
};

// Append the Gaussians of one view, pixel by pixel in row-major order.
void lift_view(const LiftView& v, int c, std::vector<double>& mean, std::vector<double>& scale,
               std::vector<double>& opac, std::vector<double>& feat) {
  const CamD& k = v.cam;
  for (int j = 0; j < k.H; ++j)
    for (int i = 0; i < k.W; ++i) {
      const int64_t p = (int64_t)j * k.W + i;
      if (!v.mask[p]) continue;
      double z;
      if (v.disparity) {
        const double d = v.disparity[p];
        if (!(d > 0.0)) continue;
        z = PLANT(12, k.fx * v.baseline / d, v.baseline / d);
      } else {
        z = v.depth[p];
        if (!(z > 0.0)) continue;
      }
      // the camera-space point on the ray through the pixel centre at depth z
      const double xc[3] = {(i + PLANT(13, 0.5, 0.0) - k.cx) / k.fx * z, (j + 0.5 - k.cy) / k.fy * z, z};
      // world point: x_w = R^T (x_c - t)
      for (int a = 0; a < 3; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 3; ++b)
          acc += PLANT(14, k.R[3 * b + a], k.R[3 * a + b]) * (xc[b] - k.t[b]);
        mean.push_back(acc);
      }
      for (int a = 0; a < 3; ++a) scale.push_back(v.scale[3 * p + a]);
      opac.push_back(v.opacity[p]);
      for (int ch = 0; ch < c; ++ch) feat.push_back(v.feat[(size_t)p * c + ch]);
    }
}

// ------------------------------------------------------ z-buffer splat
// The cascaded disparity initialisation (§4.1): the point cloud lifted from
// cam0's depth is rasterized into the viewpoint of another camera, the
// z-buffer (the nearest depth per pixel) is extracted and converted back to
// a disparity map.  Reading: each point is a one-pixel splat; it lands in
// the pixel (floor(u), floor(v)) that contains its projection and competes
// there with its view depth t_z; points with t_z <= znear or outside the
// image land nowhere.  The pixel and the depth are discrete decisions, taken
// in float32 with the operation order of the binning spec (a)-(c) so that
// they are reproducible bit for bit; disparity = fx B / z in FP64, rounded
// to float32, and 0 where no point landed.
struct SplatHit { bool ok; int i, j; float z; };

SplatHit splat_point(const CamF& c, const float mu[3]) {
  SplatHit h{false, 0, 0, 0.f};
  const float tx = ((c.R[0] * mu[0] + c.R[1] * mu[1]) + c.R[2] * mu[2]) + c.t[0];
  const float ty = ((c.R[3] * mu[0] + c.R[4] * mu[1]) + c.R[5] * mu[2]) + c.t[1];
  const float tz = ((c.R[6] * mu[0] + c.R[7] * mu[1]) + c.R[8] * mu[2]) + c.t[2];
  if (!(tz > c.znear)) return h;
  const float u = (c.fx * tx) / tz + c.cx;
  const float v = (c.fy * ty) / tz + c.cy;
  const float fi = std::floor(PLANT(15, u, u + 0.5f)), fj = std::floor(v);
  if (!(fi >= 0.0f && fi < (float)c.W && fj >= 0.0f && fj < (float)c.H)) return h;
  h.ok = true;
  h.i = (int)fi;
  h.j = (int)fj;
  h.z = tz;
  return h;
}

// ------------------------------------------- occlusion-aware view blending
// §4.3 blends the source views' colours into the novel view to give the
// high-resolution image I_blend that the refiner takes:
//   1. the predicted depth maps are warped onto the novel view into a fused
//      depth z_fused (the caller passes it; here it is the z-buffer splat of
//      the lifted points into the novel camera);
//   2. every novel pixel with a fused depth is back-projected and projected
//      into every source view, x_i = Pi_i(Pi_novel^-1(u, v, z_fused)) (Eq. 6);
//   3. colour c_i and depth z_i are fetched from view i by bilinear
//      sampling at x_i's pixel coordinates (Eq. 7);
//   4. weight w_i = M_i(x_i) Occ(x_i) cos<r(u, v), n_i> / |x_i^cam| (Eq. 8)
//      with Occ = 1 iff |x_i.z - z_i| < delta (Eq. 9);
//   5. I_blend = sum_i w_i c_i / sum_i w_i (Eq. 10).
// Readings where the paper is silent:
//   * pixel centres at (i + 0.5, j + 0.5) in every view; bilinear sampling
//     between the four pixel centres around the point (the top-left one
//     clamped so that all four lie inside the view), for points inside the
//     rectangle spanned by the view's pixel centres (elsewhere the view
//     gets no weight);
//   * M_i(x_i) is the bilinear sample of the 0/1 mask (so it fades over one
//     pixel at the mask's border), like every other map fetched at x_i;
//   * the normal n_i is the unit normal of view i's depth surface (below),
//     bilinearly sampled and renormalised, oriented toward view i's camera;
//     the cosine is taken against the reversed ray, max(0, -<r, n_i>), so a
//     surface facing the novel camera weighs most and one seen edge-on or
//     from behind weighs nothing;
//   * colours are 8-bit RGBA (alpha unused), blended as value / 255;
//   * a pixel without a fused depth (not > 0 or infinite), or whose weights
//     sum to zero, gets colour 0 and weight sum 0 (the refiner's mask).
// Every step is an FP64 operation in the written order, so an IEEE
// implementation of the same sequence reproduces the float32 outputs bit
// for bit.

// Unit normal of a depth map at pixel (i, j), in the world frame: the
// cross product of the central differences of the camera-space points
// P(i +- 1, j) and P(i, j +- 1) (pixel centres unprojected at their depth),
// turned toward the camera (<n, P(i, j)> < 0).  Zero at the border and
// where any of the five depths is not positive.
void normal_at(const CamD& k, const float* depth, int i, int j, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  if (i < 1 || j < 1 || i > k.W - 2 || j > k.H - 2) return;
  auto z_at = [&](int a, int b) { return (double)depth[(int64_t)b * k.W + a]; };
  const double zc = z_at(i, j), zl = z_at(i - 1, j), zr = z_at(i + 1, j), zu = z_at(i, j - 1),
               zd = z_at(i, j + 1);
  if (!(zc > 0.0 && zl > 0.0 && zr > 0.0 && zu > 0.0 && zd > 0.0)) return;
  auto P = [&](int a, int b, double z, double p[3]) {
    p[0] = ((a + 0.5) - k.cx) / k.fx * z;
    p[1] = ((b + 0.5) - k.cy) / k.fy * z;
    p[2] = z;
  };
  double pc[3], pl[3], pr[3], pu[3], pd[3];
  P(i, j, zc, pc); P(i - 1, j, zl, pl); P(i + 1, j, zr, pr); P(i, j - 1, zu, pu); P(i, j + 1, zd, pd);
  const double dx[3] = {pr[0] - pl[0], pr[1] - pl[1], pr[2] - pl[2]};
  const double dy[3] = {pd[0] - pu[0], pd[1] - pu[1], pd[2] - pu[2]};
  double c[3] = {dx[1] * dy[2] - dx[2] * dy[1], dx[2] * dy[0] - dx[0] * dy[2],
                 PLANT(17, dx[0] * dy[1] - dx[1] * dy[0], dx[0] * dy[1] + dx[1] * dy[0])};
  const double len = std::sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
  if (!(len > 0.0)) return;
  const double side = (c[0] * pc[0] + c[1] * pc[1]) + c[2] * pc[2];
  const double sgn = PLANT(18, side > 0.0 ? -1.0 : 1.0, 1.0);
  const double n[3] = {sgn * c[0] / len, sgn * c[1] / len, sgn * c[2] / len};
  for (int a = 0; a < 3; ++a) {
    double acc = 0.0;
    for (int b = 0; b < 3; ++b) acc = acc + k.R[3 * b + a] * n[b];
    out[a] = acc;
  }
}

struct BlendView {
  CamD cam;
  const uint8_t* rgba;    // [H][W][4]
  const float* depth;     // [H][W]
  const uint8_t* mask;    // [H][W]
  const float* normal;    // [H][W][3] world frame
};

// Colour (3) and weight sum of novel pixel (i, j) at fused depth z.
void blend_pixel(const CamD& nv, const std::vector<BlendView>& views, int i, int j, double z, double delta,
                 double rgb[3], double& wsum) {
  rgb[0] = rgb[1] = rgb[2] = 0.0;
  wsum = 0.0;
  if (!(z > 0.0) || std::isinf(z)) return;
  // Eq. 6: back-projection into the world
  const double pn[3] = {((i + 0.5) - nv.cx) / nv.fx * z, ((j + 0.5) - nv.cy) / nv.fy * z, z};
  double X[3], r[3];
  const double pl = std::sqrt((pn[0] * pn[0] + pn[1] * pn[1]) + pn[2] * pn[2]);
  const double rc[3] = {pn[0] / pl, pn[1] / pl, pn[2] / pl};
  for (int a = 0; a < 3; ++a) {
    double acc = 0.0, ra = 0.0;
    for (int b = 0; b < 3; ++b) {
      acc = acc + nv.R[3 * b + a] * (pn[b] - nv.t[b]);
      ra = ra + nv.R[3 * b + a] * rc[b];
    }
    X[a] = acc;
    r[a] = ra;
  }
  double acc[3] = {0.0, 0.0, 0.0}, ws = 0.0;
  for (const BlendView& v : views) {
    const CamD& k = v.cam;
    double xc[3];
    for (int a = 0; a < 3; ++a) xc[a] = ((k.R[3 * a] * X[0] + k.R[3 * a + 1] * X[1]) + k.R[3 * a + 2] * X[2]) + k.t[a];
    if (!(xc[2] > k.znear)) continue;
    const double u = (k.fx * xc[0]) / xc[2] + k.cx, w = (k.fy * xc[1]) / xc[2] + k.cy;
    // Eq. 7: bilinear taps around (u, w) between pixel centres; (su, sw)
    // must lie in the rectangle spanned by the view's pixel centres
    const double su = u - PLANT(19, 0.5, 0.0), sw = w - 0.5;
    if (!(su >= 0.0 && su <= k.W - 1.0 && sw >= 0.0 && sw <= k.H - 1.0)) continue;
    const double fu = std::min(std::floor(su), std::max(k.W - 2.0, 0.0));
    const double fw = std::min(std::floor(sw), std::max(k.H - 2.0, 0.0));
    const int i0 = (int)fu, j0 = (int)fw;
    const int i1 = std::min(i0 + 1, k.W - 1), j1 = std::min(j0 + 1, k.H - 1);
    const double a = su - fu, b = sw - fw;
    const double w00 = (1.0 - a) * (1.0 - b), w10 = a * (1.0 - b), w01 = (1.0 - a) * b, w11 = a * b;
    const int64_t p00 = (int64_t)j0 * k.W + i0, p10 = (int64_t)j0 * k.W + i1, p01 = (int64_t)j1 * k.W + i0,
                  p11 = (int64_t)j1 * k.W + i1;
    auto interp = [&](double f00, double f10, double f01, double f11) {
      return ((w00 * f00 + w10 * f10) + w01 * f01) + w11 * f11;
    };
    const double m = interp(v.mask[p00] ? 1.0 : 0.0, v.mask[p10] ? 1.0 : 0.0, v.mask[p01] ? 1.0 : 0.0,
                            v.mask[p11] ? 1.0 : 0.0);
    if (!(m > 0.0)) continue;
    const double zi = interp(v.depth[p00], v.depth[p10], v.depth[p01], v.depth[p11]);
    // Eq. 9: the occlusion check against the view's own depth
    if (!(std::fabs(xc[2] - zi) < delta)) continue;
    double n[3];
    for (int q = 0; q < 3; ++q)
      n[q] = interp(v.normal[3 * p00 + q], v.normal[3 * p10 + q], v.normal[3 * p01 + q], v.normal[3 * p11 + q]);
    const double nl = std::sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
    if (!(nl > 0.0)) continue;
    const double cosv = PLANT(20, -((r[0] * n[0] + r[1] * n[1]) + r[2] * n[2]) / nl,
                              ((r[0] * n[0] + r[1] * n[1]) + r[2] * n[2]) / nl);
    if (!(cosv > 0.0)) continue;
    const double dist = std::sqrt((xc[0] * xc[0] + xc[1] * xc[1]) + xc[2] * xc[2]);
    // Eq. 8
    const double wt = (m * cosv) / PLANT(21, dist, 1.0);
    for (int q = 0; q < 3; ++q) {
      const double c = interp(v.rgba[4 * p00 + q], v.rgba[4 * p10 + q], v.rgba[4 * p01 + q], v.rgba[4 * p11 + q]) / 255.0;
      acc[q] = acc[q] + wt * c;
    }
    ws = ws + wt;
  }
  if (!(ws > 0.0)) return;
  // Eq. 10
  for (int q = 0; q < 3; ++q) rgb[q] = acc[q] / ws;
  wsum = ws;
}

// =================================================================== C ABI
extern "C" {

// Build the oracle's state for one scene.  Arrays are FP64 copies of the
// scene: mean/scale [3][n], quat [4][n] (w,x,y,z), opacity [n] (activated),
// feat [n][c]; cam = R[9], t[3], fx, fy, cx, cy, width, height, znear.
void* tgo_create(int64_t n, int c, const double* mean, const double* scale, const double* quat,
                 const double* opac, const double* feat, const double* cam, int nthreads) {
  if (n < 0 || c <= 0 || !cam) return nullptr;
  return make_ctx(n, c, mean, scale, quat, opac, feat, cam, nthreads);
}

void tgo_destroy(void* h) { delete static_cast<Ctx*>(h); }

int64_t tgo_num_keys(void* h) { return (int64_t)static_cast<Ctx*>(h)->list.size(); }

// Per-Gaussian binning spec: rect [4][n] (x0, y0, x1, y1; -1 when culled),
// depth key [n], culled [n].
void tgo_spec(void* h, int32_t* rect, uint32_t* key, uint8_t* culled) {
  Ctx& k = *static_cast<Ctx*>(h);
  for (int64_t i = 0; i < k.n; ++i) {
    const Spec& s = k.spec[i];
    const bool c = s.culled != 0;
    rect[0 * k.n + i] = c ? -1 : s.x0;
    rect[1 * k.n + i] = c ? -1 : s.y0;
    rect[2 * k.n + i] = c ? -1 : s.x1;
    rect[3 * k.n + i] = c ? -1 : s.y1;
    key[i] = c ? 0u : s.key;
    culled[i] = (uint8_t)c;
  }
}

// FP64 projected state [n][6]: u, v, A, B, C, o (NaN when culled).
void tgo_proj(void* h, double* out) {
  Ctx& k = *static_cast<Ctx*>(h);
  for (int64_t i = 0; i < k.n; ++i) {
    const Proj& p = k.proj[i];
    double* o = out + 6 * i;
    if (k.spec[i].culled) { for (int j = 0; j < 6; ++j) o[j] = NAN; continue; }
    o[0] = p.u; o[1] = p.v; o[2] = p.A; o[3] = p.B; o[4] = p.C; o[5] = p.o;
  }
}

// Tile lists in CSR form: tile_start [tiles + 1], list [K].
void tgo_tile_lists(void* h, int64_t* tile_start, int32_t* list) {
  Ctx& k = *static_cast<Ctx*>(h);
  std::copy(k.tile_start.begin(), k.tile_start.end(), tile_start);
  std::copy(k.list.begin(), k.list.end(), list);
}

// Forward render.  out_feat [c][H][W], out_alpha/out_T [H][W], out_last
// [H][W] (list position of the last blended Gaussian, -1 if none),
// out_nflags [H][W] (near-threshold decisions), work[2] = (evaluated pairs,
// blended pairs).
void tgo_render_fwd(void* h, const double* bg, double* out_feat, double* out_alpha, double* out_T,
                    int32_t* out_last, int32_t* out_nflags, int64_t* work) {
  Ctx& k = *static_cast<Ctx*>(h);
  const int W = k.cam.W, H = k.cam.H, C = k.c;
  const int64_t T = (int64_t)k.tiles_x * k.tiles_y;
  std::atomic<int64_t> ne{0}, nc{0};
  parallel_for(T, k.nthreads, [&](int64_t t) {
    const int tx = (int)(t % k.tiles_x), ty = (int)(t / k.tiles_x);
    const int64_t s = k.tile_start[t], len = k.tile_start[t + 1] - s;
    std::vector<double> F(C);
    int64_t le = 0, lc = 0;
    for (int py = ty * TILE; py < std::min(H, ty * TILE + TILE); ++py)
      for (int px = tx * TILE; px < std::min(W, tx * TILE + TILE); ++px) {
        std::fill(F.begin(), F.end(), 0.0);
        PixelRun run;
        blend_pixel(k, k.proj.data(), k.list.data() + s, len, px + 0.5, py + 0.5, F.data(), run);
        const int64_t pix = (int64_t)py * W + px;
        for (int ch = 0; ch < C; ++ch)
          out_feat[(int64_t)ch * H * W + pix] = F[ch] + run.T * (bg ? bg[ch] : 0.0);
        if (out_alpha) out_alpha[pix] = 1.0 - run.T;
        if (out_T) out_T[pix] = run.T;
        if (out_last) out_last[pix] = run.last;
        if (out_nflags) out_nflags[pix] = (int32_t)run.flags.size();
        le += run.n_eval; lc += run.n_contrib;
      }
    ne += le; nc += lc;
  });
  if (work) { work[0] = ne.load(); work[1] = nc.load(); }
}

// All branch variants of one pixel (up to 2 flagged decisions -> up to 4
// variants).  out [4][c + 1] holds (F[0..c-1], alpha) per variant.
// Returns the number of variants, or -(number of flags) when > 2 flags.
int tgo_pixel_variants(void* h, int px, int py, const double* bg, double* out) {
  Ctx& k = *static_cast<Ctx*>(h);
  const int C = k.c;
  const int64_t t = tile_of(k, px, py);
  const int64_t s = k.tile_start[t], len = k.tile_start[t + 1] - s;
  std::vector<double> F(C, 0.0);
  PixelRun base;
  blend_pixel(k, k.proj.data(), k.list.data() + s, len, px + 0.5, py + 0.5, F.data(), base);
  const int nf = (int)base.flags.size();
  if (nf > 2) return -nf;
  int nv = 0;
  for (int mask = 0; mask < (1 << nf); ++mask) {
    std::vector<int> flip;
    for (int b = 0; b < nf; ++b)
      if (mask & (1 << b)) flip.push_back(base.flags[b].pos);
    std::fill(F.begin(), F.end(), 0.0);
    PixelRun run;
    BlendOpts op;
    op.flip = &flip;
    blend_pixel(k, k.proj.data(), k.list.data() + s, len, px + 0.5, py + 0.5, F.data(), run, op);
    for (int ch = 0; ch < C; ++ch)
      out[nv * (C + 1) + ch] = F[ch] + PLANT(11, run.T * (bg ? bg[ch] : 0.0), 0.0);
    out[nv * (C + 1) + C] = PLANT(10, 1.0 - run.T, run.T);
    ++nv;
  }
  return nv;
}

// Gaussian indices a pixel's walk evaluates (up to and including the one
// that stops it).  Returns the count (<= cap entries are written).
int tgo_pixel_walk(void* h, int px, int py, int32_t* out, int cap) {
  Ctx& k = *static_cast<Ctx*>(h);
  const int64_t t = tile_of(k, px, py);
  const int64_t s = k.tile_start[t], len = k.tile_start[t + 1] - s;
  std::vector<double> F(k.c, 0.0);
  std::vector<uint8_t> dec;
  PixelRun run;
  BlendOpts op;
  op.dec = &dec;
  blend_pixel(k, k.proj.data(), k.list.data() + s, len, px + 0.5, py + 0.5, F.data(), run, op);
  const int cnt = (int)dec.size();
  for (int i = 0; i < cnt && i < cap; ++i) out[i] = k.list[s + i];
  return cnt;
}

// Brute force O(pixels x n): for every pixel, every Gaussian is tested for
// "its rectangle holds this pixel's tile", the candidates are sorted by
// (depth key, index) and blended.  Independent of the tile lists.
void tgo_render_brute(void* h, const double* bg, double* out_feat, double* out_alpha) {
  Ctx& k = *static_cast<Ctx*>(h);
  const int W = k.cam.W, H = k.cam.H, C = k.c;
  parallel_for((int64_t)H, k.nthreads, [&](int64_t py) {
    std::vector<double> F(C);
    std::vector<int32_t> cand;
    for (int px = 0; px < W; ++px) {
      const int tx = px / TILE, ty = (int)py / TILE;
      cand.clear();
      for (int64_t i = 0; i < k.n; ++i) {
        const Spec& s = k.spec[i];
        if (s.culled) continue;
        if (tx >= s.x0 && tx <= s.x1 && ty >= s.y0 && ty <= s.y1) cand.push_back((int32_t)i);
      }
      std::stable_sort(cand.begin(), cand.end(),
                       [&](int32_t a, int32_t b) { return k.spec[a].key < k.spec[b].key; });
      std::fill(F.begin(), F.end(), 0.0);
      PixelRun run;
      blend_pixel(k, k.proj.data(), cand.data(), (int64_t)cand.size(), px + 0.5, py + 0.5, F.data(),
                  run);
      const int64_t pix = py * W + px;
      for (int ch = 0; ch < C; ++ch)
        out_feat[(int64_t)ch * H * W + pix] = F[ch] + run.T * (bg ? bg[ch] : 0.0);
      out_alpha[pix] = 1.0 - run.T;
    }
  });
}

// Analytic backward (FP64).  d_feat_img [c][H][W], d_alpha_img [H][W] or
// NULL.  Outputs: g2d [n][6] (du, dv, dA, dB, dC, d opacity), and the raw
// parameter gradients g_mean [3][n], g_logscale [3][n], g_quat [4][n],
// g_logit [n], g_feat [n][c].  Any output pointer may be NULL.
// flip_mask [H][W] or NULL: bit b of a pixel's mask inverts the b-th
// near-threshold decision of its walk, numbered as tgo_pixel_variants numbers
// them (variant m of that call is mask m); a zero mask is the plain walk.
void tgo_render_bwd(void* h, const double* bg, const double* d_img, const double* d_alpha,
                    double* g2d_out, double* g_mean, double* g_ls, double* g_quat, double* g_logit,
                    double* g_feat, const uint8_t* flip_mask) {
  Ctx& k = *static_cast<Ctx*>(h);
  const int W = k.cam.W, H = k.cam.H, C = k.c;
  const int64_t T = (int64_t)k.tiles_x * k.tiles_y;
  std::vector<double> g2d((size_t)k.n * 6, 0.0), gf((size_t)k.n * C, 0.0);
  std::vector<double> zero_bg(C, 0.0);
  const double* bgp = bg ? bg : zero_bg.data();
  const int64_t CH = 512;   // tiles per chunk (bounds the per-tile scratch)
  for (int64_t t0 = 0; t0 < T; t0 += CH) {
    const int64_t t1 = std::min(T, t0 + CH);
    std::vector<std::vector<double>> tg2(t1 - t0), tgf(t1 - t0);
    parallel_for(t1 - t0, k.nthreads, [&](int64_t j) {
      const int64_t t = t0 + j;
      const int tx = (int)(t % k.tiles_x), ty = (int)(t / k.tiles_x);
      const int64_t s = k.tile_start[t], len = k.tile_start[t + 1] - s;
      tg2[j].assign((size_t)len * 6, 0.0);
      tgf[j].assign((size_t)len * C, 0.0);
      std::vector<double> F(C), g(C);
      std::vector<Contrib> cb;
      std::vector<int> flip;
      for (int py = ty * TILE; py < std::min(H, ty * TILE + TILE); ++py)
        for (int px = tx * TILE; px < std::min(W, tx * TILE + TILE); ++px) {
          const int64_t pix = (int64_t)py * W + px;
          for (int ch = 0; ch < C; ++ch) g[ch] = d_img[(int64_t)ch * H * W + pix];
          const double gA = d_alpha ? d_alpha[pix] : 0.0;
          std::fill(F.begin(), F.end(), 0.0);
          cb.clear();
          PixelRun run;
          BlendOpts op;
          op.contrib = &cb;
          const unsigned m = flip_mask ? flip_mask[pix] : 0u;
          if (m) {   // the plain walk numbers the flagged decisions
            PixelRun probe;
            blend_pixel(k, k.proj.data(), k.list.data() + s, len, px + 0.5, py + 0.5, F.data(),
                        probe);
            std::fill(F.begin(), F.end(), 0.0);
            flip.clear();
            for (int b = 0; b < (int)probe.flags.size() && b < 8; ++b)
              if (m & (1u << b)) flip.push_back(probe.flags[b].pos);
            op.flip = &flip;
          }
          blend_pixel(k, k.proj.data(), k.list.data() + s, len, px + 0.5, py + 0.5, F.data(), run,
                      op);
          pixel_adjoint(k, cb, run.T, g.data(), gA, bgp, k.proj.data(), tg2[j].data(),
                        tgf[j].data());
        }
    });
    for (int64_t t = t0; t < t1; ++t) {          // deterministic reduction in tile order
      const int64_t s = k.tile_start[t], len = k.tile_start[t + 1] - s;
      const std::vector<double>& a = tg2[t - t0];
      const std::vector<double>& b = tgf[t - t0];
      for (int64_t p = 0; p < len; ++p) {
        const int32_t gi = k.list[s + p];
        for (int q = 0; q < 6; ++q) g2d[(size_t)gi * 6 + q] += a[(size_t)p * 6 + q];
        for (int ch = 0; ch < C; ++ch) gf[(size_t)gi * C + ch] += b[(size_t)p * C + ch];
      }
    }
  }
  if (g2d_out) std::copy(g2d.begin(), g2d.end(), g2d_out);
  if (g_feat) std::copy(gf.begin(), gf.end(), g_feat);
  if (g_mean || g_ls || g_quat || g_logit) {
    parallel_for((k.n + 1023) / 1024, k.nthreads, [&](int64_t b) {
      for (int64_t i = b * 1024; i < std::min<int64_t>(k.n, (b + 1) * 1024); ++i) {
        double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dl = 0;
        if (!k.spec[i].culled) chain_to_raw(k.cam, k.g[i], &g2d[(size_t)i * 6], dmu, dls, dq, dl);
        for (int d = 0; d < 3; ++d) {
          if (g_mean) g_mean[d * k.n + i] = dmu[d];
          if (g_ls) g_ls[d * k.n + i] = dls[d];
        }
        for (int d = 0; d < 4; ++d)
          if (g_quat) g_quat[d * k.n + i] = dq[d];
        if (g_logit) g_logit[i] = dl;
      }
    });
  }
}

// Central finite differences (FP64) of L = sum_p <dF(p), F(p)> + dA(p) A(p)
// with respect to the raw parameters of the Gaussians in `sel`.  Parameter
// order per Gaussian: mean x,y,z; log-scale x,y,z; quat w,x,y,z; opacity
// logit; features 0..c-1  (11 + c values).  A perturbation of Gaussian g
// only changes the pixels of g's own tiles, and in each of them only the
// part of the walk from g's list position on, so only that part is
// re-evaluated (the shared prefix cancels in L(+eps) - L(-eps)).  A
// parameter whose +-eps perturbation changes any discrete decision (cull,
// rectangle, list order, skip / blend / stop / clamp state of any pixel) is
// excluded: out_excl = 1.  Features do not enter any decision and channel c
// of F depends on feature c only, so one walk per side evaluates all c
// feature perturbations at once (each channel's share of L separately).
void tgo_fd(void* h, const double* bg, const double* d_img, const double* d_alpha, int64_t nsel,
            const int64_t* sel, double eps, double* out_fd, uint8_t* out_excl) {
  Ctx& k = *static_cast<Ctx*>(h);
  const int W = k.cam.W, H = k.cam.H, C = k.c;
  const int NP = 11 + C;
  std::vector<double> zero_bg(C, 0.0);
  const double* bgp = bg ? bg : zero_bg.data();
  parallel_for(nsel, k.nthreads, [&](int64_t si) {
    const int64_t gi = sel[si];
    double* res = out_fd + si * NP;
    uint8_t* ex = out_excl + si * NP;
    for (int q = 0; q < NP; ++q) { res[q] = 0.0; ex[q] = 0; }
    const Spec& s0 = k.spec[gi];
    if (s0.culled) { for (int q = 0; q < NP; ++q) ex[q] = 1; return; }
    // pixels of g's tiles where g is reached: (tile list, position, pixel, T at position)
    struct Px { const int32_t* lst; int64_t len, pos; int px, py; double T; std::vector<uint8_t> dec; };
    std::vector<Px> pix;
    for (int ty = s0.y0; ty <= s0.y1; ++ty)
      for (int tx = s0.x0; tx <= s0.x1; ++tx) {
        const int64_t t = (int64_t)ty * k.tiles_x + tx;
        const int64_t st = k.tile_start[t], len = k.tile_start[t + 1] - st;
        const int32_t* lst = k.list.data() + st;
        int64_t pos = -1;
        for (int64_t p = 0; p < len; ++p)
          if (lst[p] == gi) { pos = p; break; }
        if (pos < 0) continue;
        for (int py = ty * TILE; py < std::min(H, ty * TILE + TILE); ++py)
          for (int px = tx * TILE; px < std::min(W, tx * TILE + TILE); ++px) {
            std::vector<double> F(C, 0.0);
            PixelRun pre;
            BlendOpts op;
            op.end = pos;
            blend_pixel(k, k.proj.data(), lst, len, px + 0.5, py + 0.5, F.data(), pre, op);
            if (pre.stopped) continue;                    // g is never reached here
            Px e{lst, len, pos, px, py, pre.T, {}};
            PixelRun suf;
            BlendOpts o2;
            o2.start = pos; o2.T0 = pre.T; o2.dec = &e.dec;
            std::fill(F.begin(), F.end(), 0.0);
            blend_pixel(k, k.proj.data(), lst, len, px + 0.5, py + 0.5, F.data(), suf, o2);
            pix.push_back(std::move(e));
          }
      }
    // the list-order check of a perturbed depth key
    auto order_ok = [&](uint32_t key) {
      for (int ty = s0.y0; ty <= s0.y1; ++ty)
        for (int tx = s0.x0; tx <= s0.x1; ++tx) {
          const int64_t t = (int64_t)ty * k.tiles_x + tx;
          const int64_t st = k.tile_start[t], len = k.tile_start[t + 1] - st;
          const int32_t* lst = k.list.data() + st;
          for (int64_t p = 0; p < len; ++p) {
            if (lst[p] != gi) continue;
            auto less = [](uint32_t ka, int64_t ia, uint32_t kb, int64_t ib) {
              return ka != kb ? ka < kb : ia < ib;
            };
            if (p > 0 && !less(k.spec[lst[p - 1]].key, lst[p - 1], key, gi)) return false;
            if (p + 1 < len && !less(key, gi, k.spec[lst[p + 1]].key, lst[p + 1])) return false;
          }
        }
      return true;
    };
    const Gauss& g0 = k.g[gi];
    const double* f0 = &k.feat[(size_t)gi * C];
    std::vector<double> fpert(C), F(C), Lc(C);
    std::vector<uint8_t> dec;
    // geometry and opacity parameters
    for (int pi = 0; pi < 11; ++pi) {
      double L[2] = {0.0, 0.0};
      bool bad = false;
      for (int side = 0; side < 2 && !bad; ++side) {
        const double e = side == 0 ? eps : -eps;
        Gauss gp = g0;
        if (pi < 3) gp.mu[pi] += e;
        else if (pi < 6) gp.s[pi - 3] = std::exp(std::log(g0.s[pi - 3]) + e);
        else if (pi < 10) gp.q[pi - 6] += e;
        else {
          const double lg = std::log(g0.o / (1.0 - g0.o)) + e;
          gp.o = 1.0 / (1.0 + std::exp(-lg));
        }
        const Spec sp = spec_of(k, gp);
        Proj pp; double S3[9], Am[6], r[9], qn[4];
        if (sp.culled || sp.x0 != s0.x0 || sp.x1 != s0.x1 || sp.y0 != s0.y0 || sp.y1 != s0.y1 ||
            !order_ok(sp.key) || !project64(k.cam, gp, pp, S3, Am, r, qn)) {
          bad = true;
          break;
        }
        double Ls = 0.0;
        for (const Px& e2 : pix) {
          std::fill(F.begin(), F.end(), 0.0);
          dec.clear();
          PixelRun run;
          BlendOpts op;
          op.start = e2.pos; op.T0 = e2.T; op.dec = &dec;
          op.swap_gi = (int32_t)gi; op.swap_p = &pp;
          blend_pixel(k, k.proj.data(), e2.lst, e2.len, e2.px + 0.5, e2.py + 0.5, F.data(), run, op);
          if (dec != e2.dec) { bad = true; break; }
          const int64_t p = (int64_t)e2.py * W + e2.px;
          for (int ch = 0; ch < C; ++ch) Ls += d_img[(int64_t)ch * H * W + p] * (F[ch] + run.T * bgp[ch]);
          if (d_alpha) Ls += d_alpha[p] * (1.0 - run.T);
        }
        L[side] = Ls;
      }
      if (bad) ex[pi] = 1;
      else res[pi] = (L[0] - L[1]) / (2.0 * eps);
    }
    // feature parameters: one walk per side, channel c's share of L per channel
    double Lf[2][256];
    const int Cc = std::min(C, 256);
    for (int side = 0; side < 2; ++side) {
      const double e = side == 0 ? eps : -eps;
      for (int ch = 0; ch < C; ++ch) fpert[ch] = f0[ch] + e;
      std::fill(Lc.begin(), Lc.end(), 0.0);
      for (const Px& e2 : pix) {
        std::fill(F.begin(), F.end(), 0.0);
        PixelRun run;
        BlendOpts op;
        op.start = e2.pos; op.T0 = e2.T;
        op.swap_gi = (int32_t)gi; op.swap_f = fpert.data();
        blend_pixel(k, k.proj.data(), e2.lst, e2.len, e2.px + 0.5, e2.py + 0.5, F.data(), run, op);
        const int64_t p = (int64_t)e2.py * W + e2.px;
        for (int ch = 0; ch < C; ++ch) Lc[ch] += d_img[(int64_t)ch * H * W + p] * F[ch];
      }
      for (int ch = 0; ch < Cc; ++ch) Lf[side][ch] = Lc[ch];
    }
    for (int ch = 0; ch < Cc; ++ch) res[11 + ch] = (Lf[0][ch] - Lf[1][ch]) / (2.0 * eps);
    for (int ch = Cc; ch < C; ++ch) ex[11 + ch] = 1;
  });
}

// Lift n_views source views (see lift_view).  Per view v, cams[19 v ..] is
// the camera vector of tgo_create; disp[v] or depth[v] [H][W], mask[v]
// [H][W], feat[v] [H][W][c], scale[v] [H][W][3], opacity[v] [H][W],
// baseline[v].  Pass out_* = null to get the count only.  Outputs (each
// sized for at least the count): mean [3][n], scale [3][n], opacity [n],
// feat [n][c] with n the count (the rotation is the identity for every
// Gaussian).  Returns the count.
int64_t tgo_lift(int n_views, int c, const double* cams, const double* const* disp,
                 const double* const* depth, const uint8_t* const* mask, const double* const* feat,
                 const double* const* scale, const double* const* opac, const double* baseline,
                 double* out_mean, double* out_scale, double* out_opac, double* out_feat) {
  std::vector<double> m, s, o, f;
  for (int v = 0; v < n_views; ++v) {
    LiftView lv;
    lv.cam = cam_from(cams + 19 * v);
    lv.disparity = disp ? disp[v] : nullptr;
    lv.depth = depth ? depth[v] : nullptr;
    lv.mask = mask[v];
    lv.feat = feat[v];
    lv.scale = scale[v];
    lv.opacity = opac[v];
    lv.baseline = baseline[v];
    lift_view(lv, c, m, s, o, f);
  }
  const int64_t n = (int64_t)o.size();
  if (out_mean)
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        out_mean[a * n + i] = m[3 * i + a];
        out_scale[a * n + i] = s[3 * i + a];
      }
  if (out_opac) std::copy(o.begin(), o.end(), out_opac);
  if (out_feat) std::copy(f.begin(), f.end(), out_feat);
  return n;
}

// Z-buffer of n points (mean [3][n], float32 values given as FP64) in the
// camera `cam` (camera vector of tgo_create): zbuf [H][W] float32 (+inf where
// no point landed) and, if disp is not null, disparity [H][W] float32
// (fx B / z, 0 where empty).
void tgo_zsplat(const double* cam, const double* mean, int64_t n, double baseline, float* zbuf,
                float* disp) {
  const CamF c = to_f32(cam_from(cam));
  const int64_t P = (int64_t)c.W * c.H;
  for (int64_t p = 0; p < P; ++p) zbuf[p] = INFINITY;
  for (int64_t k = 0; k < n; ++k) {
    const float mu[3] = {(float)mean[k], (float)mean[n + k], (float)mean[2 * n + k]};
    const SplatHit h = splat_point(c, mu);
    if (!h.ok) continue;
    float& z = zbuf[(int64_t)h.j * c.W + h.i];
    if (PLANT(16, h.z < z, true)) z = h.z;
  }
  if (disp)
    for (int64_t p = 0; p < P; ++p)
      disp[p] = std::isinf(zbuf[p]) ? 0.0f : (float)((double)c.fx * (double)(float)baseline / (double)zbuf[p]);
}

// Normal map [H][W][3] (float32, world frame) of a depth map [H][W] seen
// by the camera `cam` (camera vector of tgo_create); see normal_at.
void tgo_normals(const double* cam, const float* depth, float* normal) {
  const CamD k = cam_from(cam);
  for (int j = 0; j < k.H; ++j)
    for (int i = 0; i < k.W; ++i) {
      double n[3];
      normal_at(k, depth, i, j, n);
      for (int a = 0; a < 3; ++a) normal[3 * ((int64_t)j * k.W + i) + a] = (float)n[a];
    }
}

// Occlusion-aware blending of n_views source views into the novel camera
// `novel` (camera vectors as tgo_create; per view cams[19 v ..], rgba[v]
// [H][W][4] uint8, depth[v] [H][W], mask[v] [H][W], normal[v] [H][W][3]),
// given z_fused [H_n][W_n]: rgb [3][H_n][W_n] and wsum [H_n][W_n] (float32).
void tgo_blend(int n_views, const double* cams, const uint8_t* const* rgba, const float* const* depth,
               const uint8_t* const* mask, const float* const* normal, const double* novel, const float* z_fused,
               double delta, float* rgb, float* wsum) {
  std::vector<BlendView> views((size_t)n_views);
  for (int v = 0; v < n_views; ++v) {
    views[v].cam = cam_from(cams + 19 * v);
    views[v].rgba = rgba[v];
    views[v].depth = depth[v];
    views[v].mask = mask[v];
    views[v].normal = normal[v];
  }
  const CamD nv = cam_from(novel);
  const int64_t P = (int64_t)nv.W * nv.H;
  for (int j = 0; j < nv.H; ++j)
    for (int i = 0; i < nv.W; ++i) {
      const int64_t p = (int64_t)j * nv.W + i;
      double c[3], ws;
      blend_pixel(nv, views, i, j, (double)z_fused[p], delta, c, ws);
      for (int q = 0; q < 3; ++q) rgb[q * P + p] = (float)c[q];
      wsum[p] = (float)ws;
    }
}

}  // extern "C"
