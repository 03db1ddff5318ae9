/* tg.h -- C ABI of the MI355X latent Gaussian rasterizer.
 *
 * The operation is the neural rasterizer R_G of Tele-Aloha (arXiv 2405.14866,
 * §4.2, "Latent-based Gaussian Splatting"): every foreground source pixel is
 * lifted to a Gaussian with position x, latent feature f (d = C channels),
 * scale s (3 values) and opacity alpha, and the set is splatted into the
 * target camera Pi_novel to give the latent map F_novel = R_G({G}, Pi_novel).
 * §4.2 makes R_G differentiable (the decoder is trained through it); §5.3
 * runs the system under CUDA Graphs, which the serving calls mirror with HIP
 * graphs.  The paper fixes the Gaussian rotation to identity; this ABI takes
 * a quaternion per Gaussian, identity (1, 0, 0, 0) being the paper's case.
 *
 * Conventions (the paper only cites the 3D Gaussian splatting rasterizer):
 *   - EWA projection with the perspective Jacobian, 0.3 px^2 added to the
 *     diagonal of the 2D covariance, radius r = ceil(3 sqrt(lambda_max)),
 *     16x16 tiles, the tile rectangle [floor((u-r)/16), floor((u+r)/16)]
 *     (clamped to the image) is a Gaussian's support;
 *   - per tile, Gaussians in ascending (view depth t_z, index) order;
 *   - alpha = min(0.99, o exp(-d^T Sigma'^-1 d / 2)) at pixel centres
 *     (i + 0.5, j + 0.5); alpha < 1/255 is skipped; a Gaussian that would take
 *     the transmittance below 1e-4 is not blended and ends the pixel;
 *   - F = sum_i alpha_i T_i f_i + T_final bg, alpha_out = 1 - T_final.
 *   Culling, tile rectangles and depth keys come from a fixed float32
 *   operation sequence, so the tile lists are reproducible bit for bit.
 *
 * Memory: every pointer argument is a DEVICE pointer unless marked (host).
 * The caller owns all inputs, outputs and gradient buffers; the library
 * owns contexts, frames and servers and the workspaces inside them.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 * default stream).  Every enqueue call only enqueues work on `stream` and
 * returns; results are valid once the stream has reached that point.  No
 * enqueue call synchronises the host or allocates memory, so a sequence of
 * them can be captured into a HIP graph.
 * Errors: functions return tg_status; nothing throws across the ABI.
 * Argument errors are detected before anything is enqueued.  Overflow of
 * the frame's key capacity is detected on the device: the frame is marked,
 * the later kernels of that frame do nothing, and tg_frame_check reports
 * TG_ERR_CAPACITY (the outputs of such a frame are undefined).
 */
#ifndef TG_H
#define TG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tg_status {
  TG_OK = 0,
  TG_PENDING = 1,          /* serving: request not finished yet */
  TG_ERR_INVALID = -1,     /* bad argument (null pointer, size, channel count) */
  TG_ERR_OOM = -2,         /* device allocation failed (create calls only) */
  TG_ERR_CAPACITY = -3,    /* more (tile, Gaussian) keys than the frame holds */
  TG_ERR_BUDGET = -4,      /* serving: request larger than the memory budget */
  TG_ERR_HIP = -5,         /* a HIP runtime call failed */
  TG_ERR_UNSUPPORTED = -6, /* e.g. channel count not compiled in */
  TG_ERR_NOT_FOUND = -7    /* serving: unknown ticket */
} tg_status;

/* Target camera Pi_novel (§4.2).  World -> camera x_c = R x_w + t with R
 * row-major, OpenCV axes (x right, y down, z forward).  Pixel (i, j) has its
 * centre at (i + 0.5, j + 0.5); u = fx x_c / z_c + cx.  Gaussians with view
 * depth z_c <= znear are culled.  Passed by host pointer. */
typedef struct tg_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear;
} tg_camera;

/* The Gaussian set {G} (§4.2: position x, latent feature f, scale s,
 * opacity alpha), structure-of-arrays float32 in device memory:
 *   mean    [3][n]   world position
 *   scale   [3][n]   activated scales (> 0)
 *   quat    [4][n]   rotation (w, x, y, z), need not be normalised, |q| > 0
 *   opacity [n]      activated opacity in [0, 1]
 *   feat    [n][c]   latent features, row-major
 * c must be 8, 16, 32 or 64.  The struct itself is a host object. */
typedef struct tg_gaussians {
  const float* mean;
  const float* scale;
  const float* quat;
  const float* opacity;
  const float* feat;
  int64_t n;
  int32_t c;
} tg_gaussians;

/* Gradients with respect to the raw parameters (same layouts as the
 * inputs): mean [3][n], log-scale [3][n] (scale = exp(log_scale)),
 * unnormalised quaternion [4][n], opacity logit [n] (opacity =
 * sigmoid(logit)), features [n][c].  Buffers are overwritten.  Host struct
 * of device pointers. */
typedef struct tg_grads {
  float* d_mean;
  float* d_log_scale;
  float* d_quat;
  float* d_opacity_logit;
  float* d_feat;
} tg_grads;

typedef struct tg_ctx tg_ctx;
typedef struct tg_frame tg_frame;
typedef struct tg_server tg_server;

/* Human-readable name of a status code (static string). */
const char* tg_status_string(tg_status s);

/* Create a context on HIP device `device`.  *out receives the handle. */
tg_status tg_ctx_create(int device, tg_ctx** out);
void tg_ctx_destroy(tg_ctx* ctx);

/* A frame is the resident workspace of one render: projected 2D state for
 * up to max_n Gaussians, tile counters, up to max_keys (tile, Gaussian)
 * keys, and the per-pixel final transmittance and last-contributor index of
 * up to max_w x max_h pixels that the backward pass reads.  It is reused
 * across renders; one frame serves one stream at a time.  max_n rounded up
 * to a multiple of 1024 (times max_views for tg_frame_create_views) is at
 * most 2^28: the binning packs a 4-bit quadrant mask above the Gaussian
 * index in its 32-bit index field (TG_ERR_INVALID beyond).  Allocates device
 * memory (TG_ERR_OOM on failure). */
tg_status tg_frame_create(tg_ctx* ctx, int64_t max_n, int32_t max_w, int32_t max_h,
                          int64_t max_keys, tg_frame** out);
void tg_frame_destroy(tg_frame* frame);

/* Step 1 -- projection (§4.2: the Gaussians are splatted into each target
 * view through its projection Pi_novel).  Per Gaussian: camera transform,
 * EWA 2D covariance with dilation, conic, 3-sigma radius, tile rectangle,
 * depth key, cull.  Reads g (n <= max_n), writes the frame's 2D state.
 * cam is a host pointer; its width/height must fit the frame. */
tg_status tg_project(tg_frame* frame, const tg_gaussians* g, const tg_camera* cam, void* stream);

/* Step 2 -- binning: count (tile, Gaussian) keys per tile, scan, scatter the
 * keys into per-tile segments and sort each segment by (depth key, index)
 * with an LDS radix sort.  Uses the state of the last tg_project.
 * The paper is silent on binning: §4.2 cites the tile-based 3D Gaussian
 * splatting rasterizer, whose front-to-back blend needs each 16x16 tile's
 * Gaussians in depth order; this call produces exactly that order, with the
 * Gaussian index breaking depth ties.  Errors: TG_ERR_INVALID for a null
 * frame or one never projected; key overflow is reported by tg_frame_check. */
tg_status tg_bin_sort(tg_frame* frame, void* stream);

/* Step 3 -- front-to-back blend (F_novel of §4.2).  out_feat [c][H][W]
 * (planar float32), out_alpha [H][W]; bg [c] or NULL (black).  g must be
 * the set given to tg_project. */
tg_status tg_render_fwd(tg_frame* frame, const tg_gaussians* g, const float* bg, float* out_feat,
                        float* out_alpha, void* stream);

/* tg_render_fwd that also counts the blend's work: the (pixel, Gaussian)
 * pairs each pixel evaluates before it ends and the pairs it blends.  Same
 * results as tg_render_fwd; slower; meant for measurement.  Read the counts
 * with tg_frame_work. */
tg_status tg_render_fwd_counted(tg_frame* frame, const tg_gaussians* g, const float* bg,
                                float* out_feat, float* out_alpha, void* stream);

/* SYNCHRONISES the frame's last stream and writes the first n_counts (<= 5)
 * counts of the last tg_render_fwd_counted to counts (host): the (pixel,
 * Gaussian) pairs the per-pixel walks visit up to and including the one
 * that ends them, the pairs blended, and three wave-level counts of the
 * implementation (Gaussian steps a wave takes after culling, steps in
 * which some lane passes the opacity threshold, steps in which some lane
 * blends). */
tg_status tg_frame_work(tg_frame* frame, int64_t* counts, int32_t n_counts);

/* Adjoint of steps 1-3 (§4.2: R_G is differentiable and the decoder is
 * trained through it).  d_feat [c][H][W], d_alpha [H][W] or NULL.  Uses the
 * final transmittance and last-contributor index stored by the last
 * tg_render_fwd of this frame and recomputes every earlier transmittance by
 * walking each pixel's list backwards.  g and bg must be those of that
 * forward (the stored state describes that render; the library keeps no
 * copy to compare with, so other values give gradients of no render).
 * Writes the raw-parameter gradients
 * of `out` (overwritten, device pointers; any of them may be NULL except
 * d_feat, which may be NULL only when g->n == 0). */
tg_status tg_render_bwd(tg_frame* frame, const tg_gaussians* g, const float* bg,
                        const float* d_feat, const float* d_alpha, const tg_grads* out,
                        void* stream);

/* SYNCHRONISES the frame's last stream.  Returns TG_ERR_CAPACITY when the
 * last binning overflowed max_keys, else TG_OK; *n_keys (host, may be NULL)
 * receives the number of keys the last binning needed. */
tg_status tg_frame_check(tg_frame* frame, int64_t* n_keys);

/* Copies of the last binning into caller buffers (device, enqueued on
 * `stream`): tile_start [n_tiles + 1] int32 offsets into sorted [n_keys]
 * int32 Gaussian indices, n_tiles = ceil(W/16) * ceil(H/16) of the last
 * tg_project, n_keys from tg_frame_check; per tile the segment is ordered
 * by (depth key, index).  Either output may be NULL. */
tg_status tg_frame_lists(tg_frame* frame, int32_t* tile_start, int32_t* sorted, int64_t n_keys,
                         void* stream);

/* Copies of the per-pixel state of the last forward into caller buffers
 * (device, enqueued on `stream`): T_final [H][W] float32 and last [H][W]
 * int32 (position in the pixel's tile list of the last blended Gaussian,
 * -1 if none).  Either output may be NULL. */
tg_status tg_frame_pixel_state(tg_frame* frame, float* T_final, int32_t* last, void* stream);

/* ------------------------------------------------ several target views
 * §4.2 renders the Gaussian set into the novel views of the user's left
 * and right eyes.  A frame created with max_views > 1 renders up to
 * max_views target cameras of one Gaussian set together: one projection
 * launch reads each Gaussian's 44 bytes once and writes its 2D state for
 * every view, the binning and sort run once over all views' tiles, and one
 * blend launch renders every view.  Each view's image is bit-identical to
 * rendering that camera alone.  The adjoint returns the gradients of the
 * sum of the views' losses (per Gaussian, the sum of its per-view
 * gradients). */

#define TG_MAX_VIEWS 8

/* As tg_frame_create, for up to max_views (1..TG_MAX_VIEWS) views of at
 * most max_n Gaussians and max_w x max_h pixels each; max_keys counts the
 * keys of all views together. */
tg_status tg_frame_create_views(tg_ctx* ctx, int32_t max_views, int64_t max_n, int32_t max_w,
                                int32_t max_h, int64_t max_keys, tg_frame** out);

/* Project g into n_views cameras (host array, 1..max_views).  tg_bin_sort
 * then bins every view; tg_frame_lists returns the lists of all views' tiles
 * (view v's tiles follow those of views 0..v-1); tg_frame_pixel_state
 * returns the views' pixel state one after another.  After a projection of
 * more than one view, use tg_render_fwd_views / tg_render_bwd_views
 * (tg_render_fwd and tg_render_bwd return TG_ERR_INVALID). */
tg_status tg_project_views(tg_frame* frame, const tg_gaussians* g, const tg_camera* cams /* host */,
                           int32_t n_views, void* stream);

/* Blend every view of the last tg_project_views: out_feat (host array of
 * n_views device pointers) [c][H_v][W_v], out_alpha (host array, or NULL)
 * [H_v][W_v] (entries may be NULL); bg [c] or NULL for every view. */
tg_status tg_render_fwd_views(tg_frame* frame, const tg_gaussians* g, const float* bg,
                              float* const* out_feat /* host */, float* const* out_alpha /* host */,
                              void* stream);

/* Adjoint of tg_render_fwd_views for the loss summed over the views:
 * d_feat (host array of device pointers) [c][H_v][W_v] per view, d_alpha
 * (host array or NULL; entries may be NULL) [H_v][W_v]; the gradients in
 * out are those of tg_render_bwd, summed over the views. */
tg_status tg_render_bwd_views(tg_frame* frame, const tg_gaussians* g, const float* bg,
                              const float* const* d_feat /* host */, const float* const* d_alpha /* host */,
                              const tg_grads* out, void* stream);

/* ------------------------------------------- render without allocating
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * render as tg_project + tg_bin_sort + tg_render_fwd on a frame (same
 * kernels, bit-identical results), with the workspace in a static device
 * array of TG_NOALLOC_SCRATCH_BYTES (150 MiB) instead of a tg_frame: no call
 * to hipMalloc, hipFree or any allocating routine.  Each device holds its
 * own array for the life of the process; tg_ctx_create resolves its address
 * on the context's device.  Limits: g->n <= TG_NOALLOC_MAX_N, width x height
 * <= TG_NOALLOC_MAX_PIXELS, ceil(W/16) x ceil(H/16) <= TG_NOALLOC_MAX_TILES
 * (TG_ERR_CAPACITY before anything is enqueued otherwise), and at most
 * TG_NOALLOC_MAX_KEYS (tile, Gaussian) keys: with more, the binning marks
 * the render, the outputs are not written and *status (a device int32,
 * optional) receives TG_ERR_CAPACITY, else TG_OK, once the stream reaches
 * that point.  Every call on a device shares that device's array: calls
 * that overlap on one device (two streams, two threads) race and must be
 * serialised by the caller.  Arguments as for tg_render_fwd; cam (host) as
 * for tg_project. */
#define TG_NOALLOC_MAX_N 524288
#define TG_NOALLOC_MAX_KEYS 2097152
#define TG_NOALLOC_MAX_PIXELS 1048576
#define TG_NOALLOC_MAX_TILES 8192
#define TG_NOALLOC_SCRATCH_BYTES 157680128
tg_status tg_render_noalloc(tg_ctx* ctx, const tg_gaussians* g, const tg_camera* cam, const float* bg,
                            float* out_feat, float* out_alpha, int32_t* status, void* stream);

/* ------------------------------------------------ lifting source views
 * The step upstream of the rasterizer, on the device.  §4.1 converts each
 * source view's disparity map to depth (a rectified pair of baseline B:
 * depth z = fx B / d for a disparity of d pixels); §4.2 unprojects the depth
 * maps with the camera parameters and makes every foreground pixel a
 * pixel-aligned Gaussian: position = the world point on the ray through the
 * pixel centre (i + 0.5, j + 0.5) at depth z, i.e. R^T (x_c - t) with
 * x_c = (z (i + 0.5 - cx) / fx, z (j + 0.5 - cy) / fy, z); feature, scale
 * and opacity = the encoder's maps at that pixel (Eq. 4); rotation = the
 * identity quaternion (1, 0, 0, 0).  A pixel is lifted when its mask byte is
 * non-zero and its disparity (or depth) is positive (NaN is not). */

#define TG_LIFT_MAX_VIEWS 8

/* One source view (host struct of device pointers).  cam is the source
 * camera (world -> camera, as tg_camera; width x height = the maps' size;
 * znear is not used).  Maps, row-major over pixels:
 *   disparity [H][W] float32 pixels, or NULL: then depth [H][W] (metres)
 *   mask      [H][W] uint8, foreground != 0
 *   feat      [H][W][c] float32 (channels last, 16-byte aligned)
 *   scale     [H][W][3] float32, activated
 *   opacity   [H][W] float32, activated
 * baseline: metres (> 0 when a disparity map is given). */
typedef struct tg_source_view {
  tg_camera cam;
  const float* disparity;
  const float* depth;
  const uint8_t* mask;
  const float* feat;
  const float* scale;
  const float* opacity;
  float baseline;
} tg_source_view;

/* Output buffers of a Gaussian set (host struct of device pointers), each
 * sized for cap Gaussians: mean [3][cap], scale [3][cap], quat [4][cap],
 * opacity [cap], feat [cap][c] (16-byte aligned).  A set of n <= cap
 * Gaussians is written in the layout of tg_gaussians with that n: mean
 * [3][n] occupies the first 3n floats, and so on. */
typedef struct tg_gaussian_buffers {
  float* mean;
  float* scale;
  float* quat;
  float* opacity;
  float* feat;
  int64_t cap;
} tg_gaussian_buffers;

typedef struct tg_lifter tg_lifter;

/* Workspace of the lifting for up to max_pixels source pixels per call (the
 * sum over its views).  Allocates device memory (TG_ERR_OOM). */
tg_status tg_lifter_create(tg_ctx* ctx, int64_t max_pixels, tg_lifter** out);
void tg_lifter_destroy(tg_lifter* lifter);

/* Lift n_views (1..TG_LIFT_MAX_VIEWS) source views (host array) with c
 * channels (8, 16, 32, 64) into out, in (view, row-major pixel) order.
 * n_out: device int64 that receives the number of lifted pixels n.  If
 * n > out->cap nothing is written to out (n_out still receives n).
 * Enqueue only; the caller reads *n_out after the stream reaches it and
 * passes it as tg_gaussians.n.  TG_ERR_CAPACITY (before anything is
 * enqueued) when the views hold more pixels than the lifter. */
tg_status tg_lift(tg_lifter* lifter, const tg_source_view* views /* host */, int32_t n_views,
                  int32_t c, const tg_gaussian_buffers* out /* host */, int64_t* n_out, void* stream);

/* ------------------------------------------------ z-buffer point splat
 * The cascaded disparity initialisation of §4.1 (Eq. 2-3): the point cloud
 * lifted from one source view's depth is rasterized into the viewpoints of
 * other cameras, and each z-buffer (the nearest depth per pixel) is
 * extracted and converted to a disparity map.  The paper gives no splat
 * size; here a point is a one-pixel splat: it lands in the pixel
 * (floor(u), floor(v)) containing its projection u = fx x_c / z_c + cx,
 * v = fy y_c / z_c + cy, and the pixel keeps the smallest view depth z_c.
 * Points with z_c <= znear or outside the image land nowhere.  Pixel and
 * depth follow a fixed float32 operation order (the view transform and
 * projection of the binning spec), so the z-buffer is reproducible bit for
 * bit and does not depend on the order of the points. */

#define TG_ZSPLAT_MAX_VIEWS 8

/* mean [3][n] float32 world points (for instance tg_lift's output); cams
 * (host) [n_views] target cameras (1..TG_ZSPLAT_MAX_VIEWS, znear >= 0);
 * zbuf: float32, the n_views planes [H_k][W_k] one after the other, +inf
 * where no point landed; disparity: NULL or float32 planes of the same
 * layout, fx_k B_k / z (rounded from FP64), 0 where no point landed, with
 * baselines (host) [n_views] in metres (may be NULL when disparity is).
 * Enqueue only, on the context's device. */
tg_status tg_zsplat(tg_ctx* ctx, const float* mean, int64_t n, const tg_camera* cams /* host */,
                    const float* baselines /* host */, int32_t n_views, float* zbuf, float* disparity,
                    void* stream);

/* ------------------------------------- occlusion-aware view blending
 * §4.3 gives the refiner a high-resolution image I_blend blended from the
 * source views (Eq. 6-10).  Per novel pixel (u, v) with fused depth z (the
 * source depth maps warped onto the novel view, for instance with
 * tg_zsplat of their lifted points): back-project the pixel centre to the
 * world point X (Eq. 6), project X into every source view, fetch colour,
 * depth, mask and normal there by bilinear sampling (Eq. 7), weigh view i
 * by w_i = M_i * Occ_i * max(0, -<r, n_i>) / |x_i^cam| (Eq. 8) with
 * Occ_i = 1 iff |x_i.z - z_i| < delta (Eq. 9), r the unit ray of the novel
 * pixel and n_i the sampled normal renormalised, and average the colours
 * with these weights (Eq. 10).  Readings where the paper is silent:
 * bilinear sampling between the four pixel centres around the point (the
 * top-left one clamped so all four lie in the view), only inside the
 * rectangle spanned by the view's pixel centres; the 0/1 mask is sampled
 * like the other maps; colours are 8-bit over 255.  Every quantity is FP64
 * in a fixed operation order, so the float32 outputs are reproducible bit
 * for bit. */

#define TG_BLEND_MAX_VIEWS 8

/* One source view of the blending (host struct of device pointers):
 *   rgba   [H][W][4] uint8 colour (alpha unused), 4-byte aligned
 *   depth  [H][W] float32 depth in metres (the view's predicted depth)
 *   mask   [H][W] uint8, M_i: non-zero where the view's pixels are valid
 *   normal [H][W][3] float32 world-frame unit normals (tg_depth_normals) */
typedef struct tg_blend_view {
  tg_camera cam;
  const uint8_t* rgba;
  const float* depth;
  const uint8_t* mask;
  const float* normal;
} tg_blend_view;

/* Unit normals [H][W][3] (world frame) of a depth map [H][W] seen by cam:
 * the cross product of the central differences of the unprojected pixel
 * centres P(i +- 1, j), P(i, j +- 1), turned toward the camera; 0 on the
 * border and where a depth of the five-point stencil is not positive. */
tg_status tg_depth_normals(tg_ctx* ctx, const tg_camera* cam /* host */, const float* depth, float* normal,
                           void* stream);

/* Blend n_views (0..TG_BLEND_MAX_VIEWS) source views (host array) into the
 * novel camera (host): z_fused [H][W] float32 (pixels whose depth is not
 * positive or infinite get nothing), delta > 0 in metres.  Outputs:
 * out_rgb [3][H][W] float32 in [0, 1] and out_wsum [H][W] float32, the sum
 * of the weights (0 where no view contributes; the colour is then 0). */
tg_status tg_blend_views(tg_ctx* ctx, const tg_blend_view* views /* host */, int32_t n_views,
                         const tg_camera* novel /* host */, const float* z_fused, float delta, float* out_rgb,
                         float* out_wsum, void* stream);

/* ------------------------------------------------------------------ serving
 * A request loop that renders many target views at once (the system of §5.3
 * renders every frame of every terminal through R_G, under CUDA Graphs).
 * Requests of uneven Gaussian counts and resolutions are admitted first in,
 * first out while the device bytes of the requests in flight stay within a
 * budget; whenever a slot is free, all admitted requests (up to max_batch)
 * form one batch that runs as a single persistent launch of every step,
 * replayed from a HIP graph captured once per slot.  Slots run on their own
 * streams, so a batch formed while others are on the GPU overlaps with
 * them.  Each request's result is the same as when rendered alone. */

typedef struct tg_serve_opts {
  int64_t budget_bytes;         /* device bytes the requests in flight may occupy */
  int32_t slots;                /* batches in flight at once (one HIP stream each), 1..8 */
  int32_t max_batch;            /* requests per batch, 1..64 */
  int64_t max_gauss_per_batch;  /* slot workspace: Gaussians (sum over the batch); rounded up
                                   to a multiple of 1024, plus 1024 per request of max_batch,
                                   at most 2^28 */
  int64_t max_keys_per_batch;   /* slot workspace: (tile, Gaussian) keys */
  int64_t max_pixels_per_batch; /* slot workspace: target pixels */
  int32_t max_side;             /* largest target width or height accepted */
  int32_t c;                    /* channel count of every request: 8, 16, 32 or 64 */
  int32_t use_graph;            /* 1: replay a captured HIP graph per slot; 0: launch directly */
  float keys_per_gaussian;      /* key estimate per Gaussian used for admission */
  int32_t batch_window_us;      /* a free slot waits up to this long after the oldest queued
                                   request arrived for more requests before it launches a
                                   batch of fewer than max_batch (0: launch at once), 0..1e6 */
  int32_t backward;             /* 1: slots also hold the adjoint's workspace and accept
                                   requests that carry an upstream gradient */
} tg_serve_opts;

/* One render request.  g points at device buffers that the caller keeps
 * resident (for instance the stream's arena from tg_serve_stream_arena) and
 * must not modify until the request is done; out_feat [c][H][W] and
 * out_alpha [H][W] (or NULL) are device buffers the caller owns.
 * Differentiation (§4.2 trains through R_G; a server created with backward
 * = 1): with d_feat [c][H][W] (and d_alpha [H][W] or NULL) the request also
 * runs the adjoint of its render in the same batch and writes the raw-
 * parameter gradients of tg_render_bwd into grads (d_feat required unless
 * g.n == 0, the others may be NULL); d_feat NULL renders only.
 * share = 1 lets the request reuse the projection and sorted tile lists of
 * an earlier request of the same batch and stream_id with the same n and
 * an identical camera (consecutive frames whose geometry did not change,
 * only their features).  The reuse is checked on the device: if any byte of
 * the two requests' mean, scale, quat or opacity differs, the request is
 * rendered again on its own (counted in tg_result.retries). */
typedef struct tg_request {
  int32_t stream_id;
  tg_gaussians g;
  tg_camera cam;
  const float* bg;              /* [c] or NULL */
  float* out_feat;
  float* out_alpha;
  const float* d_feat;          /* upstream gradient dL/dF or NULL */
  const float* d_alpha;         /* upstream gradient dL/dalpha or NULL */
  tg_grads grads;
  int32_t share;
} tg_request;

typedef struct tg_result {
  int32_t status;               /* TG_OK, TG_PENDING or an error code */
  int32_t batch_size;           /* requests in the batch that rendered it */
  int32_t slot;
  int32_t retries;              /* re-admissions (key-capacity overflow, geometry not shared) */
  int32_t shared;               /* 1: rendered with the projection and lists of an earlier request */
  int32_t pad;
  int64_t t_submit_ns;          /* host steady clock, nanoseconds */
  int64_t t_launch_ns;
  int64_t t_done_ns;            /* when the server observed completion */
} tg_result;

/* Create a server: allocates every slot's workspace, creates the slot
 * streams and, with use_graph, captures one graph per slot.  Starts the
 * scheduler thread. */
tg_status tg_serve_create(tg_ctx* ctx, const tg_serve_opts* opts /* host */, tg_server** out);

/* Device buffers for the Gaussians of stream `stream_id`, allocated on the
 * first call (max_n Gaussians, the server's c channels) and kept for the
 * server's lifetime; later calls return the same buffers (max_n must not
 * grow).  Their bytes count against the budget for as long as they exist.
 * *out (host) receives the pointers with n = max_n. */
tg_status tg_serve_stream_arena(tg_server* srv, int32_t stream_id, int64_t max_n,
                                tg_gaussians* out /* host */);

/* Thread-safe, non-blocking: queue a request; *ticket (host) identifies it.
 * TG_ERR_BUDGET if the request alone can never fit a slot or the budget. */
tg_status tg_serve_submit(tg_server* srv, const tg_request* req /* host */, uint64_t* ticket);

/* Non-blocking: TG_PENDING while queued or in flight, else the request's
 * final status; *out (host, may be NULL) receives its record.  A finished
 * ticket stays readable until tg_serve_release. */
tg_status tg_serve_poll(tg_server* srv, uint64_t ticket, tg_result* out);

/* Blocks until the ticket is finished; returns its final status
 * (TG_ERR_NOT_FOUND for an unknown ticket, or one that another caller
 * releases while this one waits). */
tg_status tg_serve_wait(tg_server* srv, uint64_t ticket, tg_result* out);

/* Forget a finished ticket (TG_PENDING, and nothing is forgotten, while it
 * is queued or in flight). */
tg_status tg_serve_release(tg_server* srv, uint64_t ticket);

/* Stops the scheduler after the requests in flight finish (queued requests
 * are dropped with TG_ERR_INVALID) and frees every resource. */
void tg_serve_destroy(tg_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* TG_H */
