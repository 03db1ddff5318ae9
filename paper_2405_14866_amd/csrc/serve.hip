// serve.hip -- the batched serving loop of include/tg.h (tg_serve_*).
//
// Continuous batching of render requests on one GPU:
//   * clients submit requests from any thread (a ticket per request); each
//     points at Gaussian buffers that stay resident on the device;
//   * a scheduler thread admits queued requests first in, first out while
//     the bytes of the requests in flight (workspace share + outputs) plus
//     the streams' resident arenas stay within the budget, and while the
//     slot's capacities (Gaussians, keys, tiles, pixels) hold;
//   * whenever a slot is free it forms a batch of everything admissible (up
//     to max_batch requests; with a batching window, a batch of fewer
//     waits until the oldest queued request is that old) and launches it: the request table goes to
//     the device by one pinned copy, then one launch per step (projection,
//     binning, sort, blend) covers every request of the batch - the kernels
//     read the table, their grids are the slot's capacity and the blend is a
//     persistent work-queue kernel over the batch's tiles.  With use_graph
//     that whole sequence is a HIP graph captured once per slot and
//     replayed per batch;
//   * slots run on separate streams, so a batch formed while others are on
//     the GPU overlaps with them on the device;
//   * a batch whose keys overflow the slot is re-admitted request by request
//     (a request that overflows alone fails with TG_ERR_CAPACITY);
//   * a request with an upstream gradient (a server created with backward)
//     also runs the adjoint in its batch: such batches replay a second graph
//     that appends the adjoint kernels, which skip the batch's forward-only
//     requests;
//   * a request marked share that repeats an earlier request of the batch
//     (same stream, n and camera) reads that request's projection and a copy
//     of its sorted tile lists instead of projecting and sorting again; a
//     kernel compares the two requests' geometry bytes and a request whose
//     geometry differs is re-admitted to render on its own.
// Latency of a request = completion observed by the scheduler - submit.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tg.h"
#include "serve_policy.h"
#include "tg_internal.h"

namespace tg {
int ctx_device(const tg_ctx* c);
}

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Ticket {
  tg_request req{};
  int32_t status = TG_PENDING;
  int32_t batch_size = 0, slot = -1, retries = 0;
  bool solo = false;             // re-admitted after an overflow: run alone
  bool no_share = false;         // re-admitted after a geometry mismatch: project and sort itself
  bool shared = false;           // rendered with an earlier request's projection and lists
  int64_t footprint = 0;
  int64_t t_submit = 0, t_launch = 0, t_done = 0;
};

struct Arena {
  float* mean = nullptr;
  float* scale = nullptr;
  float* quat = nullptr;
  float* opacity = nullptr;
  float* feat = nullptr;
  int64_t max_n = 0;
  int64_t bytes = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // workspace
  double2* xy = nullptr;
  float4* conic_o = nullptr;
  float4* wq = nullptr;
  float4* ext = nullptr;
  uint2* rect = nullptr;
  uint32_t* depth = nullptr;
  int32_t* tile_count = nullptr;
  int32_t* tile_start = nullptr;
  int32_t* tile_cursor = nullptr;
  int32_t* tile_order = nullptr;
  uint64_t* keys = nullptr;
  uint64_t* keys_tmp = nullptr;
  int32_t* sorted = nullptr;
  int2* qlist = nullptr;
  int32_t* qcount = nullptr;
  int32_t* qcut = nullptr;
  float* T_final = nullptr;
  int32_t* last = nullptr;
  float* g2d = nullptr;
  tg::FrameDev* dev = nullptr;
  tg::ReqDev* table_dev = nullptr;
  tg::BatchHdr* hdr_dev = nullptr;
  // pinned host mirrors
  tg::ReqDev* table_host = nullptr;
  tg::BatchHdr* hdr_host = nullptr;
  tg::FrameDev* dev_host = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_fb = nullptr;       // forward + adjoint
  hipGraphExec_t exec_fb = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
};

template <class T>
bool dalloc(T** p, size_t count) {
  *p = nullptr;
  return hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T)) == hipSuccess;
}
template <class T>
bool halloc(T** p, size_t count) {
  *p = nullptr;
  return hipHostMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T), 0) == hipSuccess;
}

}  // namespace

struct tg_server {
  tg_ctx* ctx = nullptr;
  int device = 0;
  tg_serve_opts opts{};
  int64_t cap_gauss = 0, cap_keys = 0, cap_pixels = 0;
  int32_t cap_tiles = 0, max_tiles_req = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;        // wakes the scheduler
  std::condition_variable done_cv;   // wakes tg_serve_wait
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::unordered_map<int32_t, Arena> arenas;
  uint64_t next_ticket = 1;
  int64_t budget_used = 0;            // arenas + requests in flight
  int64_t arena_bytes = 0;            // arenas alone (held for the server's lifetime)
  bool stop = false;
  std::thread sched;
  bool failed = false;               // a HIP error stopped the scheduler
};

namespace {

int32_t tiles_of(const tg_camera& c) {
  return ((c.width + tg::TILE - 1) / tg::TILE) * ((c.height + tg::TILE - 1) / tg::TILE);
}

int64_t keys_est(const tg_server* s, int64_t n) {
  return (int64_t)((double)n * s->opts.keys_per_gaussian) + 1024;
}

// device bytes a request occupies while in flight: its share of the slot
// workspace (with the adjoint's accumulators when it asks for gradients)
// and its outputs
int64_t footprint_of(const tg_server* s, const tg_request& r) {
  const int64_t px = (int64_t)r.cam.width * r.cam.height;
  const int64_t per_g = r.d_feat ? 76 + 24 : 76;
  // per key: key, scratch key, sorted index and room for four quadrant entries (52 B)
  return tg::padded(r.g.n) * per_g + keys_est(s, r.g.n) * 52 + px * (8 + 4 * ((int64_t)s->opts.c + 1));
}

// Clear the per-batch device flags.
__global__ void k_batch_reset(tg::FrameDev* d) { d->geom_mismatch = 0ull; }

// Byte comparison of the geometry of every sharing request with its
// source's (mean, scale, quat, opacity; n is equal by admission): bit r of
// geom_mismatch is set when request r's geometry differs.
__global__ void __launch_bounds__(256) k_geom_check(tg::BatchArgs a) {
  const tg::BatchHdr h = tg::batch_hdr(a);
  if (h.n_shared == 0) return;
  for (int r = 0; r < h.n_req; ++r) {
    const tg::ReqDev& q = a.table[r];
    if (q.src == 0) continue;
    const tg::ReqDev& p = a.table[q.src - 1];
    const int64_t n = q.n;
    bool diff = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        diff |= __float_as_uint(q.mean[k * n + i]) != __float_as_uint(p.mean[k * n + i]);
        diff |= __float_as_uint(q.scale[k * n + i]) != __float_as_uint(p.scale[k * n + i]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) diff |= __float_as_uint(q.quat[k * n + i]) != __float_as_uint(p.quat[k * n + i]);
      diff |= __float_as_uint(q.opacity[i]) != __float_as_uint(p.opacity[i]);
    }
    if (__syncthreads_or(diff) && threadIdx.x == 0) atomicOr(&a.dev->geom_mismatch, 1ull << r);
  }
}

tg::BatchArgs slot_args(const tg_server* s, const Slot& sl) {
  tg::BatchArgs b{};
  b.table = sl.table_dev;
  b.hdr_dev = sl.hdr_dev;
  b.xy = sl.xy;
  b.conic_o = sl.conic_o;
  b.wq = sl.wq;
  b.ext = sl.ext;
  b.rect = sl.rect;
  b.depth = sl.depth;
  b.tile_count = sl.tile_count;
  b.tile_start = sl.tile_start;
  b.tile_cursor = sl.tile_cursor;
  b.tile_order = sl.tile_order;
  b.keys = sl.keys;
  b.keys_tmp = sl.keys_tmp;
  b.sorted = sl.sorted;
  b.qlist = sl.qlist;
  b.qcount = sl.qcount;
  b.qcut = sl.qcut;
  b.g2d = sl.g2d;
  b.g_cap = s->cap_gauss;
  b.key_cap = s->cap_keys;
  b.dev = sl.dev;
  return b;
}

// the batch's work on the slot stream: table upload, every step (and the
// adjoint with `backward`), status download
hipError_t enqueue_batch(const tg_server* s, const Slot& sl, bool backward) {
  hipError_t e;
  if ((e = hipMemcpyAsync(sl.table_dev, sl.table_host, sizeof(tg::ReqDev) * tg::MAX_BATCH,
                          hipMemcpyHostToDevice, sl.stream)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(sl.hdr_dev, sl.hdr_host, sizeof(tg::BatchHdr), hipMemcpyHostToDevice,
                          sl.stream)) != hipSuccess)
    return e;
  const tg::BatchArgs a = slot_args(s, sl);
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, sl.stream, sl.dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_geom_check, dim3(1024), dim3(256), 0, sl.stream, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = tg::launch_project(a, s->cap_gauss, sl.stream)) != hipSuccess) return e;
  if ((e = tg::launch_bin_sort(a, s->cap_gauss, s->cap_tiles, s->max_tiles_req, sl.stream)) != hipSuccess)
    return e;
  if ((e = tg::launch_render_fwd(a, s->opts.c, s->cap_tiles, sl.stream)) != hipSuccess) return e;
  if (backward && (e = tg::launch_render_bwd(a, s->opts.c, s->cap_gauss, s->cap_tiles, sl.stream)) != hipSuccess)
    return e;
  return hipMemcpyAsync(sl.dev_host, sl.dev, sizeof(tg::FrameDev), hipMemcpyDeviceToHost, sl.stream);
}

// capture one batch sequence into a graph (replays read the table the first node uploads)
bool capture(const tg_server* s, Slot& sl, bool backward, hipGraph_t* graph, hipGraphExec_t* exec) {
  if (hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  const hipError_t e = enqueue_batch(s, sl, backward);
  hipGraph_t gr = nullptr;
  const hipError_t e2 = hipStreamEndCapture(sl.stream, &gr);
  if (e != hipSuccess || e2 != hipSuccess || !gr) {
    if (gr) (void)hipGraphDestroy(gr);
    return false;
  }
  *graph = gr;
  return hipGraphInstantiate(exec, gr, nullptr, nullptr, 0) == hipSuccess;
}

void free_slot(Slot& sl) {
  if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
  if (sl.graph) (void)hipGraphDestroy(sl.graph);
  if (sl.exec_fb) (void)hipGraphExecDestroy(sl.exec_fb);
  if (sl.graph_fb) (void)hipGraphDestroy(sl.graph_fb);
  void* d[] = {sl.xy, sl.conic_o, sl.wq, sl.ext, sl.rect, sl.depth, sl.tile_count, sl.tile_start, sl.tile_cursor,
               sl.tile_order,
               sl.keys, sl.keys_tmp, sl.sorted, sl.qlist, sl.qcount, sl.qcut, sl.T_final, sl.last, sl.g2d, sl.dev,
               sl.table_dev,
               sl.hdr_dev};
  for (void* p : d)
    if (p) (void)hipFree(p);
  void* h[] = {sl.table_host, sl.hdr_host, sl.dev_host};
  for (void* p : h)
    if (p) (void)hipHostFree(p);
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  sl = Slot{};
}

bool alloc_slot(tg_server* s, Slot& sl) {
  const size_t g = (size_t)s->cap_gauss, k = (size_t)s->cap_keys, t = (size_t)s->cap_tiles,
               px = (size_t)s->cap_pixels;
  bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
            dalloc(&sl.xy, g) && dalloc(&sl.conic_o, g) && dalloc(&sl.wq, g) && dalloc(&sl.ext, g) &&
            dalloc(&sl.rect, g) && dalloc(&sl.depth, g) &&
            dalloc(&sl.tile_count, t) && dalloc(&sl.tile_start, t + 1) && dalloc(&sl.tile_cursor, t) &&
            dalloc(&sl.tile_order, t) &&
            dalloc(&sl.keys, k) && dalloc(&sl.keys_tmp, k) && dalloc(&sl.sorted, k) &&
            dalloc(&sl.qlist, 4 * k) && dalloc(&sl.qcount, 4 * t) && dalloc(&sl.qcut, 4 * t) &&
            dalloc(&sl.T_final, px) && dalloc(&sl.last, px) &&
            dalloc(&sl.g2d, s->opts.backward ? 8 * g : 1) && dalloc(&sl.dev, 1) &&
            dalloc(&sl.table_dev, tg::MAX_BATCH) && dalloc(&sl.hdr_dev, 1) &&
            halloc(&sl.table_host, tg::MAX_BATCH) && halloc(&sl.hdr_host, 1) && halloc(&sl.dev_host, 1);
  if (!ok) return false;
  ok = hipMemset(sl.dev, 0, sizeof(tg::FrameDev)) == hipSuccess &&
       hipMemset(sl.table_dev, 0, sizeof(tg::ReqDev) * tg::MAX_BATCH) == hipSuccess &&
       hipMemset(sl.hdr_dev, 0, sizeof(tg::BatchHdr)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) return false;
  std::fill_n(reinterpret_cast<char*>(sl.table_host), sizeof(tg::ReqDev) * tg::MAX_BATCH, 0);
  *sl.hdr_host = tg::BatchHdr{};
  if (s->opts.use_graph) {
    // capture the batch sequences once
    if (!capture(s, sl, false, &sl.graph, &sl.exec)) return false;
    if (s->opts.backward && !capture(s, sl, true, &sl.graph_fb, &sl.exec_fb)) return false;
  }
  return true;
}

// Form and launch one batch on a free slot.  Called with the lock held.
// Returns false if nothing could be admitted.
bool launch_batch(tg_server* s, int slot_id) {
  Slot& sl = s->slots[slot_id];
  const tg::policy::Limits lim{s->opts.max_batch, s->cap_gauss, s->cap_keys, s->cap_pixels, s->cap_tiles,
                               s->opts.budget_bytes};
  std::vector<uint64_t> batch = tg::policy::form_batch(
      s->queue,
      [&](uint64_t id) {
        const Ticket& t = s->tickets[id];
        return tg::policy::Demand{tg::padded(t.req.g.n), keys_est(s, t.req.g.n),
                                  (int64_t)t.req.cam.width * t.req.cam.height, tiles_of(t.req.cam), t.footprint,
                                  t.solo};
      },
      lim, s->budget_used);
  int64_t sum_g = 0, sum_px = 0;
  int32_t sum_t = 0, n_shared = 0;
  bool backward = false;
  for (size_t b = 0; b < batch.size(); ++b) {
    Ticket& t = s->tickets[batch[b]];
    const int64_t ng = tg::padded(t.req.g.n);
    const int64_t npx = (int64_t)t.req.cam.width * t.req.cam.height;
    const int32_t nt = tiles_of(t.req.cam);
    tg::ReqDev& r = sl.table_host[b];
    r = tg::ReqDev{};
    r.mean = t.req.g.mean; r.scale = t.req.g.scale; r.quat = t.req.g.quat;
    r.opacity = t.req.g.opacity; r.feat = t.req.g.feat;
    r.bg = t.req.bg; r.out_feat = t.req.out_feat; r.out_alpha = t.req.out_alpha;
    r.T_final = sl.T_final + sum_px;
    r.last = sl.last + sum_px;
    r.n = t.req.g.n;
    r.g_off = sum_g;
    r.s_off = sum_g;
    r.tile_off = sum_t;
    r.d_img = t.req.d_feat;
    r.d_alpha = t.req.d_alpha;
    r.d_mean = t.req.grads.d_mean;
    r.d_log_scale = t.req.grads.d_log_scale;
    r.d_quat = t.req.grads.d_quat;
    r.d_logit = t.req.grads.d_opacity_logit;
    r.d_feat = t.req.grads.d_feat;
    backward = backward || t.req.d_feat != nullptr;
    // reuse of an earlier request's projection and lists: same stream, n and camera
    t.shared = false;
    if (t.req.share && !t.no_share && t.req.g.n > 0) {
      for (size_t p = 0; p < b; ++p) {
        const Ticket& o = s->tickets[batch[p]];
        const tg::ReqDev& src = sl.table_host[p];
        if (src.src == 0 && o.req.stream_id == t.req.stream_id && o.req.g.n == t.req.g.n &&
            std::memcmp(&o.req.cam, &t.req.cam, sizeof(tg_camera)) == 0) {
          r.src = (int32_t)p + 1;
          r.s_off = src.g_off;
          t.shared = true;
          ++n_shared;
          break;
        }
      }
    }
    tg::CamArgs& c = r.cam;
    for (int i = 0; i < 9; ++i) c.R[i] = t.req.cam.R[i];
    for (int i = 0; i < 3; ++i) c.t[i] = t.req.cam.t[i];
    c.fx = t.req.cam.fx; c.fy = t.req.cam.fy; c.cx = t.req.cam.cx; c.cy = t.req.cam.cy;
    c.znear = t.req.cam.znear;
    c.W = t.req.cam.width; c.H = t.req.cam.height;
    c.tiles_x = (c.W + tg::TILE - 1) / tg::TILE;
    c.tiles_y = (c.H + tg::TILE - 1) / tg::TILE;
    sum_g += ng; sum_px += npx; sum_t += nt;
  }
  if (batch.empty()) return false;
  *sl.hdr_host = tg::BatchHdr{(int32_t)batch.size(), sum_t, sum_g, n_shared, 0};
  const int64_t t0 = now_ns();
  hipError_t e = hipSuccess;
  if (s->opts.use_graph) e = hipGraphLaunch(backward ? sl.exec_fb : sl.exec, sl.stream);
  else e = enqueue_batch(s, sl, backward);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  for (uint64_t id : batch) {
    Ticket& t = s->tickets[id];
    t.t_launch = t0;
    t.slot = slot_id;
    t.batch_size = (int32_t)batch.size();
    if (e != hipSuccess) {
      t.status = TG_ERR_HIP;
      t.t_done = now_ns();
      s->budget_used -= t.footprint;
    }
  }
  if (e != hipSuccess) {
    s->failed = true;
    s->done_cv.notify_all();
    return false;
  }
  sl.tickets = std::move(batch);
  sl.busy = true;
  return true;
}

// Retire a finished slot.  Called with the lock held.
void finish_slot(tg_server* s, Slot& sl) {
  const bool over = sl.dev_host->overflow != 0;
  const unsigned long long mismatch = sl.dev_host->geom_mismatch;
  const int64_t t1 = now_ns();
  std::vector<uint64_t> retry;
  for (size_t k = 0; k < sl.tickets.size(); ++k) {
    const uint64_t id = sl.tickets[k];
    Ticket& t = s->tickets[id];
    s->budget_used -= t.footprint;
    switch (tg::policy::retire(over, sl.tickets.size(), ((mismatch >> k) & 1ull) != 0)) {
      case tg::policy::Outcome::RetrySolo:
        t.retries += 1;
        t.solo = true;
        retry.push_back(id);
        break;
      case tg::policy::Outcome::RetryNoShare:   // its geometry differs from the request it shared
        t.retries += 1;
        t.no_share = true;
        retry.push_back(id);
        break;
      case tg::policy::Outcome::Capacity:
        t.status = TG_ERR_CAPACITY;
        t.t_done = t1;
        break;
      case tg::policy::Outcome::Done:
        t.status = TG_OK;
        t.t_done = t1;
        break;
    }
  }
  tg::policy::requeue(s->queue, retry);
  sl.tickets.clear();
  sl.busy = false;
  s->done_cv.notify_all();
}

void scheduler(tg_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool any_busy = false;
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) finish_slot(s, sl);
      else if (q == hipErrorNotReady) any_busy = true;
      else {   // device error: fail the slot's requests
        for (uint64_t id : sl.tickets) {
          Ticket& t = s->tickets[id];
          t.status = TG_ERR_HIP;
          t.t_done = now_ns();
          s->budget_used -= t.footprint;
        }
        sl.tickets.clear();
        sl.busy = false;
        s->failed = true;
        s->done_cv.notify_all();
      }
    }
    // batching window: while fewer than max_batch requests are queued, hold
    // them until the oldest has waited batch_window_us
    bool hold = false;
    int64_t deadline = 0;
    if (!s->queue.empty()) {
      const Ticket& front = s->tickets[s->queue.front()];
      deadline = front.t_submit + (int64_t)s->opts.batch_window_us * 1000;
      hold = tg::policy::holds(s->queue.size(), s->opts.max_batch, s->opts.batch_window_us, front.t_submit,
                               front.solo, now_ns());
    }
    if (!s->stop && !s->failed && !hold) {
      for (size_t i = 0; i < s->slots.size() && !s->queue.empty(); ++i)
        if (!s->slots[i].busy && launch_batch(s, (int)i)) any_busy = true;
    }
    if (s->stop || s->failed) {
      if (!any_busy) break;
    }
    if (any_busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else if (hold && !s->stop && !s->failed) {
      // woken early by a submit; the loop re-evaluates the window
      s->cv.wait_until(lk, std::chrono::steady_clock::time_point(std::chrono::nanoseconds(deadline)));
    } else {
      s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    }
  }
  // drop whatever is still queued
  for (uint64_t id : s->queue) {
    Ticket& t = s->tickets[id];
    t.status = s->failed ? TG_ERR_HIP : TG_ERR_INVALID;
    t.t_done = now_ns();
  }
  s->queue.clear();
  s->done_cv.notify_all();
}

}  // namespace

extern "C" {

tg_status tg_serve_create(tg_ctx* ctx, const tg_serve_opts* opts, tg_server** out) {
  if (!ctx || !opts || !out) return TG_ERR_INVALID;
  *out = nullptr;
  const tg_serve_opts& o = *opts;
  if (o.slots < 1 || o.slots > 8 || o.max_batch < 1 || o.max_batch > tg::MAX_BATCH ||
      o.max_gauss_per_batch < 1 || o.max_keys_per_batch < 1 || o.max_keys_per_batch >= ((int64_t)1 << 31) ||
      o.max_pixels_per_batch < 1 || o.max_side < 1 || o.max_side > 65535 * tg::TILE || o.budget_bytes <= 0 ||
      !(o.c == 8 || o.c == 16 || o.c == 32 || o.c == 64) || !(o.keys_per_gaussian > 0.f) ||
      o.batch_window_us < 0 || o.batch_window_us > 1000000 || (o.backward != 0 && o.backward != 1) ||
      o.max_gauss_per_batch >= tg::MAX_GAUSS_SPACE ||
      tg::padded(o.max_gauss_per_batch) + (int64_t)o.max_batch * tg::BIN_CHUNK > tg::MAX_GAUSS_SPACE)
    return TG_ERR_INVALID;
  const int device = tg::ctx_device(ctx);
  if (hipSetDevice(device) != hipSuccess) return TG_ERR_HIP;
  tg_server* s = new (std::nothrow) tg_server;
  if (!s) return TG_ERR_OOM;
  s->ctx = ctx;
  s->device = device;
  s->opts = o;
  s->cap_gauss = tg::padded(o.max_gauss_per_batch) + (int64_t)o.max_batch * tg::BIN_CHUNK;
  s->cap_keys = o.max_keys_per_batch;
  s->cap_pixels = o.max_pixels_per_batch;
  const int64_t side_tiles = (o.max_side + tg::TILE - 1) / tg::TILE;
  s->max_tiles_req = (int32_t)std::min<int64_t>(side_tiles * side_tiles, tg::BIN_LDS_MAX_TILES);
  s->cap_tiles = (int32_t)(o.max_pixels_per_batch / (tg::TILE * tg::TILE) + (int64_t)o.max_batch * (2 * side_tiles + 1));
  s->slots.resize(o.slots);
  for (Slot& sl : s->slots) {
    if (!alloc_slot(s, sl)) {
      for (Slot& x : s->slots) free_slot(x);
      delete s;
      return TG_ERR_OOM;
    }
  }
  s->sched = std::thread(scheduler, s);
  *out = s;
  return TG_OK;
}

tg_status tg_serve_stream_arena(tg_server* s, int32_t stream_id, int64_t max_n, tg_gaussians* out) {
  if (!s || !out || max_n < 1) return TG_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->arenas.find(stream_id);
  if (it == s->arenas.end()) {
    const int64_t bytes = max_n * (44 + 4 * (int64_t)s->opts.c);
    if (s->budget_used + bytes > s->opts.budget_bytes) return TG_ERR_BUDGET;
    if (hipSetDevice(s->device) != hipSuccess) return TG_ERR_HIP;
    Arena a;
    a.max_n = max_n;
    a.bytes = bytes;
    if (!dalloc(&a.mean, 3 * max_n) || !dalloc(&a.scale, 3 * max_n) || !dalloc(&a.quat, 4 * max_n) ||
        !dalloc(&a.opacity, max_n) || !dalloc(&a.feat, max_n * s->opts.c)) {
      float* p[] = {a.mean, a.scale, a.quat, a.opacity, a.feat};
      for (float* x : p)
        if (x) (void)hipFree(x);
      return TG_ERR_OOM;
    }
    s->budget_used += bytes;
    s->arena_bytes += bytes;
    it = s->arenas.emplace(stream_id, a).first;
  } else if (max_n > it->second.max_n) {
    return TG_ERR_INVALID;
  }
  const Arena& a = it->second;
  out->mean = a.mean; out->scale = a.scale; out->quat = a.quat; out->opacity = a.opacity; out->feat = a.feat;
  out->n = a.max_n;
  out->c = s->opts.c;
  return TG_OK;
}

tg_status tg_serve_submit(tg_server* s, const tg_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return TG_ERR_INVALID;
  const tg_gaussians& g = req->g;
  if (g.c != s->opts.c || g.n < 0 || (g.n > 0 && (!g.mean || !g.scale || !g.quat || !g.opacity || !g.feat)) ||
      !req->out_feat || req->cam.width <= 0 || req->cam.height <= 0 || req->cam.width > s->opts.max_side ||
      req->cam.height > s->opts.max_side)
    return TG_ERR_INVALID;
  // an adjoint needs a server built for it, and feature gradients unless the set is empty
  if (req->d_feat && (!s->opts.backward || (g.n > 0 && !req->grads.d_feat))) return TG_ERR_INVALID;
  Ticket t;
  t.req = *req;
  t.footprint = footprint_of(s, *req);
  t.t_submit = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop || s->failed) return TG_ERR_INVALID;
  if (tg::padded(g.n) > s->cap_gauss || (int64_t)req->cam.width * req->cam.height > s->cap_pixels ||
      tiles_of(req->cam) > s->cap_tiles || t.footprint + s->arena_bytes > s->opts.budget_bytes)
    return TG_ERR_BUDGET;
  const uint64_t id = s->next_ticket++;
  s->tickets.emplace(id, t);
  s->queue.push_back(id);
  *ticket = id;
  s->cv.notify_one();
  return TG_OK;
}

static void fill_result(const Ticket& t, tg_result* out) {
  if (!out) return;
  out->status = t.status;
  out->batch_size = t.batch_size;
  out->slot = t.slot;
  out->retries = t.retries;
  out->shared = t.shared ? 1 : 0;
  out->pad = 0;
  out->t_submit_ns = t.t_submit;
  out->t_launch_ns = t.t_launch;
  out->t_done_ns = t.t_done;
}

tg_status tg_serve_poll(tg_server* s, uint64_t ticket, tg_result* out) {
  if (!s) return TG_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return TG_ERR_NOT_FOUND;
  fill_result(it->second, out);
  return (tg_status)it->second.status;
}

tg_status tg_serve_wait(tg_server* s, uint64_t ticket, tg_result* out) {
  if (!s) return TG_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return TG_ERR_NOT_FOUND;
  // another caller may release the ticket while this one waits: look it up
  // afresh on every wake-up (operator[] would re-create it as pending)
  const Ticket* t = nullptr;
  s->done_cv.wait(lk, [&] {
    auto j = s->tickets.find(ticket);
    t = j == s->tickets.end() ? nullptr : &j->second;
    return !t || t->status != TG_PENDING;
  });
  if (!t) return TG_ERR_NOT_FOUND;
  fill_result(*t, out);
  return (tg_status)t->status;
}

tg_status tg_serve_release(tg_server* s, uint64_t ticket) {
  if (!s) return TG_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return TG_ERR_NOT_FOUND;
  if (it->second.status == TG_PENDING) return TG_PENDING;
  s->tickets.erase(it);
  return TG_OK;
}

void tg_serve_destroy(tg_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (Slot& sl : s->slots) free_slot(sl);
  for (auto& kv : s->arenas) {
    float* p[] = {kv.second.mean, kv.second.scale, kv.second.quat, kv.second.opacity, kv.second.feat};
    for (float* x : p)
      if (x) (void)hipFree(x);
  }
  delete s;
}

}  // extern "C"
