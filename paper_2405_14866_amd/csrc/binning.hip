// binning.hip -- step 2 of the rasterizer: (tile, Gaussian) keys grouped by
// tile and sorted by (view depth, index) inside each tile (gfx950).
//
// The order the blend needs is ascending (tile, depth key, Gaussian index).
// It is produced as a most-significant-digit split on the tile followed by
// an LDS radix sort of each tile's segment:
//
//   k_count  per workgroup of 1024 Gaussians, count keys per tile in LDS
//            (ds_add), then one global atomic per (workgroup, touched tile);
//   k_scan   one workgroup: exclusive scan of the tile counts -> segment
//            offsets; the key total is checked against the frame capacity
//            on the device (no host round trip); a counting sort of the
//            tiles by descending key count (buckets of 32 keys) gives the
//            order in which the sort, the blend and its adjoint take tiles,
//            longest first, so that the last tiles to start are short ones;
//   k_fill   same LDS binning, then one global atomic per (workgroup, tile)
//            reserves a contiguous run of the tile's segment and LDS
//            atomics hand out slots inside it; each slot receives the 64-bit
//            key (depth << 32) | (quadrant mask << 28) | index, the mask
//            holding the 8x8 quadrants of the tile that the Gaussian's alpha
//            support can reach (the blend's conservative quadrant test,
//            taken here while the Gaussian's mean and extents are in
//            registers; indices stay below 2^28).  The order inside a
//            segment is not deterministic here; the sort makes it so;
//   k_sort   one 256-lane workgroup per tile, tiles taken longest first
//            (the scan's order): the segment is loaded eight keys per lane
//            (all loads in flight at once) and stays in those registers
//            while it is ordered on the top 16 bits of the depth re-based
//            to the segment's minimum: a 10-bit pass that needs no
//            stability (LDS atomics hand out slots) straight from the
//            registers into one LDS buffer, then a stable 6-bit pass
//            (each wave ranks its contiguous range by ballot matching and
//            a running count per digit, then scatters in place); runs of
//            keys equal in those bits (a few keys: ~750 keys over 65,536
//            bins) are then ordered by the whole (depth, index) key, one
//            lane per run, and only a run longer than 32 sends the tile to
//            a sort on the composite (depth - min, index - min) key.
//            Either way the result is the unique (depth, index) order.
//            Segments up to 2048 keys run in a launch with one workgroup
//            per tile and 22 KB of LDS (six workgroups per CU), larger ones
//            in a second launch with 64 KB whose small grid walks the head
//            of the tile order, and beyond 8192 keys (or with a too long
//            run) on global scratch buffers.  The sorted segment is
//            written as the tile's index list and, from the same registers,
//            split into four quadrant lists: entry j goes to the list of
//            each quadrant its key's mask holds, in list order, as
//            (index, j); the forward blend walks one quadrant per wave.
//
// Compared with a global LSD sort of all K keys (4-6 passes of K x 12-24 B
// over HBM plus a launch per pass), the keys cross HBM about three times.
#include "blend_common.h"

namespace tg {
namespace {

// low half of a key: quadrant mask in bits 28..31, Gaussian index below
constexpr int KEY_MASK_SHIFT = 28;
constexpr uint32_t KEY_INDEX = (1u << KEY_MASK_SHIFT) - 1u;
static_assert(MAX_GAUSS_SPACE <= ((int64_t)1 << KEY_MASK_SHIFT), "indices fit below the quadrant mask");

__device__ __forceinline__ void rect_of(uint2 r, int& x0, int& x1, int& y0, int& y1) {
  x0 = (int)(r.x & 0xffffu); x1 = (int)(r.x >> 16);
  y0 = (int)(r.y & 0xffffu); y1 = (int)(r.y >> 16);
}

// The workgroup's request: chunk [g0, g0 + BIN_CHUNK) of the padded index space.
struct ChunkReq {
  int r;
  int64_t i0, i1;      // local Gaussian range of the chunk
  int64_t g_off;
  int tiles_x, n_tiles, tile_off;
};

__device__ __forceinline__ bool chunk_req(const BatchArgs& a, const BatchHdr& h, ChunkReq& c) {
  const int64_t g0 = (int64_t)blockIdx.x * BIN_CHUNK;
  c.r = req_of_gauss(a, h, g0);
  if (c.r < 0) return false;
  const ReqDev& q = batch_req(a, c.r);
  if (q.src != 0) return false;       // a sharing request bins nothing of its own
  c.g_off = q.g_off;
  c.i0 = g0 - q.g_off;
  c.i1 = min(q.n, c.i0 + BIN_CHUNK);
  c.tiles_x = q.cam.tiles_x;
  c.n_tiles = q.cam.tiles_x * q.cam.tiles_y;
  c.tile_off = q.tile_off;
  return c.i0 < c.i1;
}

// Per-tile key counts of one chunk: LDS counters for the request's tiles
// (when they fit), then one global atomic per touched tile.
__global__ void __launch_bounds__(1024) k_count(BatchArgs a) {
  extern __shared__ int32_t bins[];
  const BatchHdr h = batch_hdr(a);
  ChunkReq c;
  if (!chunk_req(a, h, c)) return;
  const int tid = threadIdx.x;
  const bool lds = c.n_tiles <= BIN_LDS_MAX_TILES;
  int32_t* gcount = a.tile_count + c.tile_off;
  if (lds) {
    for (int t = tid; t < c.n_tiles; t += 1024) bins[t] = 0;
    __syncthreads();
  }
  for (int64_t i = c.i0 + tid; i < c.i1; i += 1024) {
    int x0, x1, y0, y1;
    rect_of(a.rect[c.g_off + i], x0, x1, y0, y1);
    for (int ty = y0; ty <= y1; ++ty)
      for (int tx = x0; tx <= x1; ++tx) {
        const int t = ty * c.tiles_x + tx;
        if (lds) atomicAdd(&bins[t], 1);
        else atomicAdd(&gcount[t], 1);
      }
  }
  if (lds) {
    __syncthreads();
    for (int t = tid; t < c.n_tiles; t += 1024) {
      const int v = bins[t];
      if (v) atomicAdd(&gcount[t], v);
    }
  }
}

// Tiles of a request that shares an earlier request's projection take that
// request's key counts (so the scan reserves their segments and orders
// them by length like any other tile).
__global__ void __launch_bounds__(256) k_share_count(BatchArgs a) {
  const BatchHdr h = batch_hdr(a);
  if (h.n_shared == 0) return;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < h.n_tiles; t += gridDim.x * 256) {
    const int r = req_of_tile(a, h, t);
    if (r < 0) continue;
    const ReqDev& q = batch_req(a, r);
    if (q.src == 0) continue;
    a.tile_count[t] = a.tile_count[batch_req(a, q.src - 1).tile_off + (t - q.tile_off)];
  }
}

// ... and, once the source's segments are sorted, copies of them.
__global__ void __launch_bounds__(256) k_share_copy(BatchArgs a) {
  if (a.dev->overflow) return;
  const BatchHdr h = batch_hdr(a);
  if (h.n_shared == 0) return;
  for (int t = blockIdx.x; t < h.n_tiles; t += gridDim.x) {
    const int r = req_of_tile(a, h, t);
    if (r < 0) continue;
    const ReqDev& q = batch_req(a, r);
    if (q.src == 0) continue;
    const int ts = batch_req(a, q.src - 1).tile_off + (t - q.tile_off);
    const int d = a.tile_start[t], n = a.tile_start[t + 1] - d, sidx = a.tile_start[ts];
    for (int j = threadIdx.x; j < n; j += 256) a.sorted[d + j] = a.sorted[sidx + j];
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const int qn = a.qcount[4 * ts + qd];
      const int2* src = a.qlist + 4 * (int64_t)sidx + (int64_t)qd * n;
      int2* dst = a.qlist + 4 * (int64_t)d + (int64_t)qd * n;
      for (int j = threadIdx.x; j < qn; j += 256) dst[j] = src[j];
    }
    if (threadIdx.x < 4) a.qcount[4 * t + threadIdx.x] = a.qcount[4 * ts + threadIdx.x];
  }
}

// exclusive scan of the batch's tile counts (one workgroup of 1024 lanes)
constexpr int ORDER_BUCKETS = 64;       // key-count buckets of the tile order
constexpr int ORDER_SHIFT = 5;          // 32 keys per bucket

__device__ __forceinline__ int order_bucket(int32_t count) {
  return ORDER_BUCKETS - 1 - min(count >> ORDER_SHIFT, ORDER_BUCKETS - 1);
}

// inclusive scan over the 64 lanes of a wave
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// The scan of one workgroup over the tile counts.  Empty tiles -- most of
// a frame's, all in the last order bucket -- are counted and placed with one
// LDS atomic per wave (a ballot), since per-lane atomics on one LDS word
// serialise; the other tiles spread over the buckets and take one atomic
// each.  Positions inside a bucket are taken in arrival order; the blend of
// a tile does not depend on when it runs.
struct ScanShared {
  int64_t wsum[16];
  int32_t bucket[ORDER_BUCKETS];
};

__device__ __forceinline__ void count_bucket(int32_t c, bool v, int32_t* bucket, int lane) {
  const uint64_t empty = __ballot(v && c == 0);
  if (v && c != 0) atomicAdd(&bucket[order_bucket(c)], 1);
  if (lane == 0 && empty) atomicAdd(&bucket[ORDER_BUCKETS - 1], __popcll(empty));
}

__device__ __forceinline__ void place_tile(const BatchArgs& a, int32_t c, bool v, int t, int32_t* bucket, int lane,
                                           uint64_t below) {
  const uint64_t empty = __ballot(v && c == 0);
  int pos = 0;
  if (v && c != 0) pos = atomicAdd(&bucket[order_bucket(c)], 1);
  int e0 = 0;
  if (lane == 0 && empty) e0 = atomicAdd(&bucket[ORDER_BUCKETS - 1], __popcll(empty));
  e0 = __shfl(e0, 0, 64);
  if (v && c == 0) pos = e0 + __popcll(empty & below);
  if (v) a.tile_order[pos] = t;
}

// Exclusive scan of one sweep's lane sums over the workgroup: the lane's
// start (plus carry) and the sweep's total.
__device__ __forceinline__ void block_scan(int64_t sum, int64_t carry, ScanShared& sh, int64_t& run, int64_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t incl = wave_incl_scan(sum, lane);
  if (lane == 63) sh.wsum[wv] = incl;
  __syncthreads();
  run = carry + incl - sum;
  total = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t v = sh.wsum[k];
    run += k < wv ? v : 0;
    total += v;
  }
}

__device__ __forceinline__ void write_start(const BatchArgs& a, int t, int32_t v) {
  a.tile_start[t] = v;
  a.tile_cursor[t] = v;
  // quadrant list lengths: the sort sets those of non-empty tiles
  reinterpret_cast<int4*>(a.qcount)[t] = make_int4(0, 0, 0, 0);
}

// Key total, overflow flag and, on overflow, empty segments everywhere.
__device__ __forceinline__ bool finish_scan(const BatchArgs& a, int nt, int64_t total) {
  const bool over = total > a.key_cap;
  if (over)
    for (int t = threadIdx.x; t < nt; t += 1024) {
      a.tile_start[t] = 0;
      a.tile_cursor[t] = 0;
    }
  if (threadIdx.x == 0) {
    a.tile_start[nt] = over ? 0 : (int32_t)total;
    a.dev->n_keys = total;
    a.dev->overflow = over ? 1 : 0;
  }
  return over;
}

__device__ __forceinline__ void bucket_starts(ScanShared& sh) {
  __syncthreads();
  if (threadIdx.x < ORDER_BUCKETS) {             // bucket sizes -> first positions
    const int32_t c = sh.bucket[threadIdx.x];
    sh.bucket[threadIdx.x] = wave_incl_scan(c, (int)threadIdx.x) - c;
  }
  __syncthreads();
}

// Up to 8 tiles per lane (8,192 tiles): lane i owns tiles [8 i, 8 i + 8) and
// keeps their counts in registers, all loads in flight together.
constexpr int SCAN_REG = 8;

__device__ __forceinline__ void scan_small(const BatchArgs& a, int nt, int per, ScanShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int b = min(nt, tid * per), m = min(nt, b + per) - b;
  int32_t cnt[SCAN_REG];
#pragma unroll
  for (int k = 0; k < SCAN_REG; ++k) cnt[k] = k < m ? a.tile_count[b + k] : 0;
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_REG; ++k) {
    sum += cnt[k];
    count_bucket(cnt[k], k < m, sh.bucket, lane);
  }
  int64_t run, total;
  block_scan(sum, 0, sh, run, total);
  if (!(total > a.key_cap)) {
#pragma unroll
    for (int k = 0; k < SCAN_REG; ++k)
      if (k < m) {
        write_start(a, b + k, (int32_t)run);
        run += cnt[k];
      }
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_REG; ++k)
      if (k < m) reinterpret_cast<int4*>(a.qcount)[b + k] = make_int4(0, 0, 0, 0);
  }
  finish_scan(a, nt, total);
  bucket_starts(sh);
  const uint64_t below = lanes_below();
#pragma unroll
  for (int k = 0; k < SCAN_REG; ++k) place_tile(a, cnt[k], k < m, b + k, sh.bucket, lane, below);
}

// More tiles (batches): chunks of SCAN_CHUNK tiles staged in LDS by
// coalesced loads (all of a lane's in flight together), lane i owning the
// SCAN_PER consecutive tiles [i SCAN_PER, (i + 1) SCAN_PER) of a chunk
// (rows padded by one word against bank conflicts).  A first sweep writes
// the starts (carried across chunks) and counts the buckets, a second
// places the tiles.
constexpr int SCAN_PER = 16;
constexpr int SCAN_CHUNK = 1024 * SCAN_PER;

__device__ __forceinline__ int scan_slot(int j) { return (j / SCAN_PER) * (SCAN_PER + 1) + j % SCAN_PER; }

__device__ __forceinline__ void load_chunk(const BatchArgs& a, int c0, int nt, int32_t* cnt) {
  int32_t v[SCAN_PER];
  const int n = min(nt - c0, SCAN_CHUNK);
#pragma unroll
  for (int i = 0; i < SCAN_PER; ++i) {
    const int j = (int)threadIdx.x + 1024 * i;
    v[i] = j < n ? a.tile_count[c0 + j] : 0;
  }
#pragma unroll
  for (int i = 0; i < SCAN_PER; ++i) cnt[scan_slot((int)threadIdx.x + 1024 * i)] = v[i];
  __syncthreads();
}

__device__ __forceinline__ void scan_large(const BatchArgs& a, int nt, ScanShared& sh, int32_t* cnt) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int32_t* my = cnt + tid * (SCAN_PER + 1);
  int64_t carry = 0;
  for (int c0 = 0; c0 < nt; c0 += SCAN_CHUNK) {
    load_chunk(a, c0, nt, cnt);
    const int b = c0 + tid * SCAN_PER;
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
      sum += my[k];
      count_bucket(my[k], b + k < nt, sh.bucket, lane);
    }
    int64_t run, total;
    block_scan(sum, carry, sh, run, total);
    for (int k = 0; k < SCAN_PER && b + k < nt; ++k) {
      write_start(a, b + k, (int32_t)run);   // an overflow zeroes the starts again
      run += my[k];
    }
    carry += total;
    __syncthreads();                          // wsum and the chunk's counts are reused
  }
  finish_scan(a, nt, carry);
  bucket_starts(sh);
  const uint64_t below = lanes_below();
  for (int c0 = 0; c0 < nt; c0 += SCAN_CHUNK) {
    load_chunk(a, c0, nt, cnt);
    const int b = c0 + tid * SCAN_PER;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) place_tile(a, my[k], b + k < nt, b + k, sh.bucket, lane, below);
    __syncthreads();                          // the chunk's counts are reused
  }
}

__global__ void __launch_bounds__(1024) k_scan(BatchArgs a) {
  __shared__ ScanShared sh;
  __shared__ int32_t cnt[1024 * (SCAN_PER + 1)];
  const int nt = batch_hdr(a).n_tiles;
  if (threadIdx.x < ORDER_BUCKETS) sh.bucket[threadIdx.x] = 0;
  __syncthreads();
  const int per = (nt + 1023) / 1024;
  if (per <= SCAN_REG) scan_small(a, nt, per, sh);
  else scan_large(a, nt, sh, cnt);
}

// Scatter of one chunk's keys into the tile segments: LDS counts, one
// global atomic per touched tile reserves a run, LDS atomics hand out the
// slots of the run.
__global__ void __launch_bounds__(1024) k_fill(BatchArgs a) {
  if (a.dev->overflow) return;
  extern __shared__ int32_t bins[];
  const BatchHdr h = batch_hdr(a);
  ChunkReq c;
  if (!chunk_req(a, h, c)) return;
  const int tid = threadIdx.x;
  const bool lds = c.n_tiles <= BIN_LDS_MAX_TILES;
  int32_t* gcursor = a.tile_cursor + c.tile_off;
  if (lds) {
    for (int t = tid; t < c.n_tiles; t += 1024) bins[t] = 0;
    __syncthreads();
    for (int64_t i = c.i0 + tid; i < c.i1; i += 1024) {
      int x0, x1, y0, y1;
      rect_of(a.rect[c.g_off + i], x0, x1, y0, y1);
      for (int ty = y0; ty <= y1; ++ty)
        for (int tx = x0; tx <= x1; ++tx) atomicAdd(&bins[ty * c.tiles_x + tx], 1);
    }
    __syncthreads();
    for (int t = tid; t < c.n_tiles; t += 1024) {
      const int v = bins[t];
      if (v) bins[t] = atomicAdd(&gcursor[t], v);
    }
    __syncthreads();
  }
  for (int64_t i = c.i0 + tid; i < c.i1; i += 1024) {
    const int64_t g = c.g_off + i;
    int x0, x1, y0, y1;
    rect_of(a.rect[g], x0, x1, y0, y1);
    if (x0 > x1) continue;
    const uint64_t key = ((uint64_t)a.depth[g] << 32) | (uint64_t)(uint32_t)g;
    const double2 xy = a.xy[g];
    const float4 ext = a.ext[g];
    for (int ty = y0; ty <= y1; ++ty)
      for (int tx = x0; tx <= x1; ++tx) {
        const int t = ty * c.tiles_x + tx;
        const uint32_t m = quadrant_mask(xy, ext, (double)(tx * TILE), (double)(ty * TILE));
        const int slot = lds ? atomicAdd(&bins[t], 1) : atomicAdd(&gcursor[t], 1);
        a.keys[slot] = key | ((uint64_t)m << KEY_MASK_SHIFT);
      }
  }
}

// ------------------------------------------------------------ segment sort
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// lanes of the wave whose 8-bit digit equals this lane's (valid lanes only)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t w = (uint32_t)__shfl_xor((int)v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t w = (uint32_t)__shfl_xor((int)v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int bit_length(uint64_t x) { return x ? 64 - __clzll(x) : 0; }

// Shared scratch of the segment sort.
struct SortShared {
  union {
    uint32_t bins[1024];     // digit counts of an unstable pass, then offsets
    uint32_t hist[4][256];   // per-wave digit counts of a global-memory pass
  };
  uint32_t whist[4][64];     // per-wave digit counts of a stable 6-bit pass
  uint32_t wtot[4];
  uint64_t red[4][4];
  int32_t qw[4][4];          // per-wave quadrant counts of the output stage
};

constexpr int U_BITS = 10;   // digit of an unstable pass (1024 counters)
constexpr int S_BITS = 6;    // digit of a stable pass (64 counters per wave)

// Pass over the digit (x >> shift) & mask (at most U_BITS bits) that keeps
// no order among equal digits: an LDS atomic hands each element a slot in
// its digit's run.  The elements are this lane's x[i] for the bits i set
// in live; they land in buf[0, n) (which no lane reads during the pass, so
// buf may hold them on entry).  bins is zero on entry and on exit.
template <int K>
__device__ __forceinline__ void pass_unstable(const uint64_t (&x)[K], uint32_t live, uint64_t* buf, int shift,
                                              uint32_t mask, SortShared& sh) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  uint32_t slot[K];
#pragma unroll
  for (int i = 0; i < K; ++i)
    slot[i] = ((live >> i) & 1u) ? atomicAdd(&sh.bins[(uint32_t)(x[i] >> shift) & mask], 1u) : 0u;
  __syncthreads();
  // exclusive offsets: lane tid owns the counters [4 tid, 4 tid + 4)
  const uint4 c = reinterpret_cast<const uint4*>(sh.bins)[tid];
  const uint32_t tot = c.x + c.y + c.z + c.w;
  const uint32_t incl = wave_incl_scan(tot, lane);
  if (lane == 63) sh.wtot[w] = incl;
  __syncthreads();
  uint32_t base = incl - tot;
  for (int q = 0; q < w; ++q) base += sh.wtot[q];
  reinterpret_cast<uint4*>(sh.bins)[tid] = make_uint4(base, base + c.x, base + c.x + c.y, base + c.x + c.y + c.z);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i)
    if ((live >> i) & 1u) buf[sh.bins[(uint32_t)(x[i] >> shift) & mask] + slot[i]] = x[i];
  __syncthreads();
  reinterpret_cast<uint4*>(sh.bins)[tid] = make_uint4(0u, 0u, 0u, 0u);
}

// Stable pass over the digit (x >> shift) & 63 of buf[0, n), in place.
// Wave w takes the contiguous range [w per, (w + 1) per) into registers,
// 64 elements at a time in order, and ranks each element among the
// wave's equal digits before it: ballot matching inside the 64 gives the
// rank among them and their count, and the lowest lane of each digit adds
// that count to the wave's running count of the digit (an LDS atomic whose
// old value its group reads back).  One wave turns the per-wave counts
// into offsets (digit-major, wave-minor); every element then goes to its
// offset plus its rank.  whist is zero on entry and on exit.
template <int K>
__device__ __forceinline__ void pass_stable(uint64_t* buf, int n, int shift, SortShared& sh) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int per = ((n + 255) / 256) * 64;
  const int b = min(n, w * per), e = min(n, b + per);
  const uint64_t below = lanemask_lt();
  uint64_t x[K];
  uint32_t rank[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int j = b + 64 * i + lane;
    x[i] = j < e ? buf[j] : 0ull;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    rank[i] = 0;
    if (b + 64 * i >= e) continue;
    const bool valid = b + 64 * i + lane < e;
    const uint32_t d = (uint32_t)(x[i] >> shift) & 63u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int k = 0; k < S_BITS; ++k) {
      const bool bit = (d >> k) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int lead = __ffsll((unsigned long long)peers) - 1;
    uint32_t old = 0;
    if (valid && lane == lead) old = atomicAdd(&sh.whist[w][d], (uint32_t)__popcll(peers));
    old = (uint32_t)__shfl((int)old, lead & 63, 64);
    rank[i] = old + (uint32_t)__popcll(peers & below);
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t h0 = sh.whist[0][lane], h1 = sh.whist[1][lane], h2 = sh.whist[2][lane], h3 = sh.whist[3][lane];
    const uint32_t tot = h0 + h1 + h2 + h3;
    const uint32_t base = wave_incl_scan(tot, lane) - tot;
    sh.whist[0][lane] = base;
    sh.whist[1][lane] = base + h0;
    sh.whist[2][lane] = base + h0 + h1;
    sh.whist[3][lane] = base + h0 + h1 + h2;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i)
    if (b + 64 * i + lane < e) buf[sh.whist[w][(uint32_t)(x[i] >> shift) & 63u] + rank[i]] = x[i];
  __syncthreads();
  sh.whist[w][lane] = 0;   // the wave's own row; the next pass counts into it after a barrier
}

// One stable pass over digit (key >> shift) & 255 of elements [0, n).
// Wave w owns the contiguous element range [w * per, (w + 1) * per) and
// visits it in order, 64 at a time, so elements with equal digits keep
// their input order.  hist must be zero on entry and is zero on exit.
template <typename Ptr>
__device__ __forceinline__ void radix_pass(Ptr src, Ptr dst, int n, int shift, SortShared& sh) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int per = ((n + 255) / 256) * 64;
  const int b = min(n, w * per), e = min(n, b + per);
  for (int j = b + lane; j < e; j += 64) atomicAdd(&sh.hist[w][(uint32_t)(src[j] >> shift) & 255u], 1u);
  __syncthreads();
  // digit-major, wave-minor exclusive offsets; wave w scans digits [64 w, 64 w + 64)
  const int d = 64 * w + lane;
  const uint32_t h0 = sh.hist[0][d], h1 = sh.hist[1][d], h2 = sh.hist[2][d], h3 = sh.hist[3][d];
  const uint32_t t = h0 + h1 + h2 + h3;
  const uint32_t incl = wave_incl_scan(t, lane);
  if (lane == 63) sh.wtot[w] = incl;
  __syncthreads();
  uint32_t base = incl - t;
  for (int q = 0; q < w; ++q) base += sh.wtot[q];
  sh.hist[0][d] = base;
  sh.hist[1][d] = base + h0;
  sh.hist[2][d] = base + h0 + h1;
  sh.hist[3][d] = base + h0 + h1 + h2;
  __syncthreads();
  for (int j0 = b; j0 < e; j0 += 64) {
    const int j = j0 + lane;
    const bool valid = j < e;
    const uint64_t v = valid ? (uint64_t)src[j] : 0ull;
    const uint32_t dg = (uint32_t)(v >> shift) & 255u;
    const uint64_t peers = match_digit(dg, valid);
    const uint32_t pos = valid ? sh.hist[w][dg] : 0u;
    if (valid) dst[pos + (uint32_t)__popcll(peers & lanemask_lt())] = v;
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & lanemask_lt()) == 0) sh.hist[w][dg] = pos + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int q = lane; q < 256; q += 64) sh.hist[w][q] = 0;   // wave-private row, next pass counts into it
}

// LSD passes over bits [shift0, shift0 + bits); returns the buffer holding the result.
template <typename Ptr>
__device__ __forceinline__ Ptr radix_sort(Ptr a, Ptr b, int n, int shift0, int bits, SortShared& sh) {
  const int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    radix_pass(a, b, n, shift0 + 8 * p, sh);
    Ptr t = a; a = b; b = t;
  }
  return a;
}

// Output stage of a tile's sort.  get(j, gi, m) yields sorted entry j
// (Gaussian index gi, quadrant mask m); the entry goes to the tile's index
// list at s + j and to the list of each quadrant in m as (gi, j).  Wave w
// owns the contiguous entries [w per, (w + 1) per): it counts its entries'
// quadrant bits (a ballot per quadrant and 64 entries), the four waves'
// counts meet in LDS behind one barrier, and each wave then writes its
// entries from its own offsets, so every quadrant list keeps the list
// order.  Quadrant qd's list starts at 4 s + qd n of qlist; its length goes
// to qcount[4 t + qd].
template <typename Get>
__device__ __forceinline__ void emit_sorted(const BatchArgs& a, int t, int s, int n, Get get, SortShared& sh) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int2* out = a.qlist + 4 * (int64_t)s;
  const uint64_t below = lanemask_lt();
  const int per = ((n + 255) / 256) * 64;
  const int b = min(n, w * per), e = min(n, b + per);
  int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  for (int j0 = b; j0 < e; j0 += 64) {
    const int j = j0 + lane;
    uint32_t gi = 0, m = 0;
    if (j < e) get(j, gi, m);
    c0 += __popcll(__ballot(m & 1u));
    c1 += __popcll(__ballot(m & 2u));
    c2 += __popcll(__ballot(m & 4u));
    c3 += __popcll(__ballot(m & 8u));
  }
  if (lane == 0) {
    sh.qw[0][w] = c0;
    sh.qw[1][w] = c1;
    sh.qw[2][w] = c2;
    sh.qw[3][w] = c3;
  }
  __syncthreads();
  int base[4];
#pragma unroll
  for (int qd = 0; qd < 4; ++qd) {
    int pre = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) pre += ww < w ? sh.qw[qd][ww] : 0;
    base[qd] = pre;
  }
  for (int j0 = b; j0 < e; j0 += 64) {
    const int j = j0 + lane;
    uint32_t gi = 0, m = 0;
    if (j < e) {
      get(j, gi, m);
      a.sorted[s + j] = (int32_t)gi;
    }
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const uint64_t bal = __ballot((m >> qd) & 1u);
      if ((m >> qd) & 1u) out[(int64_t)qd * n + base[qd] + __popcll(bal & below)] = make_int2((int)gi, j);
      base[qd] += __popcll(bal);
    }
  }
  // (qw is next written after the next tile's first barriers)
  if (tid < 4) a.qcount[4 * t + tid] = sh.qw[tid][0] + sh.qw[tid][1] + sh.qw[tid][2] + sh.qw[tid][3];
}

constexpr int MAX_TIE_RUN = 32;
constexpr int SORT_TOP_BITS = U_BITS + S_BITS;   // depth bits the passes order; the rest by run insertion

// Segment sort of tile t, whose key count lies in (lo, hi]: sort by depth
// alone (the key's high half, re-based to its minimum), then order each run
// of equal depths by index; only a run longer than MAX_TIE_RUN makes the
// tile redo the sort on the composite (depth, index) key.  Either way the
// result is the (depth, index) order.  Segments up to CAP keys stay in the
// registers they are loaded into (CAP / 256 per lane) and in one LDS
// buffer: an unstable pass on the lower digit straight from the registers,
// then a stable pass on the top six bits.  Larger segments, and the rare
// ones with a too long run, run the composite sort with 8-bit stable passes
// on the global scratch buffers.
// The quadrant mask rides along: in the low half of the depth-only element
// (above the index, which alone is compared among equal depths), below the
// composite key (whose (depth, index) part is unique, so the mask never
// decides the order).
template <int CAP>
__device__ __forceinline__ void sort_tile(const BatchArgs& a, int t, int s, int n, uint64_t* buf, SortShared& sh) {
  constexpr int K = CAP / 256;
  static_assert(K >= 1 && K <= 32, "one live bit per register slot");
  const int tid = threadIdx.x, w = tid >> 6;
  if (n == 1) {
    const uint32_t lo = (uint32_t)a.keys[s];
    emit_sorted(a, t, s, 1, [&](int, uint32_t& gi, uint32_t& m) { gi = lo & KEY_INDEX; m = lo >> KEY_MASK_SHIFT; }, sh);
    return;
  }
  // ranges of depth and index in the segment; a segment up to CAP keys is
  // loaded K keys per lane with all loads in flight at once and stays in
  // registers
  uint64_t kv[K];
  uint32_t live = 0;
  uint64_t dmin = ~0ull, dmax = 0, imin = ~0ull, imax = 0;
  auto widen = [&](uint64_t k) {
    const uint64_t d = k >> 32, ix = (uint32_t)k & KEY_INDEX;
    dmin = d < dmin ? d : dmin; dmax = d > dmax ? d : dmax;
    imin = ix < imin ? ix : imin; imax = ix > imax ? ix : imax;
  };
  if (n <= CAP) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int j = tid + 256 * i;
      kv[i] = j < n ? a.keys[s + j] : 0ull;
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (tid + 256 * i < n) {
        live |= 1u << i;
        widen(kv[i]);
      }
  } else {
    for (int j = tid; j < n; j += 256) widen(a.keys[s + j]);
  }
  // depth and index are 32-bit quantities: 32-bit wave reductions (one lane
  // permute per step instead of two)
  dmin = wave_min_u32((uint32_t)dmin); dmax = wave_max_u32((uint32_t)dmax);
  imin = wave_min_u32((uint32_t)imin); imax = wave_max_u32((uint32_t)imax);
  if ((tid & 63) == 0) { sh.red[w][0] = dmin; sh.red[w][1] = dmax; sh.red[w][2] = imin; sh.red[w][3] = imax; }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    dmin = sh.red[q][0] < dmin ? sh.red[q][0] : dmin; dmax = sh.red[q][1] > dmax ? sh.red[q][1] : dmax;
    imin = sh.red[q][2] < imin ? sh.red[q][2] : imin; imax = sh.red[q][3] > imax ? sh.red[q][3] : imax;
  }
  const int db = bit_length(dmax - dmin), ib = bit_length(imax - imin);
  const uint64_t imask = ib == 0 ? 0ull : (~0ull >> (64 - ib));
  // composite element: (depth - dmin, index - imin, mask), at most 32 + 28 + 4 bits
  const int cbits = db + ib + 4;
  auto composite = [&](uint64_t k) -> uint64_t {
    return (((k >> 32) - dmin) << (ib + 4)) | ((((uint32_t)k & KEY_INDEX) - imin) << 4) |
           (uint64_t)((uint32_t)k >> KEY_MASK_SHIFT);
  };
  auto from_composite = [&](uint64_t e, uint32_t& gi, uint32_t& m) {
    gi = (uint32_t)(imin + ((e >> 4) & imask));
    m = (uint32_t)e & 15u;
  };
  if (n <= CAP) {
    // depth-only element: (depth - dmin) << 32 | (mask, index)
#pragma unroll
    for (int i = 0; i < K; ++i) kv[i] = (((kv[i] >> 32) - dmin) << 32) | (kv[i] & 0xffffffffull);
    // the top (at most) 16 bits of the re-based depth: one unstable pass on
    // their lower part, one stable pass on their top six bits (a typical
    // tile's depths span 20-23 bits)
    const int low = db > SORT_TOP_BITS ? db - SORT_TOP_BITS : 0;
    const int nb = db - low;
    if (nb == 0) {
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((live >> i) & 1u) buf[tid + 256 * i] = kv[i];
      __syncthreads();
    } else if (nb <= U_BITS) {
      pass_unstable<K>(kv, live, buf, 32 + low, (1u << nb) - 1u, sh);
    } else {
      pass_unstable<K>(kv, live, buf, 32 + low, (1u << (nb - S_BITS)) - 1u, sh);
      pass_stable<K>(buf, n, 32 + low + nb - S_BITS, sh);
    }
    // Keys equal in those bits are now adjacent, in arbitrary order: runs of
    // them are short (about 750 keys over 65,536 bins per tile).  A lane per
    // run orders it by the whole (depth, index) key (insertion sort); a run
    // longer than MAX_TIE_RUN sends the tile to the composite sort.
    const int hs = 32 + low;
    auto whole = [](uint64_t x) -> uint64_t { return ((x >> 32) << KEY_MASK_SHIFT) | ((uint32_t)x & KEY_INDEX); };
    int too_long = 0;
    for (int j = tid; j < n; j += 256) {
      const uint64_t dj = buf[j] >> hs;
      const bool start = (j == 0 || (buf[j - 1] >> hs) != dj) && j + 1 < n && (buf[j + 1] >> hs) == dj;
      if (!start) continue;
      int end = j + 1;
      while (end < n && (buf[end] >> hs) == dj && end - j <= MAX_TIE_RUN) ++end;
      if (end - j > MAX_TIE_RUN) { too_long = 1; continue; }
      for (int p = j + 1; p < end; ++p) {
        const uint64_t v = buf[p];
        const uint64_t vk = whole(v);
        int q = p - 1;
        while (q >= j && whole(buf[q]) > vk) { buf[q + 1] = buf[q]; --q; }
        buf[q + 1] = v;
      }
    }
    if (!__syncthreads_or(too_long)) {
      emit_sorted(a, t, s, n, [&](int j, uint32_t& gi, uint32_t& m) {
        const uint32_t lo = (uint32_t)buf[j];
        gi = lo & KEY_INDEX;
        m = lo >> KEY_MASK_SHIFT;
      }, sh);
      return;
    }
  }
  // the composite sort on the global scratch buffers: segments above CAP,
  // and segments with a run of equal depths too long for insertion (the
  // keys in global memory are still the unsorted ones)
  uint64_t* g0 = a.keys + s;
  uint64_t* g1 = a.keys_tmp + s;
  for (int j = tid; j < n; j += 256) g0[j] = composite(g0[j]);
  __syncthreads();
  const uint64_t* res = radix_sort<uint64_t*>(g0, g1, n, 0, cbits, sh);
  emit_sorted(a, t, s, n, [&](int j, uint32_t& gi, uint32_t& m) { from_composite(res[j], gi, m); }, sh);
}

// Tiles are taken in the scan's order (descending key count), so the
// longest segments start first.  Without LOOP the grid covers every tile
// slot of the batch and workgroup i takes the i-th tile of that order (no
// loop, so nothing is kept live from one tile to the next); with LOOP, a
// small grid walks the head of that order and stops at the first tile too
// short for it.
template <int CAP, bool LOOP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CAP <= 2048 ? 6 : 1, 8)))
k_sort(BatchArgs a, int lo, int hi) {
  __shared__ uint64_t buf[CAP];
  __shared__ SortShared sh;
  // both reads in flight before the first branch: most workgroups of a
  // serving slot's launch lie past the batch's tiles and leave here
  const int overflow = a.dev->overflow;
  const BatchHdr h = batch_hdr(a);
  const int nt = h.n_tiles;
  if (overflow != 0 || (!LOOP && (int)blockIdx.x >= nt)) return;
  // the passes keep their counters zero between uses
  reinterpret_cast<uint4*>(sh.bins)[threadIdx.x] = make_uint4(0u, 0u, 0u, 0u);
  (&sh.whist[0][0])[threadIdx.x] = 0u;
  __syncthreads();
  auto job = [&](int i, int& t, int& s, int& n) {   // 1: sort tile t, 0: skip it, -1: stop
    t = a.tile_order[i];
    s = a.tile_start[t];
    n = a.tile_start[t + 1] - s;
    if (n <= lo) return LOOP && n < ((ORDER_BUCKETS - 1) << ORDER_SHIFT) ? -1 : 0;   // the rest are shorter still
    if (n > hi) return 0;
    if (h.n_shared > 0 && batch_req(a, req_of_tile(a, h, t)).src != 0) return 0;   // copied later
    return 1;
  };
  int t, s, n;
  if (!LOOP) {
    if (job(blockIdx.x, t, s, n) == 1) sort_tile<CAP>(a, t, s, n, buf, sh);
    return;
  }
  for (int i = blockIdx.x; i < nt; i += gridDim.x) {
    const int r = job(i, t, s, n);
    if (r < 0) break;
    if (r == 0) continue;
    sort_tile<CAP>(a, t, s, n, buf, sh);
    __syncthreads();                 // LDS is reused by the next tile
  }
}

constexpr int SORT_SMALL = 2048;   // segments up to this size: 16 KB of LDS keys, 7 workgroups per CU
constexpr int SORT_LARGE = 8192;   // larger segments: 64 KB of LDS keys, beyond it global scratch

}  // namespace

hipError_t launch_bin_sort(const BatchArgs& a, int64_t grid_gauss, int32_t grid_tiles,
                           int32_t max_tiles_per_req, hipStream_t s) {
  const int64_t chunks = (grid_gauss + BIN_CHUNK - 1) / BIN_CHUNK;
  const int grid = (int)(chunks > 0 ? chunks : 1);
  const size_t shm = (size_t)min(max_tiles_per_req, BIN_LDS_MAX_TILES) * sizeof(int32_t);
  const int gt = grid_tiles > 0 ? grid_tiles : 1;
  const bool sharing = a.table != nullptr;    // only a replayed batch can hold sharing requests
  const int share_grid = gt < 1024 ? gt : 1024;
  hipLaunchKernelGGL(k_count, dim3(grid), dim3(1024), shm, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (sharing) {
    hipLaunchKernelGGL(k_share_count, dim3((gt + 255) / 256 < 1024 ? (gt + 255) / 256 : 1024), dim3(256), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(1024), shm, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  // gt is the batch's tile capacity: one workgroup per tile slot
  hipLaunchKernelGGL((k_sort<SORT_SMALL, false>), dim3(gt), dim3(256), 0, s, a, 0, SORT_SMALL);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL((k_sort<SORT_LARGE, true>), dim3(gt < 256 ? gt : 256), dim3(256), 0, s, a, SORT_SMALL,
                     0x7fffffff);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (sharing) {
    hipLaunchKernelGGL(k_share_copy, dim3(share_grid), dim3(256), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t bin_set_attributes() {
  const int bytes = BIN_LDS_MAX_TILES * (int)sizeof(int32_t);
  hipError_t e = hipFuncSetAttribute((const void*)k_count, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_fill, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace tg
