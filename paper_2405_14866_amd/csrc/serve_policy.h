// serve_policy.h -- the admission and retirement rules of the serving loop
// (serve.hip), free of device code so that the host can exercise them with
// a fake executor.
//
// Admission: requests leave the queue first in, first out, into the batch
// being formed on a free slot, while the batch stays within the slot's
// workspace (padded Gaussians, tiles, pixels, estimated keys -- a request
// whose key estimate alone exceeds the slot still goes, alone, and the
// device reports its overflow), within max_batch, and while the bytes of
// every request in flight stay within the budget.  A request marked solo
// (one that overflowed in a batch) only ever runs alone.
// Retirement: a batch whose binning overflowed is retried request by
// request, each alone; an overflow of a request alone is its final
// TG_ERR_CAPACITY; a request whose geometry differed from the request it
// shared lists with is retried without sharing.  Retried requests go back
// to the queue front in their batch order, ahead of everything newer.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace tg {
namespace policy {

struct Limits {
  int max_batch;
  int64_t cap_gauss, cap_keys, cap_pixels;
  int32_t cap_tiles;
  int64_t budget;
};

// What one queued request needs.
struct Demand {
  int64_t gauss;       // padded Gaussian count
  int64_t keys;        // key estimate
  int64_t pixels;
  int32_t tiles;
  int64_t footprint;   // bytes counted against the budget while in flight
  bool solo;
};

// Move the requests that join the next batch from the queue front into the
// returned batch, adding their footprints to budget_used.  Queue: a deque
// of request ids; demand_of(id) -> Demand.
template <class Queue, class DemandOf>
std::vector<uint64_t> form_batch(Queue& queue, DemandOf demand_of, const Limits& L, int64_t& budget_used) {
  std::vector<uint64_t> batch;
  int64_t sum_g = 0, sum_k = 0, sum_px = 0;
  int32_t sum_t = 0;
  while (!queue.empty() && (int)batch.size() < L.max_batch) {
    const Demand d = demand_of(queue.front());
    if (d.solo && !batch.empty()) break;
    if (sum_g + d.gauss > L.cap_gauss || sum_t + d.tiles > L.cap_tiles || sum_px + d.pixels > L.cap_pixels ||
        (sum_k + d.keys > L.cap_keys && !batch.empty()))
      break;
    if (budget_used + d.footprint > L.budget) break;
    budget_used += d.footprint;
    batch.push_back(queue.front());
    queue.pop_front();
    sum_g += d.gauss;
    sum_k += d.keys;
    sum_px += d.pixels;
    sum_t += d.tiles;
    if (d.solo) break;
  }
  return batch;
}

enum class Outcome { Done, Capacity, RetrySolo, RetryNoShare };

// Outcome of request k of a finished batch of batch_size requests: overflow
// is the batch's key overflow, mismatch its bit k of the geometry check.
inline Outcome retire(bool overflow, size_t batch_size, bool mismatch) {
  if (overflow && batch_size > 1) return Outcome::RetrySolo;
  if (!overflow && mismatch) return Outcome::RetryNoShare;
  return overflow ? Outcome::Capacity : Outcome::Done;
}

// Retried requests back to the queue front, in their batch order.
template <class Queue>
void requeue(Queue& queue, const std::vector<uint64_t>& retry) {
  for (auto it = retry.rbegin(); it != retry.rend(); ++it) queue.push_front(*it);
}

// Batching window: with fewer than max_batch requests queued, a free slot
// holds them until the oldest (submitted at front_submit_ns) has waited
// window_us; a solo request is never held.
inline bool holds(size_t queued, int max_batch, int window_us, int64_t front_submit_ns, bool front_solo,
                  int64_t now_ns) {
  if (queued == 0 || window_us <= 0 || (int)queued >= max_batch || front_solo) return false;
  return now_ns < front_submit_ns + (int64_t)window_us * 1000;
}

}  // namespace policy
}  // namespace tg
