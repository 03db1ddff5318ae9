// Host-only driver of the serving loop's admission and retirement rules
// (paper_2405_14866_amd/csrc/serve_policy.h) with a fake executor: batches
// "run" for a time proportional to their Gaussians, a batch overflows when
// its requests' true key counts exceed the slot's key capacity, and a
// random subset of sharing requests reports a geometry mismatch on its
// first run.  Every launch and retirement is checked against the rules the
// header states; the result is one JSON line.
//
//   serve_policy_sim SEED N_REQ SLOTS MAX_BATCH WINDOW_US SPACING_US
//
// Built with -DPLANT_FOOTPRINT the harness hands the rules half of each
// request's footprint (a planted fault the checks must catch).
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <random>
#include <string>
#include <vector>

#include "serve_policy.h"

namespace {

struct Req {
  int64_t submit_ns;
  tg::policy::Demand d;
  int64_t true_keys;
  bool mismatch_once;      // shares lists and differs in geometry on its first run
  bool no_share = false;
  int status = -1;         // 0 done, 1 capacity
  int retries = 0;
  int first_launch = -1;   // launch sequence number of its first batch
  int runs = 0;
};

struct Slot {
  bool busy = false;
  int64_t done_ns = 0;
  std::vector<uint64_t> batch;
};

int failures = 0;
std::string first_failure;

void check(bool ok, const char* what) {
  if (!ok) {
    if (failures == 0) first_failure = what;
    ++failures;
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: %s SEED N_REQ SLOTS MAX_BATCH WINDOW_US SPACING_US\n", argv[0]);
    return 2;
  }
  const unsigned seed = (unsigned)atoi(argv[1]);
  const int n_req = atoi(argv[2]), n_slots = atoi(argv[3]), max_batch = atoi(argv[4]);
  const int window_us = atoi(argv[5]);
  const int64_t spacing_ns = (int64_t)atoi(argv[6]) * 1000;
  std::mt19937_64 rng(seed);
  auto uni = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };

  const tg::policy::Limits L{max_batch, 4'000'000, 16'000'000, 8 << 20, 40'000, 3'000'000'000LL};
  std::vector<Req> reqs(n_req);
  int64_t t = 0;
  for (Req& r : reqs) {
    t += uni(0, spacing_ns);                           // arrivals up to SPACING_US apart
    r.submit_ns = t;
    const int64_t n = uni(1, 900'000);
    const int64_t side = uni(64, 1024);
    r.d.gauss = (n + 1023) / 1024 * 1024;
    r.d.keys = n * 4;                                 // the loop's estimate
    r.d.pixels = side * side;
    r.d.tiles = (int32_t)(((side + 15) / 16) * ((side + 15) / 16));
    r.d.footprint = r.d.gauss * 76 + r.d.keys * 52 + r.d.pixels * 140;
    r.d.solo = false;
    // true keys: usually near the estimate, sometimes far above it (and a
    // few beyond what even a slot alone holds)
    const int64_t pick = uni(0, 99);
    r.true_keys = pick < 85 ? n * uni(2, 5) : (pick < 97 ? n * uni(8, 16) : L.cap_keys + uni(1, 1000));
    r.mismatch_once = uni(0, 9) == 0;
  }

  std::deque<uint64_t> queue;
  std::vector<Slot> slots(n_slots);
  int64_t budget_used = 0, now = 0;
  size_t next_arrival = 0;
  int launches = 0, batches_multi = 0, overflow_batches = 0, held = 0;
  int64_t max_budget_seen = 0;
  std::vector<uint64_t> first_order;                  // ids in order of first launch

  auto demand_of = [&](uint64_t id) {
    tg::policy::Demand d = reqs[id].d;
#ifdef PLANT_FOOTPRINT
    d.footprint /= 2;
#endif
    return d;
  };
  for (int guard = 0; guard < 10'000'000; ++guard) {
    // arrivals up to now
    while (next_arrival < reqs.size() && reqs[next_arrival].submit_ns <= now) queue.push_back(next_arrival++);
    // retire finished slots
    for (Slot& sl : slots) {
      if (!sl.busy || sl.done_ns > now) continue;
      int64_t keys = 0;
      for (uint64_t id : sl.batch) keys += reqs[id].true_keys;
      const bool over = keys > L.cap_keys;
      if (over) ++overflow_batches;
      std::vector<uint64_t> retry;
      for (uint64_t id : sl.batch) {
        Req& r = reqs[id];
        budget_used -= r.d.footprint;
        const bool mism = r.mismatch_once && !r.no_share && r.runs == 1;
        switch (tg::policy::retire(over, sl.batch.size(), mism)) {
          case tg::policy::Outcome::RetrySolo:
            check(sl.batch.size() > 1, "solo retry of a request that ran alone");
            r.retries += 1;
            r.d.solo = true;
            retry.push_back(id);
            break;
          case tg::policy::Outcome::RetryNoShare:
            check(!over, "no-share retry after an overflow");
            r.retries += 1;
            r.no_share = true;
            retry.push_back(id);
            break;
          case tg::policy::Outcome::Capacity:
            check(over && sl.batch.size() == 1, "capacity error outside a lone overflow");
            r.status = 1;
            break;
          case tg::policy::Outcome::Done:
            check(!over, "done after an overflow");
            r.status = 0;
            break;
        }
      }
      tg::policy::requeue(queue, retry);
      // the retried requests now lead the queue, in their batch order
      for (size_t k = 0; k < retry.size(); ++k) check(queue[k] == retry[k], "requeue order");
      sl.busy = false;
      sl.batch.clear();
    }
    // launch onto free slots
    const bool hold = !queue.empty() && tg::policy::holds(queue.size(), max_batch, window_us,
                                                          reqs[queue.front()].submit_ns, reqs[queue.front()].d.solo,
                                                          now);
    if (hold) ++held;
    for (Slot& sl : slots) {
      if (hold || sl.busy || queue.empty()) continue;
      const std::deque<uint64_t> before = queue;
      const int64_t used0 = budget_used;
      std::vector<uint64_t> b = tg::policy::form_batch(queue, demand_of, L, budget_used);
      if (b.empty()) {
        check(queue == before && budget_used == used0, "empty batch changed state");
        continue;
      }
      // first in, first out: the batch is the queue's head
      for (size_t k = 0; k < b.size(); ++k) check(b[k] == before[k], "batch is not the queue head");
      check((int)b.size() <= max_batch, "batch above max_batch");
      int64_t g = 0, k = 0, px = 0, fp = 0;
      int64_t tl = 0;
      for (uint64_t id : b) {
        const Req& r = reqs[id];
        g += r.d.gauss; k += r.d.keys; px += r.d.pixels; tl += r.d.tiles; fp += r.d.footprint;
        if (r.d.solo) check(b.size() == 1, "solo request in a shared batch");
      }
      check(g <= L.cap_gauss && px <= L.cap_pixels && tl <= L.cap_tiles, "batch above the slot workspace");
      check(k <= L.cap_keys || b.size() == 1, "batch above the key capacity");
      check(budget_used == used0 + fp, "budget accounting");
      check(budget_used <= L.budget, "budget exceeded");
      // the request after the batch did not fit (or the batch is full / ended by a solo request)
      if (!queue.empty() && (int)b.size() < max_batch && !reqs[b.back()].d.solo) {
        const Req& nx = reqs[queue.front()];
        const bool fits = !nx.d.solo && g + nx.d.gauss <= L.cap_gauss && px + nx.d.pixels <= L.cap_pixels &&
                          tl + nx.d.tiles <= L.cap_tiles && k + nx.d.keys <= L.cap_keys &&
                          budget_used + nx.d.footprint <= L.budget;
        check(!fits, "a fitting request was left in the queue");
      }
      max_budget_seen = std::max(max_budget_seen, budget_used);
      for (uint64_t id : b) {
        Req& r = reqs[id];
        if (r.first_launch < 0) {
          r.first_launch = launches;
          first_order.push_back(id);
        }
        r.runs += 1;
      }
      if (b.size() > 1) ++batches_multi;
      ++launches;
      sl.busy = true;
      sl.done_ns = now + 50'000 + g / 20;             // 50 us + 50 ns per Gaussian
      sl.batch = std::move(b);
    }
    // advance time to the next event
    int64_t next = INT64_MAX;
    for (const Slot& sl : slots)
      if (sl.busy) next = std::min(next, sl.done_ns);
    if (next_arrival < reqs.size()) next = std::min(next, reqs[next_arrival].submit_ns);
    if (hold) next = std::min(next, reqs[queue.front()].submit_ns + (int64_t)window_us * 1000);
    if (next == INT64_MAX) break;
    now = std::max(now, next);
  }

  int done = 0, capacity = 0, unfinished = 0, retried = 0, max_retries = 0;
  for (const Req& r : reqs) {
    if (r.status == 0) ++done;
    else if (r.status == 1) ++capacity;
    else ++unfinished;
    if (r.retries > 0) ++retried;
    max_retries = std::max(max_retries, r.retries);
    if (r.status == 1) check(r.true_keys > L.cap_keys, "capacity error for a request that fits alone");
    if (r.status == 0 && r.true_keys > L.cap_keys) check(false, "an oversize request finished");
  }
  check(unfinished == 0, "requests left unfinished");
  check(queue.empty() && budget_used == 0, "queue or budget not drained");
  check(max_retries <= 2, "more than two retries");
  // first launches follow submission order
  check(std::is_sorted(first_order.begin(), first_order.end()), "first launches out of submission order");
  printf("{\"failures\": %d, \"first_failure\": \"%s\", \"requests\": %d, \"done\": %d, \"capacity\": %d, "
         "\"retried\": %d, \"launches\": %d, \"batches_multi\": %d, \"overflow_batches\": %d, \"held\": %d, "
         "\"max_budget_frac\": %.3f}\n",
         failures, first_failure.c_str(), n_req, done, capacity, retried, launches, batches_multi,
         overflow_batches, held, (double)max_budget_seen / (double)L.budget);
  return failures == 0 ? 0 : 1;
}
