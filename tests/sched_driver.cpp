// Host-only checks of the solve server's scheduling pieces (bdrs_sched.h):
// the pool allocator's invariants under a seeded random workload, the
// admission choice case by case, and the admission / block / retire loop the
// server runs, driven by a fake executor (each request needs a fixed number of
// blocks), with its invariants checked after every boundary.  Prints "ok" and
// exits 0, or prints the first failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "bdrs_sched.h"

using bdrs_sched::PoolAlloc;
using bdrs_sched::pick_admission;
using bdrs_sched::pool_align;

static int failures = 0;
#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);        \
      if (++failures > 20) std::exit(1);                                 \
    }                                                                    \
  } while (0)

// every invariant of the allocator's bookkeeping
static void check_pool(const PoolAlloc& p) {
  size_t used = 0, free_sum = 0, end = 0;
  for (auto& a : p.allocated()) {
    CHECK(a.first % 256 == 0 && a.second % 256 == 0 && a.second > 0);
    CHECK(a.first >= end);  // disjoint, in order
    end = a.first + a.second;
    used += a.second;
  }
  CHECK(end <= p.size());
  end = 0;
  size_t prev_end = (size_t)-1;
  for (auto& f : p.free_ranges()) {
    CHECK(f.first >= end && f.second > 0);
    CHECK(f.first != prev_end);  // neighbours are merged
    end = prev_end = f.first + f.second;
    free_sum += f.second;
    // a free range overlaps no allocated range
    auto it = p.allocated().lower_bound(f.first);
    if (it != p.allocated().end()) CHECK(it->first >= f.first + f.second);
    if (it != p.allocated().begin()) {
      auto pr = std::prev(it);
      CHECK(pr->first + pr->second <= f.first);
    }
  }
  CHECK(p.used() == used);
  CHECK(used + free_sum == p.size());
}

static void allocator_random() {
  std::mt19937_64 rng(12345);
  PoolAlloc p(256 * 1000);
  std::vector<size_t> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3) {
      const size_t bytes = 1 + rng() % (256 * 60);
      // first fit: the lowest free range that holds the aligned size
      size_t expect = (size_t)-1;
      for (auto& f : p.free_ranges())
        if (f.second >= pool_align(bytes)) {
          expect = f.first;
          break;
        }
      size_t off = 0;
      const bool ok = p.alloc(bytes, &off);
      CHECK(ok == (expect != (size_t)-1));
      if (ok) {
        CHECK(off == expect);
        live.push_back(off);
      }
    } else {
      const size_t i = rng() % live.size();
      p.release(live[i]);
      live.erase(live.begin() + i);
    }
    check_pool(p);
  }
  for (size_t off : live) p.release(off);
  check_pool(p);
  CHECK(p.used() == 0 && p.free_ranges().size() == 1);
  p.release(12345 * 256);  // not an allocation: ignored
  check_pool(p);
}

static void admission_cases() {
  // no slot, or nothing queued
  CHECK(pick_admission({1, 2}, {5, 5}, 2, 0) == -1);
  CHECK(pick_admission({}, {}, 4, 0) == -1);
  // arrival order: always the head
  CHECK(pick_admission({9e9, 1}, {9e9}, 4, 0) == 0);
  // size-aware: a large request waits while another large one runs, small ones pass it
  CHECK(pick_admission({9e9, 9e9, 1, 2}, {5e9}, 4, 1e9) == 2);
  CHECK(pick_admission({9e9, 9e9}, {5e9}, 4, 1e9) == -1);
  // ... and runs when no large request does
  CHECK(pick_admission({9e9, 1}, {5e8, 1}, 4, 1e9) == 0);
  // the threshold is strict: a request of exactly big_work is not large
  CHECK(pick_admission({1e9}, {5e9}, 4, 1e9) == 0);
}

struct FakeRequest {
  size_t bytes;
  double work;
  int blocks;  // blocks until the fake certificate meets the target
  int id;
  size_t off = 0;
  int admitted_at = -1, done_at = -1;
};

// The server's boundary loop with a fake executor; returns the requests in
// completion order after checking the invariants at every boundary.
static std::vector<FakeRequest> simulate(std::vector<FakeRequest> reqs, size_t pool_bytes, int max_slots,
                                         double big_work) {
  PoolAlloc pool(pool_bytes);
  std::deque<FakeRequest> queue(reqs.begin(), reqs.end());
  std::vector<FakeRequest> running, done;
  std::vector<int> admitted_ids;
  for (int boundary = 0; boundary < 100000 && (!queue.empty() || !running.empty()); ++boundary) {
    while (!queue.empty()) {
      std::vector<double> qw, rw;
      for (auto& r : queue) qw.push_back(r.work);
      for (auto& r : running) rw.push_back(r.work);
      const int pi = pick_admission(qw, rw, max_slots, big_work);
      if (pi < 0) break;
      FakeRequest r = queue[pi];
      if (!pool.alloc(r.bytes, &r.off)) break;  // waits for memory; nothing passes it
      r.admitted_at = boundary;
      admitted_ids.push_back(r.id);
      queue.erase(queue.begin() + pi);
      running.push_back(r);
    }
    // invariants at the block boundary
    CHECK((int)running.size() <= max_slots);
    size_t sum = 0;
    int big = 0;
    for (auto& r : running) {
      sum += pool_align(r.bytes);
      big += big_work > 0 && r.work > big_work;
    }
    CHECK(sum == pool.used() && sum <= pool_bytes);
    CHECK(big <= 1 || big_work == 0);
    if (!queue.empty() && running.empty()) CHECK(false);  // a queued request that fits an empty pool runs
    // one block of every running request, then the finished ones retire
    std::vector<FakeRequest> still;
    for (auto& r : running) {
      if (--r.blocks == 0) {
        r.done_at = boundary;
        pool.release(r.off);
        done.push_back(r);
      } else {
        still.push_back(r);
      }
    }
    running.swap(still);
    check_pool(pool);
  }
  CHECK(queue.empty() && running.empty());
  CHECK(done.size() == reqs.size());
  CHECK(pool.used() == 0);
  if (big_work == 0) {
    // arrival order: requests are admitted exactly in submission order
    for (size_t i = 0; i < admitted_ids.size(); ++i) CHECK(admitted_ids[i] == reqs[i].id);
  }
  return done;
}

static void server_loop() {
  const size_t MB = 1 << 20;
  std::mt19937_64 rng(777);
  for (int trial = 0; trial < 40; ++trial) {
    std::vector<FakeRequest> reqs;
    for (int i = 0; i < 60; ++i) {
      const bool large = rng() % 5 == 0;
      reqs.push_back(FakeRequest{(size_t)(1 + rng() % (large ? 40 : 8)) * MB, large ? 4e9 : 1e6 * (1 + rng() % 100),
                                 1 + (int)(rng() % (large ? 12 : 4)), i});
    }
    const int slots = 1 + (int)(rng() % 8);
    simulate(reqs, 64 * MB, slots, 0);
    simulate(reqs, 64 * MB, slots, 1e9);
  }
  // head-of-line blocking by memory in arrival order: the 40 MB request waits
  // for the 30 MB one to finish, and the small one behind it waits too
  std::vector<FakeRequest> hol = {{30 * MB, 1, 5, 0}, {40 * MB, 1, 1, 1}, {1 * MB, 1, 1, 2}};
  auto d = simulate(hol, 64 * MB, 8, 0);
  CHECK(d.size() == 3 && d[0].id == 0 && d[1].id == 1 && d[2].id == 2);
  // size-aware: two large requests never share a block, the small ones ride along
  std::vector<FakeRequest> sa = {{8 * MB, 5e9, 6, 0}, {8 * MB, 5e9, 6, 1}, {1 * MB, 1e6, 1, 2}, {1 * MB, 1e6, 1, 3}};
  auto e = simulate(sa, 64 * MB, 8, 1e9);
  CHECK(e.size() == 4);
  int small_done_first = 0;
  for (auto& r : e)
    if (r.id >= 2) small_done_first += r.done_at < 6;
  CHECK(small_done_first == 2);  // the small ones finished while the first large one ran
  for (auto& r : e)
    if (r.id == 1) CHECK(r.admitted_at >= 6);  // the second large one waited for the first
}

// Admission with the batch engine's region (place_with_engine): the engine
// needs a region that grows with the running set; a request is admitted only
// when its workspace and the grown region both fit, so no admitted request
// ever finds the engine without room.  Random workloads in a tight pool, the
// invariants checked after every admission and every retirement.
static void engine_admission() {
  using bdrs_sched::place_with_engine;
  const size_t KB = 1024;
  // exact cases: a pool of 10 units of 256 KiB
  {
    PoolAlloc pool(10 * 256 * KB);
    size_t eoff = 0, ebytes = 0, w1 = 0, w2 = 0, w3 = 0;
    bool moved = false;
    CHECK(place_with_engine(pool, 3 * 256 * KB, 1 * 256 * KB, &w1, &eoff, &ebytes, &moved));
    CHECK(moved && ebytes == 256 * KB && pool.used() == 4 * 256 * KB);
    CHECK(place_with_engine(pool, 3 * 256 * KB, 2 * 256 * KB, &w2, &eoff, &ebytes, &moved));
    CHECK(moved && ebytes == 2 * 256 * KB && pool.used() == 8 * 256 * KB);
    // the workspace would fit (2 units free) but not with the grown region
    // (2 + 3 units against the 2 free and the engine's 2): the request waits
    // and the pool is as before (the engine's region taken again)
    const size_t used = pool.used();
    CHECK(!place_with_engine(pool, 2 * 256 * KB, 3 * 256 * KB, &w3, &eoff, &ebytes, &moved));
    CHECK(pool.used() == used && ebytes == 2 * 256 * KB);
    CHECK(pool.allocated().count(eoff) == 1);
    // a region that is already large enough is left alone
    pool.release(w1);
    CHECK(place_with_engine(pool, 256 * KB, 2 * 256 * KB, &w3, &eoff, &ebytes, &moved));
    CHECK(!moved && ebytes == 2 * 256 * KB);
    check_pool(pool);
  }
  std::mt19937_64 rng(4242);
  for (int trial = 0; trial < 200; ++trial) {
    PoolAlloc pool((size_t)(8 + rng() % 24) * 256 * KB);
    struct R {
      size_t ws, items, off;
      int blocks;
    };
    std::deque<R> queue;
    for (int i = 0; i < 30; ++i)
      queue.push_back(R{(size_t)(1 + rng() % 4) * 256 * KB - (rng() % 200), (size_t)(1 + rng() % 64) * KB, 0,
                        1 + (int)(rng() % 5)});
    std::vector<R> running;
    size_t eoff = 0, ebytes = 0;
    auto need_of = [&](const std::vector<R>& set, const R* extra) {
      size_t n = 4 * KB;  // descriptors and the fixed part
      for (auto& r : set) n += r.items;
      if (extra) n += extra->items;
      return n;
    };
    int guard = 0;
    while ((!queue.empty() || !running.empty()) && ++guard < 10000) {
      while (!queue.empty() && running.size() < 6) {
        R r = queue.front();
        bool moved = false;
        const size_t before = pool.used();
        const size_t need = need_of(running, &r);
        if (!place_with_engine(pool, r.ws, need, &r.off, &eoff, &ebytes, &moved)) {
          CHECK(pool.used() == before);
          break;
        }
        queue.pop_front();
        running.push_back(r);
        // the engine's region holds the grown set's work lists
        CHECK(ebytes >= pool_align(need_of(running, nullptr)));
        CHECK(pool.allocated().count(eoff) == 1 && pool.allocated().at(eoff) == ebytes);
      }
      size_t sum = ebytes;
      for (auto& r : running) sum += pool_align(r.ws);
      CHECK(sum == pool.used());
      // with nothing running a request waits only if it can never fit
      if (running.empty() && !queue.empty()) {
        const R& r = queue.front();
        CHECK(pool.used() == ebytes);
        CHECK(pool_align(r.ws) + pool_align(need_of({}, &r)) > pool.size());
        queue.pop_front();  // the server rejects such a request at submit
        continue;
      }
      std::vector<R> still;
      for (auto& r : running) {
        if (--r.blocks == 0) pool.release(r.off);
        else still.push_back(r);
      }
      running.swap(still);
      check_pool(pool);
    }
    CHECK(guard < 10000);
    if (ebytes) pool.release(eoff);
    CHECK(pool.used() == 0);
  }
}

int main() {
  allocator_random();
  admission_cases();
  server_loop();
  engine_admission();
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
