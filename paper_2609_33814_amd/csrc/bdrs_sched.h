// Host-only scheduling pieces of the solve server (no HIP): the first-fit
// allocator of the server's memory pool and the admission choice made at every
// block boundary.  Kept apart from the worker thread so that they can be
// exercised on a machine without a GPU.
#ifndef BDRS_SCHED_H_
#define BDRS_SCHED_H_

#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace bdrs_sched {

constexpr size_t kPoolAlign = 256;
inline size_t pool_align(size_t v) { return (v + kPoolAlign - 1) / kPoolAlign * kPoolAlign; }

// First-fit allocator over [0, size) in 256-byte units (bookkeeping only: it
// hands out offsets into memory it never touches).  Freed ranges merge with
// their free neighbours.
class PoolAlloc {
 public:
  explicit PoolAlloc(size_t size) : size_(size) {
    if (size_) free_[0] = size_;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = pool_align(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        sizes_[*off] = bytes;
        return true;
      }
    }
    return false;
  }
  // releases an offset alloc returned; other offsets are ignored
  void release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t bytes = s->second;
    sizes_.erase(s);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      free_.erase(next);
    }
    auto it = free_.lower_bound(off);
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  const std::map<size_t, size_t>& free_ranges() const { return free_; }      // offset -> bytes
  const std::map<size_t, size_t>& allocated() const { return sizes_; }       // offset -> bytes

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
  std::map<size_t, size_t> sizes_;
};

// Which queued request to admit next, as an index into the queue (arrival
// order), or -1 for none: no slot is free, or with the size-aware policy
// (big_work > 0) a request with more implicit entries per sweep than big_work
// waits while another such request runs, and the first request behind it that
// is not large is taken instead.  With big_work = 0 it is always the head.
// The caller then tries to place the pick in the pool; when it does not fit,
// admission stops for this boundary (nothing passes a request that waits for
// memory).
inline int pick_admission(const std::vector<double>& queued_work, const std::vector<double>& running_work,
                          int max_slots, double big_work) {
  if ((int)running_work.size() >= max_slots || queued_work.empty()) return -1;
  bool big_running = false;
  if (big_work > 0)
    for (double w : running_work) big_running = big_running || w > big_work;
  for (size_t i = 0; i < queued_work.size(); ++i)
    if (!(big_work > 0 && big_running && queued_work[i] > big_work)) return (int)i;
  return -1;
}

// Places a request's workspace together with the region of the batch engine
// (descriptors and work lists of all running requests), which grows with
// every admission: *eng_off / *eng_bytes describe the engine's current region
// (*eng_bytes = 0: none) and eng_need what it needs once the request runs.
// If the region is large enough and the workspace fits beside it, only the
// workspace is placed.  Otherwise the region is released and the workspace
// and a region of eng_need bytes are taken; if either does not fit, both are
// given back and the old region is taken again (it fits: the free ranges are
// the same as before it was released), and the request waits.  *moved
// reports whether the engine's region changed (its contents must then be
// bound again).  Returns true when the request is placed (workspace at
// *ws_off).  With nothing running, a waiting request therefore fails only if
// its workspace and its engine region together exceed the pool.
inline bool place_with_engine(PoolAlloc& pool, size_t ws_bytes, size_t eng_need, size_t* ws_off, size_t* eng_off,
                              size_t* eng_bytes, bool* moved) {
  *moved = false;
  if (pool_align(eng_need) <= *eng_bytes && pool.alloc(ws_bytes, ws_off)) return true;
  const size_t old_off = *eng_off, old_bytes = *eng_bytes;
  if (old_bytes) pool.release(old_off);
  size_t wo = 0, eo = 0;
  if (pool.alloc(ws_bytes, &wo)) {
    if (pool.alloc(eng_need, &eo)) {
      *ws_off = wo;
      *eng_off = eo;
      *eng_bytes = pool_align(eng_need);
      *moved = true;
      return true;
    }
    pool.release(wo);
  }
  if (old_bytes) {
    size_t back = 0;
    if (pool.alloc(old_bytes, &back)) {
      *moved = back != old_off;
      *eng_off = back;
    } else {  // cannot happen (see above); the region is then gone
      *eng_bytes = 0;
      *moved = true;
    }
  }
  return false;
}

}  // namespace bdrs_sched

#endif  // BDRS_SCHED_H_
