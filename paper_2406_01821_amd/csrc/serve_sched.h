// Admission policy of the serving loop, free of device calls so that host
// tests can drive it with a simulated executor: a first-fit allocator of
// arena ranges and the choice of the FIFO prefix that the next launch takes.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace aerl {

// First-fit allocator of ranges of an arena of `bytes` bytes (callers keep
// sizes aligned).  Free ranges are kept sorted and coalesced on release.
class ArenaAlloc {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
    used_ = 0;
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
  bool alloc(size_t n, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, start = it->first + n;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += n;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  const std::map<size_t, size_t> &free_ranges() const { return free_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used_ = 0;
};

// Footprint of a queued request as admission sees it.
struct QueuedSize {
  size_t dev;  // device bytes: inputs, outputs and work tables
  size_t in;   // bytes staged to the device: inputs and tables
  size_t out;  // bytes copied back
};

// Number of requests, from the head of the FIFO `pending`, that the next
// launch takes: the longest prefix of at most max_batch requests whose
// device bytes plus `slack` fit in `room` (the largest free arena range)
// and, past the first request, whose staged inputs plus `slack` and whose
// outputs fit the slot's pinned buffers (in_cap, out_cap; a launch grows
// them only for a first request that needs more).  0 when the head does
// not fit in `room`: the queue waits for a launch to end (back-pressure; a
// later, smaller request never overtakes the head).  *need gets the arena
// bytes of the prefix.
template <class Seq, class SizeOf>
int32_t admit_prefix(const Seq &pending, SizeOf size_of, size_t room, int32_t max_batch,
                     size_t slack, size_t in_cap, size_t out_cap, size_t *need) {
  size_t dev = slack, in = slack, out = 0;
  int32_t n = 0;
  for (const auto &r : pending) {
    if (n >= max_batch) break;
    const QueuedSize q = size_of(r);
    if (dev + q.dev > room) break;
    if (n > 0 && (in + q.in > in_cap || out + q.out > out_cap)) break;
    dev += q.dev;
    in += q.in;
    out += q.out;
    ++n;
  }
  *need = dev;
  return n;
}

}  // namespace aerl
