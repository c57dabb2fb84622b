// Host-side bookkeeping of the serving loop's device output arena: a
// first-fit range allocator and the ranges of live requests by ticket.
// Plain C++ (no HIP), so that host tests can build it on its own.
#pragma once

#include <cstdint>
#include <deque>
#include <map>
#include <utility>

namespace phprng {
namespace serve {

// First-fit allocator over [0, capacity) elements with coalescing frees.
// Free ranges are keyed by their end: an allocation takes the front of a
// range and only moves its start, and a free that extends a range moves a
// node to its new key, so that in the steady state neither allocates memory.
class Arena {
 public:
  explicit Arena(uint64_t cap) { free_[cap] = 0; }
  bool alloc(uint64_t n, uint64_t *off) {
    if (n == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->first - it->second >= n) {
        *off = it->second;
        it->second += n;
        if (it->second == it->first) free_.erase(it);
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    if (n == 0) return;
    used_ -= n;
    const uint64_t end = off + n;
    auto prev = free_.find(off);        // the free range that ends where this one starts
    auto next = free_.upper_bound(end);  // the first range ending after this one
    const bool join_prev = prev != free_.end();
    const bool join_next = next != free_.end() && next->second == end;
    if (join_next) {
      next->second = join_prev ? prev->second : off;
      if (join_prev) free_.erase(prev);
    } else if (join_prev) {
      auto node = free_.extract(prev);
      node.key() = end;
      free_.insert(std::move(node));
    } else {
      free_.emplace(end, off);
    }
  }
  uint64_t used() const { return used_; }

 private:
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;  // end -> start
};

// Output ranges of admitted, unreleased requests by ticket.  Admission takes
// requests in ticket order, so the records form a queue indexed by ticket
// minus the front's ticket; the front advances past released tickets (an
// old ticket left unreleased holds the queue, 24 bytes per later request).
class LiveRanges {
 public:
  void add(uint64_t ticket, uint64_t off, uint64_t count) {
    if (q_.empty()) base_ = ticket;
    while (base_ + q_.size() < ticket) q_.push_back(Rec{0, 0, false});  // tickets never admitted
    q_.push_back(Rec{off, count, true});
  }
  bool take(uint64_t ticket, uint64_t *off, uint64_t *count) {
    if (ticket < base_ || ticket - base_ >= q_.size()) return false;
    Rec &r = q_[ticket - base_];
    if (!r.live) return false;
    *off = r.off;
    *count = r.count;
    r.live = false;
    while (!q_.empty() && !q_.front().live) {
      q_.pop_front();
      ++base_;
    }
    return true;
  }

 private:
  struct Rec {
    uint64_t off, count;
    bool live;
  };
  std::deque<Rec> q_;
  uint64_t base_ = 0;
};

}  // namespace serve
}  // namespace phprng
