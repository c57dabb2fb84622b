// Randomised check of the serving arena's bookkeeping against brute force:
// the first-fit allocator against a per-element occupancy scan, and the live
// ranges against an ordered map.  Prints "ok" and exits 0 on success.
#include <cstdint>
#include <cstdio>
#include <map>
#include <random>
#include <utility>
#include <vector>

#include "serve_ranges.hpp"

using phprng::serve::Arena;
using phprng::serve::LiveRanges;

static int check_arena(std::mt19937_64 &g, int trials, int ops) {
  for (int t = 0; t < trials; ++t) {
    const uint64_t cap = 1 + g() % 5000;
    Arena a(cap);
    std::vector<char> used(cap, 0);
    std::vector<std::pair<uint64_t, uint64_t>> held;
    for (int op = 0; op < ops; ++op) {
      if (held.empty() || g() % 2) {
        const uint64_t n = g() % 200;
        // brute force: the lowest offset of n consecutive free elements
        uint64_t want = n == 0 ? 0 : ~0ull, run = 0;
        for (uint64_t i = 0; n && i < cap; ++i) {
          run = used[i] ? 0 : run + 1;
          if (run == n) {
            want = i + 1 - n;
            break;
          }
        }
        uint64_t off = 0;
        const bool ok = a.alloc(n, &off);
        if (ok != (want != ~0ull) || (ok && off != want)) {
          std::printf("arena: trial %d op %d n %llu got %d/%llu want %llu\n", t, op, (unsigned long long)n, ok,
                      (unsigned long long)off, (unsigned long long)want);
          return 1;
        }
        if (ok) {
          for (uint64_t i = off; i < off + n; ++i) used[i] = 1;
          held.push_back({off, n});
        }
      } else {
        const size_t j = g() % held.size();
        const auto h = held[j];
        held.erase(held.begin() + (std::ptrdiff_t)j);
        a.release(h.first, h.second);
        for (uint64_t i = h.first; i < h.first + h.second; ++i) used[i] = 0;
      }
      uint64_t u = 0;
      for (char c : used) u += (uint64_t)c;
      if (u != a.used()) {
        std::printf("arena: trial %d op %d used %llu want %llu\n", t, op, (unsigned long long)a.used(),
                    (unsigned long long)u);
        return 1;
      }
    }
  }
  return 0;
}

static int check_live(std::mt19937_64 &g, int trials, int ops) {
  for (int t = 0; t < trials; ++t) {
    LiveRanges L;
    std::map<uint64_t, std::pair<uint64_t, uint64_t>> ref;
    uint64_t next = 1 + g() % 10;
    for (int op = 0; op < ops; ++op) {
      if (g() % 3 == 0) {
        next += g() % 3;  // some tickets are never admitted
        const uint64_t off = g(), count = g();
        L.add(next, off, count);
        ref[next] = {off, count};
        ++next;
      } else {
        const uint64_t ticket = g() % (next + 3);
        uint64_t off = 0, count = 0;
        const bool ok = L.take(ticket, &off, &count);
        auto it = ref.find(ticket);
        if (ok != (it != ref.end()) || (ok && (off != it->second.first || count != it->second.second))) {
          std::printf("live: trial %d op %d ticket %llu got %d\n", t, op, (unsigned long long)ticket, ok);
          return 1;
        }
        if (ok) ref.erase(it);
      }
    }
  }
  return 0;
}

int main() {
  std::mt19937_64 g(0x14112484);
  if (check_arena(g, 200, 3000) || check_live(g, 200, 5000)) return 1;
  std::printf("ok\n");
  return 0;
}
