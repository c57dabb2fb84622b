// Serving loop: continuous batching of generation requests over the
// instances of one context.  Built only on the public C interface.
//
//   submit  -> pending FIFO (any thread)
//   scheduler thread:
//     - retire finished batches (event query) into the completion queue;
//     - admit pending requests in FIFO order while the device output arena
//       has room (memory admission) and the batch limits allow, reserve their
//       positions (phprng_generate does this in request order) and launch the
//       batch on the next stream, so that a new batch runs while earlier ones
//       are still on the device;
//   poll    -> completions (device pointer into the arena, valid until release)
//   release -> the arena range returns to the free list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "phprng.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, capacity) elements with coalescing frees.
class Arena {
 public:
  explicit Arena(uint64_t cap) { free_[0] = cap; }
  bool alloc(uint64_t n, uint64_t *off) {
    if (n == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    if (n == 0) return;
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }

 private:
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Pending {
  uint64_t ticket, tag, count;
  uint32_t instance;
  int64_t t_submit;
};

struct Batch {
  hipEvent_t done = nullptr;
  std::vector<phprng_completion> reqs;
  bool active = false;
};

}  // namespace

struct phprng_server {
  phprng_ctx *ctx = nullptr;
  phprng_server_config cfg{};
  double *arena_ptr = nullptr;
  Arena *arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<Batch> batches;  // max_inflight entries
  int next_stream = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> pending;
  std::deque<phprng_completion> completions;
  std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> live;  // ticket -> (offset, count)
  uint64_t next_ticket = 1;
  uint64_t ninst = 0;
  std::atomic<bool> stop{false};
  std::thread thread;
  phprng_status sticky = PHPRNG_OK;

  void loop();
  bool retire_finished();
  bool launch_batch(Batch &b);
};

bool phprng_server::retire_finished() {
  bool any = false;
  for (auto &b : batches) {
    if (!b.active) continue;
    hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) continue;
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lk(mu);
    for (auto &c : b.reqs) {
      c.t_done_ns = t;
      if (q != hipSuccess) c.status = PHPRNG_E_DEVICE;
      completions.push_back(c);
    }
    b.reqs.clear();
    b.active = false;
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

bool phprng_server::launch_batch(Batch &b) {
  std::vector<phprng_request> reqs;
  std::vector<phprng_completion> meta;
  {
    std::lock_guard<std::mutex> lk(mu);
    uint64_t draws = 0;
    while (!pending.empty() && reqs.size() < cfg.max_batch_requests) {
      const Pending &p = pending.front();
      if (!reqs.empty() && draws + p.count > cfg.max_batch_draws) break;
      uint64_t off = 0;
      if (!arena->alloc(p.count, &off)) break;  // memory admission: wait for releases
      phprng_request r{p.instance, 0, p.count, off};
      reqs.push_back(r);
      phprng_completion c;
      memset(&c, 0, sizeof c);
      c.ticket = p.ticket;
      c.tag = p.tag;
      c.instance = p.instance;
      c.count = p.count;
      c.data = arena_ptr + off;
      c.t_submit_ns = p.t_submit;
      live[p.ticket] = {off, p.count};
      meta.push_back(c);
      draws += p.count;
      pending.pop_front();
    }
  }
  if (reqs.empty()) return false;
  // positions before the draws of each request (request order = FIFO order)
  std::unordered_map<uint32_t, uint64_t> pos;
  for (size_t i = 0; i < reqs.size(); ++i) {
    auto it = pos.find(reqs[i].instance);
    if (it == pos.end()) {
      uint64_t k = 0;
      phprng_get_position(ctx, reqs[i].instance, &k);
      it = pos.emplace(reqs[i].instance, k).first;
    }
    meta[i].k = it->second;
    it->second += reqs[i].count;
  }
  const int64_t t_admit = now_ns();
  hipStream_t s = streams[next_stream];
  next_stream = (next_stream + 1) % (int)streams.size();
  phprng_status st = phprng_generate(ctx, reqs.data(), reqs.size(), nullptr, nullptr, arena_ptr,
                                     cfg.arena_doubles, (void *)s, PHPRNG_MODE_PERSISTENT);
  if (st == PHPRNG_OK && hipEventRecord(b.done, s) != hipSuccess) st = PHPRNG_E_DEVICE;
  for (auto &c : meta) {
    c.t_admit_ns = t_admit;
    c.status = st;
  }
  if (st != PHPRNG_OK) {
    // report the failure on every request of the batch; nothing was launched
    std::lock_guard<std::mutex> lk(mu);
    for (auto &c : meta) completions.push_back(c);
    cv_done.notify_all();
    return true;
  }
  b.reqs = std::move(meta);
  b.active = true;
  return true;
}

void phprng_server::loop() {
  while (!stop.load()) {
    bool progress = retire_finished();
    for (auto &b : batches) {
      if (b.active) continue;
      bool have;
      {
        std::lock_guard<std::mutex> lk(mu);
        have = !pending.empty();
      }
      if (!have) break;
      if (!launch_batch(b)) break;
      progress = true;
    }
    if (!progress) {
      bool inflight = false;
      for (auto &b : batches) inflight = inflight || b.active;
      std::unique_lock<std::mutex> lk(mu);
      if (inflight) {
        // a batch is on the device: keep polling its event (completion times
        // are taken here, so the loop spins rather than sleeps)
        lk.unlock();
        std::this_thread::yield();
      } else {
        cv_work.wait_for(lk, std::chrono::microseconds(200),
                         [&] { return stop.load() || !pending.empty(); });
      }
    }
  }
  // drain: wait for every batch still on the device
  for (auto &b : batches)
    if (b.active) (void)hipEventSynchronize(b.done);
  retire_finished();
}

extern "C" phprng_status phprng_server_create(phprng_ctx *ctx, const phprng_server_config *cfg,
                                              phprng_server **out) {
  if (!ctx || !out) return PHPRNG_E_INVALID;
  *out = nullptr;
  phprng_server_config c{};
  if (cfg) c = *cfg;
  if (c.arena_doubles == 0) c.arena_doubles = 1ull << 28;
  if (c.streams <= 0) c.streams = 2;
  if (c.max_inflight <= 0) c.max_inflight = c.streams;
  if (c.max_batch_requests == 0) c.max_batch_requests = 8192;
  if (c.max_batch_draws == 0) c.max_batch_draws = 1ull << 28;
  if (c.streams > 8 || c.max_inflight > 6 || c.max_batch_requests > (1u << 24)) return PHPRNG_E_INVALID;
  std::unique_ptr<phprng_server> s(new (std::nothrow) phprng_server);
  if (!s) return PHPRNG_E_NOMEM;
  s->ctx = ctx;
  s->cfg = c;
  s->ninst = phprng_instance_count(ctx);
  if (hipMalloc(&s->arena_ptr, c.arena_doubles * sizeof(double)) != hipSuccess) return PHPRNG_E_NOMEM;
  s->arena = new Arena(c.arena_doubles);
  for (int i = 0; i < c.streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return PHPRNG_E_DEVICE;
    s->streams.push_back(st);
  }
  s->batches.resize(c.max_inflight);
  for (auto &b : s->batches)
    if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) return PHPRNG_E_DEVICE;
  phprng_server *raw = s.release();
  raw->thread = std::thread([raw] { raw->loop(); });
  *out = raw;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_submit(phprng_server *s, uint32_t instance, uint64_t count, uint64_t tag,
                                              uint64_t *ticket) {
  if (!s || !ticket) return PHPRNG_E_INVALID;
  if (instance >= s->ninst) return PHPRNG_E_INVALID;
  if (count > s->cfg.arena_doubles) return PHPRNG_E_RANGE;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    *ticket = s->next_ticket++;
    s->pending.push_back(Pending{*ticket, tag, count, instance, now_ns()});
  }
  s->cv_work.notify_one();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_poll(phprng_server *s, phprng_completion *out, uint64_t max, uint64_t *n,
                                            int64_t timeout_us) {
  if (!s || !n || (max > 0 && !out)) return PHPRNG_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->completions.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->completions.empty(); });
  uint64_t k = 0;
  while (k < max && !s->completions.empty()) {
    out[k++] = s->completions.front();
    s->completions.pop_front();
  }
  *n = k;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_release(phprng_server *s, uint64_t ticket) {
  if (!s) return PHPRNG_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->live.find(ticket);
  if (it == s->live.end()) return PHPRNG_E_INVALID;
  s->arena->release(it->second.first, it->second.second);
  s->live.erase(it);
  s->cv_work.notify_one();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_stats(phprng_server *s, uint64_t *pending, uint64_t *arena_used) {
  if (!s) return PHPRNG_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (pending) *pending = s->pending.size();
  if (arena_used) *arena_used = s->arena->used();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_destroy(phprng_server *s) {
  if (!s) return PHPRNG_E_INVALID;
  s->stop.store(true);
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  for (auto &b : s->batches)
    if (b.done) (void)hipEventDestroy(b.done);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  (void)hipFree(s->arena_ptr);
  delete s->arena;
  delete s;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_replay(phprng_server *s, const phprng_arrival *arr, uint64_t n,
                                              int64_t *latency_ns, double *wall_s) {
  if (!s || (n > 0 && (!arr || !latency_ns)) || !wall_s) return PHPRNG_E_INVALID;
  for (uint64_t i = 0; i < n; ++i)
    if (arr[i].instance >= s->ninst || arr[i].count > s->cfg.arena_doubles) return PHPRNG_E_INVALID;
  const int64_t t0 = now_ns() + 2000000;  // first arrival 2 ms from now
  std::atomic<int> submit_status{PHPRNG_OK};
  std::thread submitter([&] {
    for (uint64_t i = 0; i < n; ++i) {
      const int64_t due = t0 + arr[i].t_ns;
      while (now_ns() < due) {
      }
      uint64_t ticket;
      // tag = arrival index; latency is measured from the scheduled arrival
      if (phprng_server_submit(s, arr[i].instance, arr[i].count, i, &ticket) != PHPRNG_OK)
        submit_status.store(PHPRNG_E_INVALID);
    }
  });
  phprng_status result = PHPRNG_OK;
  uint64_t done = 0;
  std::vector<phprng_completion> buf(1024);
  int64_t t_last = t0;
  const int64_t deadline = t0 + (n ? arr[n - 1].t_ns : 0) + 120ll * 1000000000ll;
  while (done < n) {
    uint64_t k = 0;
    phprng_server_poll(s, buf.data(), buf.size(), &k, 1000);
    for (uint64_t j = 0; j < k; ++j) {
      const phprng_completion &c = buf[j];
      const uint64_t i = c.tag;
      if (i < n) {
        latency_ns[i] = c.status == PHPRNG_OK ? c.t_done_ns - (t0 + arr[i].t_ns) : -1;
        if (c.status != PHPRNG_OK) result = (phprng_status)c.status;
      }
      t_last = std::max(t_last, c.t_done_ns);
      phprng_server_release(s, c.ticket);
      ++done;
    }
    if (now_ns() > deadline) {
      result = PHPRNG_E_DEVICE;
      break;
    }
  }
  submitter.join();
  if (result == PHPRNG_OK) result = (phprng_status)submit_status.load();
  *wall_s = (double)(t_last - t0) * 1e-9;
  return result;
}
