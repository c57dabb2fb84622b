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
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "phprng.h"
#include "serve_ranges.hpp"

namespace {

using phprng::serve::Arena;
using phprng::serve::LiveRanges;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pending {
  uint64_t ticket, tag, count;
  uint32_t instance;
  int64_t t_submit;
};

struct Batch {
  hipEvent_t done = nullptr;
  int stream = 0;  // index of the stream it was launched on
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

  // Two locks, so that submitters, the scheduler and releasers rarely wait
  // for each other: mu guards the request queue and the completions, amu
  // the arena, the live ranges and the counters.  Never hold amu while
  // taking mu.
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> pending;
  // pending.size(), readable without the lock: the scheduler polls it while
  // batches run, and taking mu in that loop would starve submitters
  std::atomic<size_t> npending{0};
  std::deque<phprng_completion> completions;
  uint64_t next_ticket = 1;

  std::mutex amu;
  LiveRanges live;
  phprng_server_counters counters{};
  std::atomic<uint64_t> releases{0};     // arena releases so far
  std::atomic<bool> arena_blocked{false};  // the oldest request did not fit
  uint64_t blocked_at = 0;               // releases when that was found (scheduler only)

  uint64_t ninst = 0;
  // scheduler-only scratch, kept across batches so that forming one
  // allocates nothing in the steady state
  std::vector<Pending> take;
  std::vector<phprng_request> reqs;
  std::vector<phprng_completion> meta;
  std::vector<uint64_t> pos;        // per instance: position after the batch so far, or kNoPos
  std::vector<uint32_t> pos_touched;
  static constexpr uint64_t kNoPos = ~0ull;
  std::atomic<bool> stop{false};
  std::thread thread;

  void loop();
  bool retire_finished();
  bool launch_batch(Batch &b);
  phprng_status release_many(const uint64_t *tickets, uint64_t n);

  // Frees what was created, also after a failed create; the scheduler
  // thread must have been joined.
  ~phprng_server() {
    for (auto &b : batches)
      if (b.done) (void)hipEventDestroy(b.done);
    for (auto st : streams) (void)hipStreamDestroy(st);
    if (arena_ptr) (void)hipFree(arena_ptr);
    delete arena;
  }
};

bool phprng_server::retire_finished() {
  bool any = false;
  int64_t spent = 0;
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
    spent += now_ns() - t;
  }
  if (any) {
    cv_done.notify_all();
    std::lock_guard<std::mutex> lk(amu);
    counters.retire_ns += spent;
  }
  return any;
}

bool phprng_server::launch_batch(Batch &b) {
  const int64_t t_form = now_ns();
  // take the batch's candidates off the queue (batch limits only) ...
  take.clear();
  {
    std::lock_guard<std::mutex> lk(mu);
    uint64_t draws = 0;
    while (!pending.empty() && take.size() < cfg.max_batch_requests) {
      const Pending &p = pending.front();
      if (!take.empty() && draws + p.count > cfg.max_batch_draws) break;
      draws += p.count;
      take.push_back(p);
      pending.pop_front();
    }
    npending.store(pending.size());
  }
  if (take.empty()) return false;
  // ... then admit them in FIFO order while the arena has room
  reqs.clear();
  meta.clear();
  size_t fit = 0;
  {
    std::lock_guard<std::mutex> lk(amu);
    for (; fit < take.size(); ++fit) {
      const Pending &p = take[fit];
      uint64_t off = 0;
      if (!arena->alloc(p.count, &off)) {
        counters.arena_stalls += 1;
        break;
      }
      reqs.push_back(phprng_request{p.instance, 0, p.count, off});
      phprng_completion c;
      memset(&c, 0, sizeof c);
      c.ticket = p.ticket;
      c.tag = p.tag;
      c.instance = p.instance;
      c.count = p.count;
      c.data = arena_ptr + off;
      c.t_submit_ns = p.t_submit;
      live.add(p.ticket, off, p.count);
      meta.push_back(c);
    }
    counters.arena_peak = std::max(counters.arena_peak, arena->used());
    if (fit == 0) blocked_at = releases.load();
    arena_blocked.store(fit == 0);
  }
  if (fit < take.size()) {
    // the rest waits for arena room, still at the head of the queue
    std::lock_guard<std::mutex> lk(mu);
    pending.insert(pending.begin(), take.begin() + (std::ptrdiff_t)fit, take.end());
    npending.store(pending.size());
  }
  if (reqs.empty()) return false;
  // positions before the draws of each request (request order = FIFO order)
  for (size_t i = 0; i < reqs.size(); ++i) {
    const uint32_t id = reqs[i].instance;
    if (pos[id] == kNoPos) {
      uint64_t k = 0;
      phprng_get_position(ctx, id, &k);
      pos[id] = k;
      pos_touched.push_back(id);
    }
    meta[i].k = pos[id];
    pos[id] += reqs[i].count;
  }
  for (uint32_t id : pos_touched) pos[id] = kNoPos;
  pos_touched.clear();
  const int64_t t_admit = now_ns();
  // the stream with the fewest batches on it, the rotation breaking ties, so
  // that a batch queues behind another only when every stream is busy
  const int ns = (int)streams.size();
  int pick = -1, best = 0;
  for (int i = 0; i < ns; ++i) {
    const int si = (next_stream + i) % ns;
    int load = 0;
    for (const auto &o : batches) load += (o.active && o.stream == si) ? 1 : 0;
    if (pick < 0 || load < best) {
      pick = si;
      best = load;
    }
  }
  next_stream = (pick + 1) % ns;
  b.stream = pick;
  hipStream_t s = streams[pick];
  phprng_status st = phprng_generate(ctx, reqs.data(), reqs.size(), nullptr, nullptr, arena_ptr,
                                     cfg.arena_doubles, (void *)s, PHPRNG_MODE_PERSISTENT);
  if (st == PHPRNG_OK && hipEventRecord(b.done, s) != hipSuccess) st = PHPRNG_E_DEVICE;
  {
    const int64_t dt = now_ns() - t_admit;
    uint64_t draws = 0;
    for (const auto &r : reqs) draws += r.count;
    std::lock_guard<std::mutex> lk(amu);
    counters.batches += 1;
    counters.requests += reqs.size();
    counters.draws += draws;
    counters.launch_ns += dt;
    counters.launch_ns_max = std::max(counters.launch_ns_max, dt);
    counters.form_ns += t_admit - t_form;
  }
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
  b.reqs.swap(meta);  // meta takes the retired batch's emptied buffer
  b.active = true;
  return true;
}

void phprng_server::loop() {
  while (!stop.load()) {
    bool progress = retire_finished();
    for (auto &b : batches) {
      if (b.active) continue;
      if (npending.load() == 0) break;
      if (arena_blocked.load() && releases.load() == blocked_at) break;  // no room yet
      if (!launch_batch(b)) break;
      progress = true;
    }
    if (!progress) {
      bool inflight = false;
      for (auto &b : batches) inflight = inflight || b.active;
      if (inflight) {
        // a batch is on the device: keep polling its event (completion times
        // are taken here, so the loop spins rather than sleeps) without
        // touching the lock
        std::this_thread::yield();
      } else {
        // idle, or the arena has no room for the oldest request: sleep until
        // a submission, or a release in the second case
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::microseconds(200), [&] {
          if (stop.load()) return true;
          if (arena_blocked.load() && releases.load() == blocked_at) return false;
          return !pending.empty();
        });
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
  if (c.max_inflight <= 0) c.max_inflight = std::min(c.streams + 1, 6);
  if (c.max_batch_requests == 0) c.max_batch_requests = 8192;
  if (c.max_batch_draws == 0) c.max_batch_draws = 1ull << 28;
  if (c.streams > 8 || c.max_inflight > 6 || c.max_batch_requests > (1u << 24)) return PHPRNG_E_INVALID;
  std::unique_ptr<phprng_server> s(new (std::nothrow) phprng_server);
  if (!s) return PHPRNG_E_NOMEM;
  s->ctx = ctx;
  s->cfg = c;
  s->ninst = phprng_instance_count(ctx);
  try {
    s->pos.assign(s->ninst, phprng_server::kNoPos);
  } catch (...) {
    return PHPRNG_E_NOMEM;
  }
  if (hipMalloc(&s->arena_ptr, c.arena_doubles * sizeof(double)) != hipSuccess) {
    s->arena_ptr = nullptr;
    return PHPRNG_E_NOMEM;
  }
  s->arena = new (std::nothrow) Arena(c.arena_doubles);
  if (!s->arena) return PHPRNG_E_NOMEM;
  for (int i = 0; i < c.streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return PHPRNG_E_DEVICE;
    s->streams.push_back(st);
  }
  s->batches.resize(c.max_inflight);
  for (auto &b : s->batches) {
    if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
      b.done = nullptr;
      return PHPRNG_E_DEVICE;
    }
  }
  try {
    s->thread = std::thread([raw = s.get()] { raw->loop(); });
  } catch (...) {
    return PHPRNG_E_NOMEM;  // no thread: nothing runs, the destructor frees the rest
  }
  *out = s.release();
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
    s->npending.store(s->pending.size());
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

phprng_status phprng_server::release_many(const uint64_t *tickets, uint64_t n) {
  phprng_status st = PHPRNG_OK;
  uint64_t k = 0;
  {
    std::lock_guard<std::mutex> lk(amu);
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t off = 0, count = 0;
      if (!live.take(tickets[i], &off, &count)) {
        st = PHPRNG_E_INVALID;
        continue;
      }
      arena->release(off, count);
      ++k;
    }
    releases.fetch_add(k);
  }
  if (k) {
    // a scheduler blocked on the arena checks `releases` under mu before it
    // sleeps: passing through mu orders this release before its next check
    if (arena_blocked.load()) {
      std::lock_guard<std::mutex> lk(mu);
    }
    cv_work.notify_one();
  }
  return st;
}

extern "C" phprng_status phprng_server_release(phprng_server *s, uint64_t ticket) {
  if (!s) return PHPRNG_E_INVALID;
  return s->release_many(&ticket, 1);
}

extern "C" phprng_status phprng_server_release_many(phprng_server *s, const uint64_t *tickets, uint64_t n) {
  if (!s || (n > 0 && !tickets)) return PHPRNG_E_INVALID;
  return s->release_many(tickets, n);
}

extern "C" phprng_status phprng_server_stats(phprng_server *s, uint64_t *pending, uint64_t *arena_used) {
  if (!s) return PHPRNG_E_INVALID;
  if (pending) {
    std::lock_guard<std::mutex> lk(s->mu);
    *pending = s->pending.size();
  }
  if (arena_used) {
    std::lock_guard<std::mutex> lk(s->amu);
    *arena_used = s->arena->used();
  }
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_read_counters(phprng_server *s, phprng_server_counters *out, int reset) {
  if (!s || !out) return PHPRNG_E_INVALID;
  std::lock_guard<std::mutex> lk(s->amu);
  *out = s->counters;
  if (reset) s->counters = phprng_server_counters{};
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_destroy(phprng_server *s) {
  if (!s) return PHPRNG_E_INVALID;
  s->stop.store(true);
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  delete s;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_server_replay(phprng_server *s, const phprng_arrival *arr, uint64_t n,
                                              int64_t *latency_ns, int64_t *admit_ns, double *wall_s) {
  if (!s || (n > 0 && (!arr || !latency_ns)) || !wall_s) return PHPRNG_E_INVALID;
  for (uint64_t i = 0; i < n; ++i)
    if (arr[i].instance >= s->ninst || arr[i].count > s->cfg.arena_doubles) return PHPRNG_E_INVALID;
  const int64_t t0 = now_ns() + 2000000;  // first arrival 2 ms from now
  std::atomic<int> submit_status{PHPRNG_OK};
  std::thread submitter([&] {
    // every arrival that is due goes into the queue under one lock; tag =
    // arrival index, and latency is measured from the scheduled arrival
    uint64_t i = 0;
    while (i < n) {
      if (now_ns() < t0 + arr[i].t_ns) continue;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        const int64_t t = now_ns();
        for (; i < n && t0 + arr[i].t_ns <= t; ++i)
          s->pending.push_back(Pending{s->next_ticket++, i, arr[i].count, arr[i].instance, t});
        s->npending.store(s->pending.size());
      }
      s->cv_work.notify_one();
    }
  });
  phprng_status result = PHPRNG_OK;
  uint64_t done = 0;
  std::vector<phprng_completion> buf(1024);
  std::vector<uint64_t> tickets(buf.size());
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
        if (admit_ns) admit_ns[i] = c.status == PHPRNG_OK ? c.t_admit_ns - (t0 + arr[i].t_ns) : -1;
        if (c.status != PHPRNG_OK) result = (phprng_status)c.status;
      }
      t_last = std::max(t_last, c.t_done_ns);
      tickets[j] = c.ticket;
      ++done;
    }
    s->release_many(tickets.data(), k);
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
