// Host runtime behind include/phprng.h: instance tables, seeding, the skip
// tables, request planning and kernel launches, jumps and state restore,
// captured repeat draws and the allocation-free entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <unordered_set>
#include <vector>

#include "hostmath.hpp"
#include "kernels.hpp"
#include "layout.hpp"
#include "phprng.h"

using namespace phprng;

namespace {

struct HostInst {
  uint64_t n, e;
  int width;
  uint32_t sched = kSchedSkipLcg;
  uint64_t b = 0;      // constant skip
  uint64_t mbase = 0;  // width 32: m at internal index x is mbase + q p(p-1)/2 + U(r) mod n; constant skip: m_0
  uint64_t x = 0;      // width 32 / constant skip: internal index of the current state;
                       // width 64 pseudorandom skip: skip log t of the current state (s = a^t mod p), < p - 1
  uint64_t k = 0;      // position reported to the caller
};

bool lcg64(const HostInst &h) { return h.width == 64 && h.sched == kSchedSkipLcg; }

const SkipGroup &group(int width) {
  static const SkipGroup g32(kP32, kA32);
  static const SkipGroup g64(kP64, kA64);
  return width == 32 ? g32 : g64;
}

bool width_ok(int w) { return w == 32 || w == 64; }

phprng_status check_instance_impl(int width, uint64_t n, uint64_t e) {
  if (!width_ok(width)) return PHPRNG_E_INVALID;
  const uint64_t lo = width == 32 ? (1ull << 31) : (1ull << 62);
  if (n < lo || n >= 2 * lo) return PHPRNG_E_RANGE;
  if (!is_prime64(n)) return PHPRNG_E_NOT_PRIME;
  if (e < 3 || gcd64(e, n - 1) != 1 || e % (n - 1) == 1) return PHPRNG_E_EXPONENT;
  const uint64_t p = width == 32 ? kP32 : kP64;
  if (p >= n) return PHPRNG_E_RANGE;
  return PHPRNG_OK;
}

int bit_length(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// Batches of at most this many requests are read by the kernels from pinned
// host memory instead of a device copy.
constexpr uint64_t kDirectRequests = 1024;
// Planning vectors reserved at context creation.
constexpr uint64_t kPlanReserve = 16384;
static_assert(kNoAllocMaxRequests <= kPlanReserve, "allocation-free calls plan without growing a vector");

// The width-64 reduce shrinks its units until a batch has this many of them
// (its grid holds 2048 four-wave blocks).
constexpr uint64_t kReduceWaves = 8192;

// Width-64 draws per request: tiles are counted in 32 bits.
constexpr uint64_t kMaxCount64 = (uint64_t)kTile64 << 32;
// Width-64 jumps off the positioning table sum the skips on the device; the
// remainder of a jump modulo the skip period (or its complement) must stay
// below this many draws.
constexpr uint64_t kJumpMax = 1ull << 42;
constexpr unsigned kJumpBlocks = 2048;

// Launch-shape classes: batches of width-32 requests only, width-64 only, or
// both.
enum { kMix32 = 0, kMix64 = 1, kMixBoth = 2 };

// Process-wide cache of autotuned shapes, keyed by (architecture, compute
// units, class): a new context on the same kind of device starts from it.
struct TuneKey {
  std::string arch;
  int cus;
  int cls;
  bool operator<(const TuneKey &o) const { return std::tie(arch, cus, cls) < std::tie(o.arch, o.cus, o.cls); }
};
std::mutex g_tune_mu;
std::map<TuneKey, phprng_tuning> g_tune_cache;

uint64_t add_u64_mod(uint64_t x, uint64_t y, uint64_t m) {  // (x + y) mod m, x, y < m
  const uint64_t s = x + y;
  return (s < x || s >= m) ? s - m : s;
}

}  // namespace

struct phprng_graph {
  phprng_ctx *ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint8_t *d_blk = nullptr;  // batch header + requests, refreshed before every launch
  WorkCtr *d_ctr = nullptr;
  uint64_t *d_t64 = nullptr;  // width-64 tile state
  hipEvent_t done = nullptr;  // after the previous launch
  bool launched = false;
  std::vector<phprng_request> reqs;
  uint64_t nreq64 = 0;
  uint64_t cap64 = 0;  // width-64 tile-state entries: enough for either way of finding tile starts
  uint32_t tpc = 1;
  bool has64 = false;
  ~phprng_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_blk) (void)hipFree(d_blk);
    if (d_ctr) (void)hipFree(d_ctr);
    if (d_t64) (void)hipFree(d_t64);
    if (done) (void)hipEventDestroy(done);
  }
};

// Result of planning a request list.
struct Plan {
  uint64_t nreq = 0;
  uint64_t nreq64 = 0;   // width-64 pseudorandom-skip requests (first in the staging order)
  uint64_t tiles64 = 0;  // their tiles
  uint64_t units64 = 0;  // their reduce units (reduce_tiles tiles of one request)
  uint32_t reduce_tiles = kReduceTiles;
  bool any_tab = false;     // some width-64 instance takes its tile starts from the table
  bool any_reduce = false;  // some takes them from the reduce and scan
  uint64_t tiles = 0;    // all tiles
  uint64_t total_chunks = 0;
  uint32_t tpc = 1;
  bool has32 = false, has64 = false;
  int cls = kMix32;
};

struct phprng_ctx {
  int device = 0;
  int num_cus = 0;
  std::string arch;
  uint64_t max_instances = 0;
  std::vector<HostInst> inst;
  InstRec *d_inst = nullptr;
  LaneMul *d_lanemul = nullptr;
  uint64_t *d_m64 = nullptr;  // width-64 message at each instance's committed position
  // universal width-32 skip-prefix table: host mirror and device copy
  std::vector<uint64_t> u32;
  std::vector<uint32_t> s32;
  uint64_t *d_u32 = nullptr;
  uint32_t *d_s32 = nullptr;
  // width-64 positioning table (device only), built with the first width-64 instance
  uint64_t *d_u64lo = nullptr, *d_u64hi = nullptr, *d_s64 = nullptr;
  bool have64 = false;
  uint64_t *d_partial = nullptr;  // jump partial sums
  // Width-64 messages live on the device: each batch's scan reads and
  // commits them.  Scans of successive calls are ordered by this event, so
  // that calls on different streams still continue each stream in call order.
  hipEvent_t chain_ev = nullptr;
  bool chain_pending = false;
  // Request staging: a ring of slots so that consecutive calls (possibly on
  // different streams) never overwrite a request block still in use.  A slot
  // is reused only after the event recorded behind its last kernel.
  struct Slot {
    uint8_t *h_blk = nullptr;            // pinned, mapped: BatchHdr + ReqRec[cap]
    const uint8_t *h_blk_dev = nullptr;  // h_blk's address for kernels
    uint8_t *d_blk = nullptr;            // device copy
    uint64_t cap = 0;
    WorkCtr *d_ctr = nullptr;
    uint64_t *d_t64 = nullptr;  // 3 * cap64 words
    uint64_t cap64 = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the call's kernels; ev1 also marks the slot free
    bool busy = false;
    bool timed = false;  // ev0 was recorded before the call's kernels
  };
  static constexpr int kSlots = 8;
  static constexpr uint64_t kMinSlotRequests = 8192;
  Slot slots[kSlots];
  int cur_slot = 0;
  int last_timed = -1;
  bool timing_on = true;  // record ev0 before each call's kernels (phprng_set_timing)
  double acc_ms = 0;  // cumulative kernel time of recycled slots
  uint64_t acc_calls = 0;
  // Planning scratch kept across calls, so that a batch costs O(requests)
  // and, below kPlanReserve requests, allocates nothing.
  std::vector<int64_t> where;  // per instance: index in `touched` during a plan, -1 otherwise
  std::vector<uint32_t> touched;
  std::vector<uint64_t> cur_x, cur_k;
  std::vector<uint32_t> seg_count, seg_start;
  std::vector<uint8_t> seg_tab;  // per touched instance: width-64 tile starts from the table
  std::vector<uint64_t> req_x;
  std::vector<uint32_t> req_pos;
  std::vector<uint32_t> order;
  phprng_tuning tuning[3] = {{256, 4, 8, 4}, {256, 4, 8, 4}, {256, 4, 8, 4}};
  // allocation-free entry point: the device's fixed scratch and a pinned
  // staging block for its requests
  uint8_t *scratch = nullptr;
  uint8_t *h_noalloc = nullptr;
  hipEvent_t noalloc_copied = nullptr;
  bool noalloc_pending = false;
  std::string err;

  ~phprng_ctx() {
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    (void)hipFree(d_inst);
    (void)hipFree(d_lanemul);
    (void)hipFree(d_m64);
    (void)hipFree(d_u32);
    (void)hipFree(d_s32);
    (void)hipFree(d_u64lo);
    (void)hipFree(d_u64hi);
    (void)hipFree(d_s64);
    (void)hipFree(d_partial);
    if (chain_ev) (void)hipEventDestroy(chain_ev);
    if (noalloc_copied) (void)hipEventDestroy(noalloc_copied);
    if (h_noalloc) (void)hipHostFree(h_noalloc);
    for (auto &s : slots) {
      (void)hipFree(s.d_blk);
      if (s.h_blk) (void)hipHostFree(s.h_blk);
      (void)hipFree(s.d_ctr);
      (void)hipFree(s.d_t64);
      if (s.ev0) (void)hipEventDestroy(s.ev0);
      if (s.ev1) (void)hipEventDestroy(s.ev1);
    }
  }

  phprng_status fail(phprng_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return st;
  }
  phprng_status hip_fail(hipError_t e, const char *what) {
    return fail(PHPRNG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }

  // U(r) = sum_{j=1}^{r} (a^j mod p) and a^r mod p (width 32), from the table
  // entry at or below r plus at most stride-1 host steps.
  void prefix32(uint64_t r, u128 *U, uint64_t *S) const {
    const SkipGroup &G = group(32);
    const uint64_t i = r / kTableStride;
    u128 u = (u128)u32[i];
    uint64_t s = (uint64_t)s32[i];
    for (uint64_t x = i * kTableStride; x < r; ++x) {
      s = G.mulmod(G.a, s);
      u += s;
    }
    *U = u;
    *S = s;
  }

  // State (m, s) at internal index x of a width-32 pseudorandom-skip or a
  // constant-skip instance (eq. (7); constant skip: m = m_0 + x b, s = b).
  void state_at(const HostInst &h, uint64_t x, uint64_t *m, uint64_t *s) const {
    Mont64 M(h.n);
    if (h.sched == kSchedConstant) {
      *m = M.add(h.mbase % h.n, M.mulmod(x % h.n, h.b));
      *s = h.b;
      return;
    }
    const SkipGroup &G = group(32);
    const uint64_t pm1 = G.p - 1;
    const uint64_t q = x / pm1, r = x % pm1;
    u128 U;
    prefix32(r, &U, s);
    const u128 full = ((u128)G.p * (G.p - 1)) / 2;
    uint64_t b = M.reduce128(full);
    uint64_t qb = M.mulmod(q % h.n, b);
    *m = M.add(M.add(h.mbase % h.n, M.reduce128(U)), qb);
  }

  InstRec make_record(const HostInst &h) const {
    InstRec rec;
    memset(&rec, 0, sizeof rec);
    rec.n = h.n;
    rec.e = h.e;
    rec.width = (uint32_t)h.width;
    rec.ebits = (uint32_t)bit_length(h.e);
    rec.ekind = (h.e == 3 || h.e == 5 || h.e == 9 || h.e == 17) ? (uint32_t)h.e : 0u;
    Mont64 M(h.n);
    const SkipGroup &G = group(h.width);
    const u128 full = ((u128)G.p * (G.p - 1)) / 2;
    const uint64_t b = M.reduce128(full);
    rec.mbase = h.mbase;
    rec.sched = h.sched;
    if (h.sched == kSchedConstant) {
      const uint64_t R = h.width == 32 ? (1ull << 32) % h.n : M.r1;
      const uint64_t R2 = M.mulmod(R, R);
      rec.bskip = h.b;
      rec.bR2 = M.mulmod(h.b, R2);
      rec.b64 = M.mulmod(64 % h.n, h.b);
    }
    if (h.width == 32) {
      const uint32_t n32 = (uint32_t)h.n;
      uint32_t inv = n32;
      for (int i = 0; i < 5; ++i) inv *= 2u - n32 * inv;
      rec.ninv = inv;
      const uint64_t R = (1ull << 32) % h.n;
      const uint64_t R2 = M.mulmod(R, R);
      rec.r2 = R2;
      rec.kcorr = M.powmod(R, h.e);
      rec.br2 = M.mulmod(b, R2);
      rec.den = (double)(h.n + 1);
      rec.rcp = 1.0 / (double)(h.n + 1);
    } else {
      rec.ninv = M.ninv;
      rec.r2 = M.r2;
      rec.kcorr = M.powmod(M.r1, h.e);
      rec.br2 = 0;
      rec.den = (double)(h.n + 1);
      rec.rcp = 1.0 / rec.den;
    }
    return rec;
  }

  // Wait for a slot's work and add its kernel time to the running total.
  hipError_t retire(Slot &s) {
    hipError_t e = hipEventSynchronize(s.ev1);
    if (e != hipSuccess) return e;
    float f = 0;
    if (s.timed && hipEventElapsedTime(&f, s.ev0, s.ev1) == hipSuccess) {
      acc_ms += f;
      acc_calls += 1;
    }
    s.busy = false;
    return hipSuccess;
  }

  // Take the next staging slot with room for nreq requests; waits for the
  // slot's previous work to finish.
  phprng_status take_slot(uint64_t nreq, Slot **out) {
    cur_slot = (cur_slot + 1) % kSlots;
    Slot &s = slots[cur_slot];
    if (s.busy) {
      hipError_t e = retire(s);
      if (e != hipSuccess) return hip_fail(e, "slot wait");
    }
    phprng_status st = prepare_slot(s, nreq);
    if (st != PHPRNG_OK) return st;
    *out = &s;
    return PHPRNG_OK;
  }

  // Creates a slot's events and work counter on its first use and sizes its
  // request buffers for nreq requests.  Context creation does this for every
  // slot, so that calls pay only for growth beyond typical batches.
  phprng_status prepare_slot(Slot &s, uint64_t nreq) {
    hipError_t e;
    if (!s.ev0) {
      if ((e = hipEventCreate(&s.ev0)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventCreate(&s.ev1)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipMalloc(&s.d_ctr, sizeof(WorkCtr))) != hipSuccess) return fail(PHPRNG_E_NOMEM, "work counter");
      // the generation kernel expects a zero counter and leaves it so
      if ((e = hipMemset(s.d_ctr, 0, sizeof(WorkCtr))) != hipSuccess) return hip_fail(e, "work counter");
    }
    if (nreq > s.cap) {
      // room for typical batches from the start: growing frees buffers,
      // which waits for the device
      uint64_t cap = std::max<uint64_t>({nreq, 2 * s.cap, kMinSlotRequests});
      if (s.d_blk) (void)hipFree(s.d_blk);
      if (s.h_blk) (void)hipHostFree(s.h_blk);
      s.d_blk = nullptr;
      s.h_blk = nullptr;
      s.h_blk_dev = nullptr;
      s.cap = 0;
      const uint64_t bytes = sizeof(BatchHdr) + cap * sizeof(ReqRec);
      if ((e = hipMalloc(&s.d_blk, bytes)) != hipSuccess)
        return fail(PHPRNG_E_NOMEM, "request buffer: %s", hipGetErrorString(e));
      // coherent: kernels may read the planned requests straight from it
      if ((e = hipHostMalloc(&s.h_blk, bytes, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess) {
        s.h_blk = nullptr;
        return fail(PHPRNG_E_NOMEM, "pinned request buffer: %s", hipGetErrorString(e));
      }
      void *dp = nullptr;
      if ((e = hipHostGetDevicePointer(&dp, s.h_blk, 0)) != hipSuccess || !dp)
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidValue, "pinned request buffer address");
      s.h_blk_dev = static_cast<const uint8_t *>(dp);
      s.cap = cap;
    }
    return PHPRNG_OK;
  }

  phprng_status ensure_tiles(Slot &s, uint64_t tiles64) {
    if (tiles64 <= s.cap64) return PHPRNG_OK;
    const uint64_t cap = std::max<uint64_t>({tiles64, 2 * s.cap64, 1ull << 16});
    if (s.d_t64) (void)hipFree(s.d_t64);
    s.d_t64 = nullptr;
    s.cap64 = 0;
    hipError_t e = hipMalloc(&s.d_t64, 3 * cap * sizeof(uint64_t));
    if (e != hipSuccess) return fail(PHPRNG_E_NOMEM, "tile state: %s", hipGetErrorString(e));
    s.cap64 = cap;
    return PHPRNG_OK;
  }

  phprng_status build_table32();
  phprng_status build_table64();
  phprng_status plan(const phprng_request *reqs, uint64_t nreq, uint64_t capacity, int mode, const uint32_t *tpc_fix,
                     uint64_t stage_cap, uint8_t *stage, Plan *P);
  void commit_plan();
  GenArgs args(const uint8_t *d_blk, WorkCtr *ctr, uint64_t *t64, uint64_t t64cap, uint64_t nreq, uint32_t *c32,
               uint64_t *c64, double *r, uint32_t tpc) const;
  phprng_status launch(const Plan &P, const GenArgs &A, const ReqRec *hreq, hipStream_t s, int mode);
  phprng_status sync_chain();
  phprng_status read_m64(uint32_t id, uint64_t *m);
  phprng_status write_m64(uint32_t id, uint64_t m);
  phprng_status move64(uint32_t id, uint64_t d, bool forward, bool dry_run);
};

phprng_status phprng_ctx::build_table32() {
  const uint64_t pm1 = (uint64_t)kP32 - 1;
  const uint64_t ne = (pm1 - 1) / kTableStride + 1;  // entries at 0, stride, ... <= p - 2
  uint64_t *d_sum = nullptr;
  uint32_t *d_start = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&d_sum, ne * sizeof(uint64_t))) != hipSuccess) return fail(PHPRNG_E_NOMEM, "table32 alloc");
  if ((e = hipMalloc(&d_start, ne * sizeof(uint32_t))) != hipSuccess) {
    (void)hipFree(d_sum);
    return fail(PHPRNG_E_NOMEM, "table32 alloc");
  }
  if ((e = launch_table_segments32(ne, d_sum, d_start, nullptr)) != hipSuccess) return hip_fail(e, "table32 launch");
  std::vector<uint64_t> sums(ne);
  s32.resize(ne);
  if ((e = hipMemcpy(sums.data(), d_sum, ne * sizeof(uint64_t), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "table32 copy");
  if ((e = hipMemcpy(s32.data(), d_start, ne * sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "table32 copy");
  (void)hipFree(d_sum);
  u32.resize(ne);
  uint64_t acc = 0;
  for (uint64_t i = 0; i < ne; ++i) {
    u32[i] = acc;
    acc += sums[i];
  }
  // Self-check: the full-period skip sum is p(p-1)/2 and the skip returns to 1.
  u128 U;
  uint64_t S;
  prefix32(pm1, &U, &S);
  if (U != ((u128)kP32 * pm1) / 2 || S != 1) {
    (void)hipFree(d_start);
    return fail(PHPRNG_E_DEVICE, "32-bit skip-prefix table failed its full-period check");
  }
  d_s32 = d_start;
  if ((e = hipMalloc(&d_u32, ne * sizeof(uint64_t))) != hipSuccess) return fail(PHPRNG_E_NOMEM, "table32 alloc");
  if ((e = hipMemcpy(d_u32, u32.data(), ne * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "table32 upload");
  return PHPRNG_OK;
}

phprng_status phprng_ctx::build_table64() {
  if (have64) return PHPRNG_OK;
  const uint64_t ne = kTab64Range / kTab64Stride;
  uint64_t *d_lo = nullptr, *d_hi = nullptr, *d_start = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&d_lo, ne * 8)) != hipSuccess) return fail(PHPRNG_E_NOMEM, "table64 alloc");
  if ((e = hipMalloc(&d_hi, ne * 8)) != hipSuccess) {
    (void)hipFree(d_lo);
    return fail(PHPRNG_E_NOMEM, "table64 alloc");
  }
  if ((e = hipMalloc(&d_start, ne * 8)) != hipSuccess) {
    (void)hipFree(d_lo);
    (void)hipFree(d_hi);
    return fail(PHPRNG_E_NOMEM, "table64 alloc");
  }
  auto give_up = [&](phprng_status st) {
    (void)hipFree(d_lo);
    (void)hipFree(d_hi);
    (void)hipFree(d_start);
    return st;
  };
  if ((e = launch_table_segments64(ne, d_lo, d_hi, d_start, nullptr)) != hipSuccess)
    return give_up(hip_fail(e, "table64 launch"));
  std::vector<uint64_t> lo(ne), hi(ne), s64(ne);
  if ((e = hipMemcpy(lo.data(), d_lo, ne * 8, hipMemcpyDeviceToHost)) != hipSuccess) return give_up(hip_fail(e, "copy"));
  if ((e = hipMemcpy(hi.data(), d_hi, ne * 8, hipMemcpyDeviceToHost)) != hipSuccess) return give_up(hip_fail(e, "copy"));
  if ((e = hipMemcpy(s64.data(), d_start, ne * 8, hipMemcpyDeviceToHost)) != hipSuccess)
    return give_up(hip_fail(e, "copy"));
  std::vector<u128> u(ne);
  u128 acc = 0;
  for (uint64_t i = 0; i < ne; ++i) {
    u[i] = acc;
    acc += ((u128)hi[i] << 64) | lo[i];
    lo[i] = (uint64_t)u[i];
    hi[i] = (uint64_t)(u[i] >> 64);
  }
  // Spot-check a few entries against host stepping from the previous entry.
  const SkipGroup &G = group(64);
  for (uint64_t i : {(uint64_t)1, ne / 3, ne - 1}) {
    u128 v = u[i - 1];
    uint64_t s = s64[i - 1];
    for (uint64_t x = 0; x < kTab64Stride; ++x) {
      s = G.mulmod(G.a, s);
      v += s;
    }
    if (v != u[i] || s != s64[i] || s != G.powmod(G.a, i * kTab64Stride))
      return give_up(fail(PHPRNG_E_DEVICE, "64-bit skip-prefix table failed its check at entry %llu",
                          (unsigned long long)i));
  }
  if ((e = hipMemcpy(d_lo, lo.data(), ne * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return give_up(hip_fail(e, "upload"));
  if ((e = hipMemcpy(d_hi, hi.data(), ne * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return give_up(hip_fail(e, "upload"));
  d_u64lo = d_lo;
  d_u64hi = d_hi;
  d_s64 = d_start;
  have64 = true;
  return PHPRNG_OK;
}

// Global tile index of the width-32 tile whose draws include the draw made
// from internal index x.
static inline uint64_t tile_of32(uint64_t x) {
  const uint64_t pm1 = (uint64_t)kP32 - 1;
  const uint64_t q = x / pm1, r = x - q * pm1;
  return (q << 20) | (r / kTile32);
}

// Validate a request list, reserve positions (in request order) and write
// the planned batch into `stage` (BatchHdr followed by nreq ReqRec): the
// width-64 pseudorandom-skip requests first, grouped by instance in call
// order, then the other width-64 requests, then the width-32 ones.  The new
// positions are kept in cur_x / cur_k for commit_plan once every launch has
// been issued.  tpc_fix: tiles per chunk to use as is (graphs), else the
// tuned value, halved for batches too small to give every wave 4 chunks.
phprng_status phprng_ctx::plan(const phprng_request *reqs, uint64_t nreq, uint64_t capacity, int mode,
                               const uint32_t *tpc_fix, uint64_t stage_cap, uint8_t *stage, Plan *P) {
  if (nreq > 0 && !reqs) return fail(PHPRNG_E_INVALID, "null request array");
  if (nreq > stage_cap) return fail(PHPRNG_E_RANGE, "too many requests for the staging buffer");
  if (nreq >= (1ull << 31)) return fail(PHPRNG_E_RANGE, "too many requests");
  const uint64_t pm1_64 = kP64 - 1;
  for (uint64_t i = 0; i < nreq; ++i) {
    const phprng_request &r = reqs[i];
    if (r.instance >= inst.size() || r.reserved != 0)
      return fail(PHPRNG_E_INVALID, "request %llu: bad instance", (unsigned long long)i);
    if (r.count > capacity || r.out_offset > capacity - r.count)
      return fail(PHPRNG_E_RANGE, "request %llu: output range beyond capacity", (unsigned long long)i);
  }
  if (where.size() < inst.size()) where.resize(inst.size(), -1);
  touched.clear();
  cur_x.clear();
  cur_k.clear();
  seg_count.clear();
  req_x.resize(nreq);
  req_pos.resize(nreq);
  struct Reset {  // `where` back to -1 on every way out
    std::vector<int64_t> &w;
    const std::vector<uint32_t> &t;
    ~Reset() {
      for (uint32_t i : t) w[i] = -1;
    }
  } reset{where, touched};
  // positions in request order
  uint64_t c64l = 0, c64c = 0, c32 = 0;
  for (uint64_t i = 0; i < nreq; ++i) {
    const phprng_request &r = reqs[i];
    const HostInst &h = inst[r.instance];
    if (where[r.instance] < 0) {
      where[r.instance] = (int64_t)touched.size();
      touched.push_back(r.instance);
      cur_x.push_back(h.x);
      cur_k.push_back(h.k);
      seg_count.push_back(0);
    }
    const size_t t = (size_t)where[r.instance];
    if (r.count > ~0ull - cur_k[t])
      return fail(PHPRNG_E_RANGE, "request %llu: position beyond range", (unsigned long long)i);
    req_x[i] = cur_x[t];
    if (lcg64(h)) {
      if (r.count >= kMaxCount64)
        return fail(PHPRNG_E_RANGE, "request %llu: more than 2^42 width-64 draws", (unsigned long long)i);
      cur_x[t] = add_u64_mod(cur_x[t], r.count % pm1_64, pm1_64);
      seg_count[t] += 1;
      ++c64l;
    } else {
      if (r.count > ~0ull - cur_x[t])
        return fail(PHPRNG_E_RANGE, "request %llu: position beyond range", (unsigned long long)i);
      cur_x[t] += r.count;
      if (h.width == 64) ++c64c;
      else ++c32;
    }
    cur_k[t] += r.count;
  }
  // staging order
  seg_start.resize(touched.size());
  uint32_t run = 0;
  for (size_t t = 0; t < touched.size(); ++t) {
    seg_start[t] = run;
    if (lcg64(inst[touched[t]])) run += seg_count[t];
  }
  {
    uint64_t f64c = c64l, f32 = c64l + c64c;
    // seg_count doubles as the fill count of each instance's group
    std::vector<uint32_t> &fill = seg_count;
    for (size_t t = 0; t < touched.size(); ++t) fill[t] = 0;
    for (uint64_t i = 0; i < nreq; ++i) {
      const HostInst &h = inst[reqs[i].instance];
      const size_t t = (size_t)where[reqs[i].instance];
      if (lcg64(h)) req_pos[i] = seg_start[t] + fill[t]++;
      else if (h.width == 64) req_pos[i] = (uint32_t)f64c++;
      else req_pos[i] = (uint32_t)f32++;
    }
  }
  order.resize(nreq);
  for (uint64_t i = 0; i < nreq; ++i) order[req_pos[i]] = (uint32_t)i;
  // records
  BatchHdr *H = reinterpret_cast<BatchHdr *>(stage);
  ReqRec *R = reinterpret_cast<ReqRec *>(stage + sizeof(BatchHdr));
  // A width-64 instance's tile starts come from the table when all of its
  // draws in the batch lie below the table's range (its tiles then start at
  // table entries), else from the reduce and scan of its requests' skips.
  seg_tab.assign(touched.size(), (uint8_t)have64);
  for (uint64_t i = 0; i < nreq; ++i)
    if (lcg64(inst[reqs[i].instance]) && req_x[i] + reqs[i].count >= kTab64Range)
      seg_tab[(size_t)where[reqs[i].instance]] = 0;
  bool any_tab = false, any_reduce = false;
  uint64_t tiles = 0, tiles64 = 0, units64 = 0;
  for (uint64_t p = 0; p < nreq; ++p) {
    const uint64_t i = order[p];
    const phprng_request &q = reqs[i];
    const HostInst &h = inst[q.instance];
    ReqRec &rr = R[p];
    memset(&rr, 0, sizeof rr);
    rr.x = req_x[i];
    rr.count = q.count;
    rr.out_off = q.out_offset;
    rr.inst = q.instance;
    uint64_t nt = 0;
    if (lcg64(h)) {
      const size_t t = (size_t)where[q.instance];
      const bool tab = seg_tab[t] != 0;
      if (tab)
        nt = q.count ? (rr.x + q.count - 1) / kTab64Stride - rr.x / kTab64Stride + 1 : 0;
      else
        nt = (q.count + kTile64 - 1) / kTile64;
      rr.g1 = tiles64;
      tiles64 += nt;
      rr.seg = (p == seg_start[t] ? seg_count[t] : 0) | (tab ? kSegTable : 0u);
      any_tab = any_tab || tab;
      any_reduce = any_reduce || !tab;
    } else if (h.sched == kSchedConstant) {
      rr.g1 = rr.x / kTileCS;
      nt = q.count ? (rr.x + q.count - 1) / kTileCS - rr.g1 + 1 : 0;
    } else {
      rr.g1 = tile_of32(rr.x);
      nt = q.count ? tile_of32(rr.x + q.count - 1) - rr.g1 + 1 : 0;
    }
    if (nt >= (1ull << 32)) return fail(PHPRNG_E_RANGE, "request %llu: too many tiles", (unsigned long long)i);
    rr.ntiles = (uint32_t)nt;
    tiles += nt;
  }
  // chunks
  Plan out;
  out.nreq = nreq;
  out.nreq64 = c64l;
  // width-64 reduce units: up to kReduceTiles tiles each, fewer when the
  // batch would leave most of the reduce grid idle
  uint64_t tiles_reduce = 0;
  for (uint64_t p = 0; p < c64l; ++p)
    if (!(R[p].seg & kSegTable)) tiles_reduce += R[p].ntiles;
  uint32_t rt = kReduceTiles;
  while (rt > 1 && tiles_reduce < (uint64_t)rt * kReduceWaves) rt >>= 1;
  for (uint64_t p = 0; p < c64l; ++p) {
    // requests with table tile starts take no unit (the reduce's search
    // passes over them: they share the next request's first unit)
    R[p].rbase = units64;
    if (!(R[p].seg & kSegTable)) units64 += ((uint64_t)R[p].ntiles + rt - 1) / rt;
  }
  out.tiles64 = tiles64;
  out.units64 = units64;
  out.reduce_tiles = rt;
  out.any_tab = any_tab;
  out.any_reduce = any_reduce;
  out.tiles = tiles;
  out.has64 = c64l + c64c > 0;
  out.has32 = c32 > 0;
  out.cls = out.has64 ? (out.has32 ? kMixBoth : kMix64) : kMix32;
  const phprng_tuning &T = tuning[out.cls];
  uint32_t tpc;
  if (mode == PHPRNG_MODE_PLAIN) {
    tpc = 1;
  } else if (tpc_fix) {
    tpc = *tpc_fix;
  } else {
    tpc = (uint32_t)T.tiles_per_chunk;
    const uint64_t waves = (uint64_t)num_cus * T.blocks_per_cu * (T.block_threads / 64);
    while (tpc > 1 && tiles < 4 * waves * tpc) tpc >>= 1;
  }
  out.tpc = tpc;
  uint64_t chunks = 0;
  for (uint64_t p = 0; p < nreq; ++p) {
    ReqRec &rr = R[p];
    const uint64_t nc = ((uint64_t)rr.ntiles + tpc - 1) / tpc;
    rr.chunk_base = chunks;
    rr.nchunks = (uint32_t)nc;
    chunks += nc;
  }
  // the work counter hands out chunk numbers in 32 bits
  if (chunks >= (1ull << 31)) return fail(PHPRNG_E_RANGE, "batch too large: %llu chunks", (unsigned long long)chunks);
  out.total_chunks = chunks;
  memset(H, 0, sizeof *H);
  H->total_chunks = chunks;
  H->nreq = nreq;
  H->nreq64 = c64l;
  H->tiles64 = tiles64;
  H->units64 = units64;
  H->reduce_tiles = rt;
  *P = out;
  return PHPRNG_OK;
}

void phprng_ctx::commit_plan() {
  for (size_t t = 0; t < touched.size(); ++t) {
    HostInst &h = inst[touched[t]];
    h.x = cur_x[t];
    h.k = cur_k[t];
  }
}

GenArgs phprng_ctx::args(const uint8_t *d_blk, WorkCtr *ctr, uint64_t *t64, uint64_t t64cap, uint64_t nreq,
                         uint32_t *c32, uint64_t *c64, double *r, uint32_t tpc) const {
  GenArgs A;
  memset(&A, 0, sizeof A);
  A.inst = d_inst;
  A.hdr = reinterpret_cast<const BatchHdr *>(d_blk);
  A.req = reinterpret_cast<const ReqRec *>(d_blk + sizeof(BatchHdr));
  A.nreq = nreq;
  A.ctr = ctr;
  A.tab = SkipTables{d_u32, d_s32, (uint64_t)u32.size(), d_u64lo, d_u64hi, d_s64};
  A.lanemul = d_lanemul;
  A.t64.s = t64;
  A.t64.sum = t64 ? t64 + t64cap : nullptr;
  A.t64.m = t64 ? t64 + 2 * t64cap : nullptr;
  A.m64 = d_m64;
  A.out_c32 = c32;
  A.out_c64 = c64;
  A.out_r = r;
  A.tiles_per_chunk = tpc;
  return A;
}

// Width-64 tile starts (ordered after the previous call's scan), then the
// generation kernel(s).  The batch block must already be on the device.
phprng_status phprng_ctx::launch(const Plan &P, const GenArgs &A, const ReqRec *hreq, hipStream_t s, int mode) {
  hipError_t e;
  if (P.nreq64 > 0) {
    if (P.any_reduce && (e = launch_tiles64_reduce(A, P.units64, (unsigned)num_cus * 8, s)) != hipSuccess)
      return hip_fail(e, "tile reduce");
    if (chain_pending && (e = hipStreamWaitEvent(s, chain_ev, 0)) != hipSuccess) return hip_fail(e, "chain wait");
    if (P.any_tab && (e = launch_tiles64_table(A, P.nreq64, s)) != hipSuccess) return hip_fail(e, "table tile starts");
    if (P.any_reduce && (e = launch_tiles64_scan(A, P.nreq64, s)) != hipSuccess) return hip_fail(e, "tile scan");
    if ((e = hipEventRecord(chain_ev, s)) != hipSuccess) return hip_fail(e, "chain record");
    chain_pending = true;
  }
  const phprng_tuning &T = tuning[P.cls];
  if (mode == PHPRNG_MODE_PERSISTENT) {
    if (P.total_chunks == 0) return PHPRNG_OK;
    // A batch with fewer chunks than the tuned grid has waves runs one wave
    // per chunk in one-wave blocks, so that its waves spread over every
    // compute unit instead of filling a few with whole blocks.
    const uint64_t wpb = (uint64_t)T.block_threads / 64;
    const uint64_t full = (uint64_t)num_cus * T.blocks_per_cu * wpb;
    const int block = P.total_chunks < full ? 64 : T.block_threads;
    const unsigned grid = (unsigned)(P.total_chunks < full ? P.total_chunks : (uint64_t)num_cus * T.blocks_per_cu);
    if ((e = launch_persistent(A, grid, block, T.unroll, P.has64, s)) != hipSuccess)
      return hip_fail(e, "persistent launch");
  } else {
    // one grid per request, from the host copy of the planned requests
    for (uint64_t p = 0; p < P.nreq; ++p) {
      if ((e = launch_plain(A, p, hreq[p].nchunks, T.unroll, P.has64, s)) != hipSuccess)
        return hip_fail(e, "plain launch");
    }
  }
  return PHPRNG_OK;
}

phprng_status phprng_ctx::sync_chain() {
  if (!chain_pending) return PHPRNG_OK;
  hipError_t e = hipEventSynchronize(chain_ev);
  if (e != hipSuccess) return hip_fail(e, "chain wait");
  chain_pending = false;
  return PHPRNG_OK;
}

phprng_status phprng_ctx::read_m64(uint32_t id, uint64_t *m) {
  phprng_status st = sync_chain();
  if (st != PHPRNG_OK) return st;
  hipError_t e = hipMemcpy(m, d_m64 + id, sizeof(uint64_t), hipMemcpyDeviceToHost);
  return e == hipSuccess ? PHPRNG_OK : hip_fail(e, "message read");
}

phprng_status phprng_ctx::write_m64(uint32_t id, uint64_t m) {
  phprng_status st = sync_chain();
  if (st != PHPRNG_OK) return st;
  hipError_t e = hipMemcpy(d_m64 + id, &m, sizeof(uint64_t), hipMemcpyHostToDevice);
  return e == hipSuccess ? PHPRNG_OK : hip_fail(e, "message write");
}

namespace {

// Runs position64_kernel on host arrays (one entry per instance) and waits.
phprng_status apply_table64(phprng_ctx *c, const std::vector<uint32_t> &ids, const std::vector<uint64_t> &m0,
                            const std::vector<uint64_t> &ta, const std::vector<uint64_t> &tb) {
  const uint64_t n = ids.size();
  if (n == 0) return PHPRNG_OK;
  uint8_t *d = nullptr;
  const uint64_t bytes = n * (4 + 3 * 8) + 64;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return c->fail(PHPRNG_E_NOMEM, "positioning buffer");
  uint64_t *dm = reinterpret_cast<uint64_t *>(d), *da = dm + n, *db = da + n;
  uint32_t *di = reinterpret_cast<uint32_t *>(db + n);
  if (e == hipSuccess) e = hipMemcpy(dm, m0.data(), n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(da, ta.data(), n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db, tb.data(), n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(di, ids.data(), n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_position64(c->d_inst, di, dm, da, db, n, c->d_u64lo, c->d_u64hi, c->d_s64, c->d_m64, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  (void)hipFree(d);
  return e == hipSuccess ? PHPRNG_OK : c->hip_fail(e, "positioning");
}

}  // namespace

// Moves the device message of width-64 instance `id` by d draws from skip
// log h.x (forward or backward) and reports the new skip log.  d = q (p - 1)
// + r: each whole skip period adds p(p-1)/2 (Sec. II), and the r remaining
// skips come from the positioning table when both ends lie on it, else are
// summed on the device (or, when r is within kJumpMax of a whole period,
// the complement is).  dry_run only checks that the move is supported.
phprng_status phprng_ctx::move64(uint32_t id, uint64_t d, bool forward, bool dry_run) {
  const HostInst &h = inst[id];
  const uint64_t pm1 = kP64 - 1, x = h.x;
  const uint64_t q = d / pm1, r = d % pm1;
  enum { kTable, kSum, kComplement } path;
  if (forward ? (x + r < kTab64Range) : (x >= r && x < kTab64Range)) path = kTable;
  else if (r <= kJumpMax) path = kSum;
  else if (pm1 - r <= kJumpMax) path = kComplement;
  else return fail(PHPRNG_E_RANGE, "width-64 move of %llu draws: off the table and too far from a whole skip period",
                   (unsigned long long)d);
  if (dry_run || d == 0) return PHPRNG_OK;
  if (path == kTable && !have64) {
    phprng_status bs = build_table64();
    if (bs != PHPRNG_OK) return bs;
  }
  Mont64 M(h.n);
  const uint64_t b = M.reduce128(((u128)kP64 * pm1) / 2);
  const uint64_t qb = M.mulmod(q % h.n, b);
  phprng_status st;
  if (path == kTable) {
    uint64_t m = 0;
    if ((st = read_m64(id, &m)) != PHPRNG_OK) return st;
    m = forward ? M.add(m, qb) : M.sub(m, qb);
    std::vector<uint32_t> ids{id};
    std::vector<uint64_t> m0{m}, ta{forward ? x + r : x - r}, tb{x};
    st = apply_table64(this, ids, m0, ta, tb);
  } else {
    if ((st = sync_chain()) != PHPRNG_OK) return st;
    uint64_t t, cnt, extra;
    int sign;
    if (path == kSum) {
      // forward: + (q b + skips of logs x+1 .. x+r); backward: - (q b + logs x-r+1 .. x)
      t = forward ? x : (x >= r ? x - r : x + (pm1 - r));
      cnt = r;
      extra = qb;
      sign = forward ? 1 : -1;
    } else {
      // the r skips are a whole period less the pm1 - r skips that complete it
      const uint64_t e1 = M.mulmod((q + 1) % h.n, b);
      t = forward ? add_u64_mod(x, r, pm1) : x;
      cnt = pm1 - r;
      extra = e1 ? h.n - e1 : 0;
      sign = forward ? -1 : 1;
    }
    hipError_t e = launch_skip_total64(t, cnt, h.n, d_lanemul, d_partial, kJumpBlocks, extra, sign, d_m64 + id, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    st = e == hipSuccess ? PHPRNG_OK : hip_fail(e, "skip sum");
  }
  return st;
}

// ---------------------------------------------------------------------------
// host-only helpers
// ---------------------------------------------------------------------------

extern "C" const char *phprng_status_string(phprng_status st) {
  switch (st) {
    case PHPRNG_OK: return "ok";
    case PHPRNG_E_INVALID: return "invalid argument";
    case PHPRNG_E_NOT_PRIME: return "modulus is not prime";
    case PHPRNG_E_EXPONENT: return "exponent not admissible";
    case PHPRNG_E_RANGE: return "value out of range";
    case PHPRNG_E_NOMEM: return "out of memory";
    case PHPRNG_E_DEVICE: return "device error";
  }
  return "unknown status";
}

extern "C" phprng_status phprng_skip_params(int width, uint64_t *p, uint64_t *a) {
  if (!width_ok(width) || !p || !a) return PHPRNG_E_INVALID;
  *p = width == 32 ? kP32 : kP64;
  *a = width == 32 ? kA32 : kA64;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_check_instance(int width, uint64_t n, uint64_t e) {
  return check_instance_impl(width, n, e);
}

extern "C" phprng_status phprng_draw_instances(int width, uint64_t seed, uint64_t count, const uint64_t *e_set,
                                               int e_len, uint64_t k_lo, uint64_t k_hi, uint64_t *n_out,
                                               uint64_t *e_out, uint64_t *k_out) {
  if (!width_ok(width) || !e_set || e_len <= 0 || k_hi < k_lo) return PHPRNG_E_INVALID;
  if (count > 0 && (!n_out || !e_out || !k_out)) return PHPRNG_E_INVALID;
  bool any = false;
  for (int i = 0; i < e_len; ++i) any = any || e_set[i] >= 3;
  if (!any) return PHPRNG_E_EXPONENT;
  const uint64_t lo = width == 32 ? (1ull << 31) : (1ull << 62);
  const uint64_t span = lo;  // ranges [2^31, 2^32) and [2^62, 2^63)
  if (width == 32 && count > 40000000ull) return PHPRNG_E_RANGE;
  std::unordered_set<uint64_t> seen;
  seen.reserve(count * 2 + 16);
  uint64_t st = seed;
  for (uint64_t i = 0; i < count; ++i) {
    for (;;) {
      const uint64_t x = splitmix64(st);
      const uint64_t n = (lo + x % span) | 1ull;
      if (!is_prime64(n) || seen.count(n)) continue;
      const uint64_t y = splitmix64(st);
      uint64_t chosen = 0;
      for (int t = 0; t < e_len; ++t) {
        const uint64_t cand = e_set[(y % (uint64_t)e_len + (uint64_t)t) % (uint64_t)e_len];
        if (check_instance_impl(width, n, cand) == PHPRNG_OK) {
          chosen = cand;
          break;
        }
      }
      if (chosen == 0) continue;
      seen.insert(n);
      n_out[i] = n;
      e_out[i] = chosen;
      break;
    }
    k_out[i] = k_hi > k_lo ? k_lo + splitmix64(st) % (k_hi - k_lo) : k_lo;
  }
  return PHPRNG_OK;
}

// ---------------------------------------------------------------------------
// contexts
// ---------------------------------------------------------------------------

extern "C" phprng_status phprng_create(phprng_ctx **out, int device, uint64_t max_instances) {
  if (!out || max_instances == 0 || max_instances > (1ull << 31)) return PHPRNG_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PHPRNG_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return PHPRNG_E_DEVICE;
  std::unique_ptr<phprng_ctx> c(new (std::nothrow) phprng_ctx);
  if (!c) return PHPRNG_E_NOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PHPRNG_E_DEVICE;
  c->num_cus = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  c->max_instances = max_instances;
  try {
    for (auto *v : {&c->touched, &c->seg_count, &c->seg_start, &c->req_pos, &c->order})
      v->reserve(kPlanReserve);
    c->seg_tab.reserve(kPlanReserve);
    for (auto *v : {&c->cur_x, &c->cur_k, &c->req_x}) v->reserve(kPlanReserve);
  } catch (...) {
    return PHPRNG_E_NOMEM;
  }
  if (hipMalloc(&c->d_inst, max_instances * sizeof(InstRec)) != hipSuccess) return PHPRNG_E_NOMEM;
  if (hipMalloc(&c->d_m64, max_instances * sizeof(uint64_t)) != hipSuccess) return PHPRNG_E_NOMEM;
  if (hipMemset(c->d_m64, 0, max_instances * sizeof(uint64_t)) != hipSuccess) return PHPRNG_E_DEVICE;
  if (hipMalloc(&c->d_partial, (uint64_t)kJumpBlocks * 4 * sizeof(uint64_t)) != hipSuccess) return PHPRNG_E_NOMEM;
  // lane start multipliers a^{l * run} and the powers a^{2^b} of the 64-bit skip
  LaneMul lm;
  memset(&lm, 0, sizeof lm);
  const SkipGroup &g32 = group(32), &g64 = group(64);
  for (int l = 0; l < 64; ++l) {
    lm.m32[l] = (uint32_t)g32.powmod(g32.a, (uint64_t)l * kRun32);
    lm.m64[l] = g64.powmod(g64.a, (uint64_t)l * kRun64);
  }
  uint64_t pw = g64.a;
  for (int bexp = 0; bexp < 61; ++bexp) {
    lm.pow64[bexp] = pw;
    pw = g64.mulmod(pw, pw);
  }
  if (hipMalloc(&c->d_lanemul, sizeof(LaneMul)) != hipSuccess) return PHPRNG_E_NOMEM;
  if (hipMemcpy(c->d_lanemul, &lm, sizeof lm, hipMemcpyHostToDevice) != hipSuccess) return PHPRNG_E_DEVICE;
  if (hipEventCreateWithFlags(&c->chain_ev, hipEventDisableTiming) != hipSuccess) return PHPRNG_E_DEVICE;
  // the fixed scratch of the allocation-free entry point, looked up once per device
  void *sp = nullptr;
  if (scratch_address(device, &sp) != hipSuccess || !sp) return PHPRNG_E_DEVICE;
  c->scratch = static_cast<uint8_t *>(sp);
  if (hipHostMalloc(&c->h_noalloc, sizeof(BatchHdr) + kNoAllocMaxRequests * sizeof(ReqRec), hipHostMallocDefault) !=
      hipSuccess) {
    c->h_noalloc = nullptr;
    return PHPRNG_E_NOMEM;
  }
  if (hipEventCreateWithFlags(&c->noalloc_copied, hipEventDisableTiming) != hipSuccess) return PHPRNG_E_DEVICE;
  // every staging slot ready for typical batches (8192 requests, 2^16
  // width-64 tiles): the allocations of a first use would otherwise wait
  // for the device in the middle of a caller's stream of calls
  for (auto &slot : c->slots) {
    phprng_status st = c->prepare_slot(slot, phprng_ctx::kMinSlotRequests);
    if (st == PHPRNG_OK) st = c->ensure_tiles(slot, 1);
    if (st != PHPRNG_OK) return st;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int cls = 0; cls < 3; ++cls) {
      auto it = g_tune_cache.find(TuneKey{c->arch, c->num_cus, cls});
      if (it != g_tune_cache.end()) c->tuning[cls] = it->second;
    }
  }
  phprng_status st = c->build_table32();
  if (st != PHPRNG_OK) return st;
  *out = c.release();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_destroy(phprng_ctx *c) {
  if (!c) return PHPRNG_E_INVALID;
  delete c;
  return PHPRNG_OK;
}

extern "C" const char *phprng_last_error(const phprng_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" uint64_t phprng_instance_count(const phprng_ctx *c) { return c ? c->inst.size() : 0; }

extern "C" phprng_status phprng_add_instances(phprng_ctx *c, uint64_t count, int width, const uint64_t *n,
                                              const uint64_t *e, const uint64_t *m0, const uint64_t *s0,
                                              const uint64_t *k0, uint32_t *ids) {
  if (!c || !width_ok(width)) return PHPRNG_E_INVALID;
  if (count == 0) return PHPRNG_OK;
  if (!n || !e || !ids) return c->fail(PHPRNG_E_INVALID, "null array");
  if (c->inst.size() + count > c->max_instances) return c->fail(PHPRNG_E_RANGE, "instance table full");
  (void)hipSetDevice(c->device);
  const SkipGroup &G = group(width);
  const uint64_t pm1 = G.p - 1;
  std::vector<HostInst> add(count);
  std::vector<uint64_t> t0s(count, 0);
  std::vector<uint8_t> on_table(count, 0);
  // validate everything first
  for (uint64_t i = 0; i < count; ++i) {
    phprng_status st = check_instance_impl(width, n[i], e[i]);
    if (st != PHPRNG_OK) return c->fail(st, "instance %llu rejected", (unsigned long long)i);
    const uint64_t mm0 = m0 ? m0[i] : 0, ss0 = s0 ? s0[i] : 1, kk = k0 ? k0[i] : 0;
    if (mm0 >= n[i] || ss0 == 0 || ss0 >= G.p) return c->fail(PHPRNG_E_INVALID, "bad m0/s0 at %llu", (unsigned long long)i);
    const uint64_t t0 = ss0 == 1 ? 0 : G.dlog(ss0);
    t0s[i] = t0;
    HostInst h{n[i], e[i], width};
    h.k = kk;
    if (width == 32) {
      if (kk > ~0ull - t0) return c->fail(PHPRNG_E_RANGE, "start index overflows");
      h.x = t0 + kk;
    } else {
      h.x = t0;  // moved to kk below
      if (kk < kTab64Range && t0 + kk < kTab64Range) {
        on_table[i] = 1;
      } else {
        // off the table: the start is reached by summing skips on the device
        c->inst.push_back(h);
        phprng_status ms = c->move64((uint32_t)(c->inst.size() - 1), kk, true, true);
        c->inst.pop_back();
        if (ms != PHPRNG_OK) return ms;
      }
    }
    add[i] = h;
  }
  if (width == 64 && !c->have64) {
    phprng_status bs = c->build_table64();
    if (bs != PHPRNG_OK) return bs;
  }
  for (uint64_t i = 0; i < count; ++i) {
    if (width != 32) continue;
    // mbase such that the state at internal index t0 is (m0, s0): m0 - U(t0)
    const uint64_t mm0 = m0 ? m0[i] : 0;
    if (t0s[i] != 0 || mm0 != 0) {
      HostInst tmp = add[i];
      tmp.mbase = 0;
      uint64_t mu, su;
      c->state_at(tmp, t0s[i], &mu, &su);
      Mont64 M(n[i]);
      add[i].mbase = M.sub(mm0, mu);
    }
  }
  std::vector<InstRec> recs(count);
  for (uint64_t i = 0; i < count; ++i) recs[i] = c->make_record(add[i]);
  const uint64_t base = c->inst.size();
  hipError_t he = hipMemcpy(c->d_inst + base, recs.data(), count * sizeof(InstRec), hipMemcpyHostToDevice);
  if (he != hipSuccess) return c->hip_fail(he, "instance upload");
  for (uint64_t i = 0; i < count; ++i) {
    c->inst.push_back(add[i]);
    ids[i] = (uint32_t)(base + i);
  }
  if (c->where.size() < c->inst.size()) c->where.resize(c->inst.size(), -1);
  if (width == 64) {
    // messages at the start positions: from the table where it reaches,
    // else m0 moved forward on the device
    std::vector<uint32_t> tid;
    std::vector<uint64_t> tm, ta, tb;
    phprng_status st = PHPRNG_OK;
    for (uint64_t i = 0; i < count; ++i) {
      const uint64_t mm0 = m0 ? m0[i] : 0, kk = k0 ? k0[i] : 0;
      const uint32_t id = (uint32_t)(base + i);
      if (on_table[i]) {
        tid.push_back(id);
        tm.push_back(mm0);
        ta.push_back(t0s[i] + kk);
        tb.push_back(t0s[i]);
        c->inst[id].x = t0s[i] + kk;
      } else {
        if (st == PHPRNG_OK) st = c->write_m64(id, mm0);
        if (st == PHPRNG_OK) st = c->move64(id, kk, true, false);
        c->inst[id].x = add_u64_mod(t0s[i], kk % pm1, pm1);
      }
    }
    if (st == PHPRNG_OK) st = apply_table64(c, tid, tm, ta, tb);
    if (st != PHPRNG_OK) {
      c->inst.resize(base);  // nothing added
      return st;
    }
  }
  return PHPRNG_OK;
}

namespace {

bool exponent_ok(uint64_t n, uint64_t e) { return e >= 3 && gcd64(e, n - 1) == 1 && e % (n - 1) != 1; }

// The seeding draw of phprng_draw_instances with the primality of every
// stream output decided on the device (one deterministic Rabin-Miller per
// output, in batches); the walk over the stream stays on the host and
// consumes outputs in exactly the same order.
phprng_status draw_on_device(phprng_ctx *c, int width, uint64_t seed, uint64_t count, const uint64_t *e_set,
                             int e_len, uint64_t k_lo, uint64_t k_hi, uint64_t *n_out, uint64_t *e_out,
                             uint64_t *k_out) {
  const uint64_t lo = width == 32 ? (1ull << 31) : (1ull << 62);
  const uint64_t span = lo;
  std::vector<uint8_t> flags;
  uint8_t *d_flags = nullptr;
  uint64_t d_cap = 0;
  auto extend = [&](uint64_t want) -> phprng_status {
    const uint64_t j0 = flags.size();
    const uint64_t nb = std::max<uint64_t>(want, 1ull << 20);
    if (nb > d_cap) {
      if (d_flags) (void)hipFree(d_flags);
      d_flags = nullptr;
      hipError_t e = hipMalloc(&d_flags, nb);
      if (e != hipSuccess) return c->hip_fail(e, "seed flags");
      d_cap = nb;
    }
    hipError_t e = launch_seed_prime_flags(seed, j0, nb, width, d_flags, nullptr);
    if (e != hipSuccess) return c->hip_fail(e, "seed launch");
    flags.resize(j0 + nb);
    e = hipMemcpy(flags.data() + j0, d_flags, nb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return c->hip_fail(e, "seed copy");
    return PHPRNG_OK;
  };
  const uint64_t per = width == 32 ? 14 : 26;  // expected stream outputs per instance, with margin
  phprng_status st = extend(count * per + count / 4 + 1024);
  std::unordered_set<uint64_t> seen;
  seen.reserve(count * 2 + 16);
  uint64_t sm = seed, j = 0;
  for (uint64_t i = 0; i < count && st == PHPRNG_OK; ++i) {
    for (;;) {
      if (j + 3 > flags.size()) {
        st = extend(flags.size() / 4 + 1024);
        if (st != PHPRNG_OK) break;
      }
      const uint64_t x = splitmix64(sm);
      const bool prime = flags[j++] != 0;
      const uint64_t n = (lo + x % span) | 1ull;
      if (!prime || seen.count(n)) continue;
      const uint64_t y = splitmix64(sm);
      ++j;
      uint64_t chosen = 0;
      for (int t = 0; t < e_len; ++t) {
        const uint64_t cand = e_set[(y % (uint64_t)e_len + (uint64_t)t) % (uint64_t)e_len];
        if (exponent_ok(n, cand)) {
          chosen = cand;
          break;
        }
      }
      if (chosen == 0) continue;
      seen.insert(n);
      n_out[i] = n;
      e_out[i] = chosen;
      break;
    }
    if (k_hi > k_lo) {
      k_out[i] = k_lo + splitmix64(sm) % (k_hi - k_lo);
      ++j;
    } else {
      k_out[i] = k_lo;
    }
  }
  if (d_flags) (void)hipFree(d_flags);
  return st;
}

}  // namespace

extern "C" phprng_status phprng_seed_instances(phprng_ctx *c, uint64_t count, int width, uint64_t seed,
                                               const uint64_t *e_set, int e_len, uint64_t k_lo, uint64_t k_hi,
                                               uint32_t *ids) {
  if (!c) return PHPRNG_E_INVALID;
  if (count < 1024) {
    std::vector<uint64_t> n(count), e(count), k(count);
    phprng_status st =
        phprng_draw_instances(width, seed, count, e_set, e_len, k_lo, k_hi, n.data(), e.data(), k.data());
    if (st != PHPRNG_OK) return c->fail(st, "instance draw failed");
    return phprng_add_instances(c, count, width, n.data(), e.data(), nullptr, nullptr, k.data(), ids);
  }
  // Large draws: primality on the device, records built on the device.
  if (!width_ok(width) || !e_set || e_len <= 0 || k_hi < k_lo || !ids) return c->fail(PHPRNG_E_INVALID, "seed args");
  bool any = false;
  for (int i = 0; i < e_len; ++i) any = any || e_set[i] >= 3;
  if (!any) return c->fail(PHPRNG_E_EXPONENT, "no admissible exponent in the set");
  if (c->inst.size() + count > c->max_instances) return c->fail(PHPRNG_E_RANGE, "instance table full");
  if (width == 64 && k_hi > kTab64Range)
    return c->fail(PHPRNG_E_RANGE, "bulk width-64 starts must lie below 2^34 (the positioning table)");
  (void)hipSetDevice(c->device);
  std::vector<uint64_t> n(count), e(count), k(count);
  phprng_status st = draw_on_device(c, width, seed, count, e_set, e_len, k_lo, k_hi, n.data(), e.data(), k.data());
  if (st != PHPRNG_OK) return st;
  if (width == 64 && !c->have64) {
    st = c->build_table64();
    if (st != PHPRNG_OK) return st;
  }
  uint64_t *d_ne = nullptr;
  hipError_t he = hipMalloc(&d_ne, 3 * count * sizeof(uint64_t) + count * sizeof(uint32_t));
  if (he != hipSuccess) return c->hip_fail(he, "seed records");
  const uint64_t base = c->inst.size();
  uint32_t *d_ids = reinterpret_cast<uint32_t *>(d_ne + 3 * count);
  std::vector<uint32_t> hid(count);
  for (uint64_t i = 0; i < count; ++i) hid[i] = (uint32_t)(base + i);
  he = hipMemcpy(d_ne, n.data(), count * 8, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(d_ne + count, e.data(), count * 8, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = launch_build_records(d_ne, d_ne + count, count, width, c->d_inst + base, nullptr);
  if (he == hipSuccess && width == 64) {
    // messages at the start positions from the base state (0, 1): U(k) mod n
    he = hipMemcpy(d_ne + 2 * count, k.data(), count * 8, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(d_ids, hid.data(), count * 4, hipMemcpyHostToDevice);
    if (he == hipSuccess)
      he = launch_position64(c->d_inst, d_ids, nullptr, d_ne + 2 * count, nullptr, count, c->d_u64lo, c->d_u64hi,
                             c->d_s64, c->d_m64, nullptr);
  }
  if (he == hipSuccess) he = hipDeviceSynchronize();
  (void)hipFree(d_ne);
  if (he != hipSuccess) return c->hip_fail(he, "seed records");
  for (uint64_t i = 0; i < count; ++i) {
    HostInst h{n[i], e[i], width};
    h.x = k[i];
    h.k = k[i];
    c->inst.push_back(h);
    ids[i] = (uint32_t)(base + i);
  }
  if (c->where.size() < c->inst.size()) c->where.resize(c->inst.size(), -1);
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_add_instances_skip(phprng_ctx *c, uint64_t count, int width, const uint64_t *n,
                                                   const uint64_t *e, const uint64_t *b, const uint64_t *m0,
                                                   const uint64_t *k0, uint32_t *ids) {
  if (!c || !width_ok(width)) return PHPRNG_E_INVALID;
  if (count == 0) return PHPRNG_OK;
  if (!n || !e || !b || !ids) return c->fail(PHPRNG_E_INVALID, "null array");
  if (c->inst.size() + count > c->max_instances) return c->fail(PHPRNG_E_RANGE, "instance table full");
  (void)hipSetDevice(c->device);
  std::vector<HostInst> add(count);
  std::vector<InstRec> recs(count);
  for (uint64_t i = 0; i < count; ++i) {
    phprng_status st = check_instance_impl(width, n[i], e[i]);
    if (st != PHPRNG_OK) return c->fail(st, "instance %llu rejected", (unsigned long long)i);
    const uint64_t mm0 = m0 ? m0[i] : 0;
    if (b[i] == 0 || b[i] >= n[i] || mm0 >= n[i])
      return c->fail(PHPRNG_E_INVALID, "bad skip or m0 at %llu", (unsigned long long)i);
    HostInst h{n[i], e[i], width};
    h.sched = kSchedConstant;
    h.b = b[i];
    h.mbase = mm0;
    h.x = h.k = k0 ? k0[i] : 0;
    add[i] = h;
    recs[i] = c->make_record(h);
  }
  const uint64_t base = c->inst.size();
  hipError_t he = hipMemcpy(c->d_inst + base, recs.data(), count * sizeof(InstRec), hipMemcpyHostToDevice);
  if (he != hipSuccess) return c->hip_fail(he, "instance upload");
  for (uint64_t i = 0; i < count; ++i) {
    c->inst.push_back(add[i]);
    ids[i] = (uint32_t)(base + i);
  }
  if (c->where.size() < c->inst.size()) c->where.resize(c->inst.size(), -1);
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_schedule(phprng_ctx *c, uint32_t id, int *sched, uint64_t *b) {
  if (!c || id >= c->inst.size()) return PHPRNG_E_INVALID;
  const HostInst &h = c->inst[id];
  if (sched) *sched = (int)h.sched;
  if (b) *b = h.b;
  return PHPRNG_OK;
}

// ---------------------------------------------------------------------------
// generation
// ---------------------------------------------------------------------------

extern "C" phprng_status phprng_generate(phprng_ctx *c, const phprng_request *reqs, uint64_t nreq, uint32_t *out_c32,
                                         uint64_t *out_c64, double *out_r, uint64_t capacity, void *stream,
                                         int mode) {
  if (!c) return PHPRNG_E_INVALID;
  if (mode != PHPRNG_MODE_PERSISTENT && mode != PHPRNG_MODE_PLAIN) return c->fail(PHPRNG_E_INVALID, "bad mode");
  if (nreq == 0) return PHPRNG_OK;
  (void)hipSetDevice(c->device);
  phprng_ctx::Slot *slot = nullptr;
  phprng_status st = c->take_slot(nreq, &slot);
  if (st != PHPRNG_OK) return st;
  Plan P;
  st = c->plan(reqs, nreq, capacity, mode, nullptr, slot->cap, slot->h_blk, &P);
  if (st != PHPRNG_OK) return st;
  if ((st = c->ensure_tiles(*slot, P.tiles64)) != PHPRNG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  // Small batches are read by the kernels straight from the pinned block (a
  // few reads over the bus per chunk, no copy ahead of them); larger ones are
  // copied to device memory first, where the chunk searches run locally.
  const bool direct = nreq <= kDirectRequests;
  if (!direct) {
    const uint64_t bytes = sizeof(BatchHdr) + nreq * sizeof(ReqRec);
    if ((e = hipMemcpyAsync(slot->d_blk, slot->h_blk, bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
      return c->hip_fail(e, "request copy");
  }
  GenArgs A = c->args(direct ? slot->h_blk_dev : slot->d_blk, slot->d_ctr, slot->d_t64, slot->cap64, nreq, out_c32,
                      out_c64, out_r, P.tpc);
  if (c->timing_on && (e = hipEventRecord(slot->ev0, s)) != hipSuccess) return c->hip_fail(e, "event");
  st = c->launch(P, A, reinterpret_cast<const ReqRec *>(slot->h_blk + sizeof(BatchHdr)), s, mode);
  if (st != PHPRNG_OK) return st;
  if ((e = hipEventRecord(slot->ev1, s)) != hipSuccess) return c->hip_fail(e, "event");
  slot->busy = true;
  slot->timed = c->timing_on;
  c->last_timed = c->timing_on ? c->cur_slot : -1;
  c->commit_plan();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_generate_noalloc(phprng_ctx *c, const phprng_request *reqs, uint64_t nreq,
                                                 uint32_t *out_c32, uint64_t *out_c64, double *out_r,
                                                 uint64_t capacity, void *stream) {
  if (!c) return PHPRNG_E_INVALID;
  if (nreq == 0) return PHPRNG_OK;
  if (nreq > kNoAllocMaxRequests)
    return c->fail(PHPRNG_E_RANGE, "allocation-free generation takes at most %llu requests per call",
                   (unsigned long long)kNoAllocMaxRequests);
  (void)hipSetDevice(c->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  // the pinned staging block is rewritten only after the previous call's copy ran
  if (c->noalloc_pending) {
    if ((e = hipEventSynchronize(c->noalloc_copied)) != hipSuccess) return c->hip_fail(e, "staging wait");
    c->noalloc_pending = false;
  }
  Plan P;
  phprng_status st = c->plan(reqs, nreq, capacity, PHPRNG_MODE_PERSISTENT, nullptr, kNoAllocMaxRequests,
                             c->h_noalloc, &P);
  if (st != PHPRNG_OK) return st;
  if (P.tiles64 > kNoAllocMaxTiles64)
    return c->fail(PHPRNG_E_RANGE, "allocation-free generation takes at most %llu width-64 tiles (%llu draws) per call",
                   (unsigned long long)kNoAllocMaxTiles64, (unsigned long long)(kNoAllocMaxTiles64 * kTile64));
  uint8_t *blk = c->scratch + kScratchHdrOff;
  const uint64_t bytes = sizeof(BatchHdr) + nreq * sizeof(ReqRec);
  if ((e = hipMemcpyAsync(blk, c->h_noalloc, bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return c->hip_fail(e, "request copy");
  if ((e = hipEventRecord(c->noalloc_copied, s)) != hipSuccess) return c->hip_fail(e, "event");
  c->noalloc_pending = true;
  GenArgs A = c->args(blk, reinterpret_cast<WorkCtr *>(c->scratch + kScratchCtrOff),
                      reinterpret_cast<uint64_t *>(c->scratch + kScratchTileOff), kNoAllocMaxTiles64, nreq, out_c32,
                      out_c64, out_r, P.tpc);
  st = c->launch(P, A, reinterpret_cast<const ReqRec *>(c->h_noalloc + sizeof(BatchHdr)), s, PHPRNG_MODE_PERSISTENT);
  if (st != PHPRNG_OK) return st;
  c->commit_plan();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_last_kernel_ms(phprng_ctx *c, double *ms) {
  if (!c || !ms) return PHPRNG_E_INVALID;
  if (c->last_timed < 0)
    return c->fail(PHPRNG_E_INVALID, "the last call was not timed (no call yet, or timing off: phprng_set_timing)");
  phprng_ctx::Slot &s = c->slots[c->last_timed];
  hipError_t e = hipEventSynchronize(s.ev1);
  if (e != hipSuccess) return c->hip_fail(e, "event sync");
  float f = 0;
  if ((e = hipEventElapsedTime(&f, s.ev0, s.ev1)) != hipSuccess) return c->hip_fail(e, "event time");
  *ms = f;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_timing_reset(phprng_ctx *c) {
  if (!c) return PHPRNG_E_INVALID;
  for (auto &s : c->slots) {
    if (s.busy) {
      hipError_t e = c->retire(s);
      if (e != hipSuccess) return c->hip_fail(e, "timing reset");
    }
  }
  c->acc_ms = 0;
  c->acc_calls = 0;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_set_timing(phprng_ctx *c, int on) {
  if (!c) return PHPRNG_E_INVALID;
  c->timing_on = on != 0;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_timing_read(phprng_ctx *c, double *total_ms, uint64_t *calls) {
  if (!c || !total_ms || !calls) return PHPRNG_E_INVALID;
  for (auto &s : c->slots) {
    if (s.busy) {
      hipError_t e = c->retire(s);
      if (e != hipSuccess) return c->hip_fail(e, "timing read");
    }
  }
  *total_ms = c->acc_ms;
  *calls = c->acc_calls;
  return PHPRNG_OK;
}

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------

extern "C" phprng_status phprng_get_params(phprng_ctx *c, uint32_t id, uint64_t *n, uint64_t *e, uint64_t *p,
                                           uint64_t *a, int *width) {
  if (!c || id >= c->inst.size()) return PHPRNG_E_INVALID;
  const HostInst &h = c->inst[id];
  if (n) *n = h.n;
  if (e) *e = h.e;
  if (p) *p = group(h.width).p;
  if (a) *a = group(h.width).a;
  if (width) *width = h.width;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_state(phprng_ctx *c, uint32_t id, phprng_state *out) {
  if (!c || !out || id >= c->inst.size()) return PHPRNG_E_INVALID;
  (void)hipSetDevice(c->device);
  const HostInst &h = c->inst[id];
  uint64_t m, s;
  if (lcg64(h)) {
    phprng_status st = c->read_m64(id, &m);
    if (st != PHPRNG_OK) return st;
    s = group(64).powmod(kA64, h.x);
  } else {
    c->state_at(h, h.x, &m, &s);
  }
  Mont64 M(h.n);
  out->m = m;
  out->s = s;
  out->c = M.powmod(m, h.e);
  out->k = h.k;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_position(phprng_ctx *c, uint32_t id, uint64_t *k) {
  if (!c || !k || id >= c->inst.size()) return PHPRNG_E_INVALID;
  *k = c->inst[id].k;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_jump(phprng_ctx *c, uint32_t id, int64_t delta) {
  if (!c || id >= c->inst.size()) return PHPRNG_E_INVALID;
  (void)hipSetDevice(c->device);
  HostInst &h = c->inst[id];
  const bool forward = delta >= 0;
  const uint64_t d = forward ? (uint64_t)delta : (uint64_t)(-(delta + 1)) + 1;
  if (forward ? d > ~0ull - h.k : d > h.k) return c->fail(PHPRNG_E_RANGE, "jump beyond the position range");
  if (lcg64(h)) {
    phprng_status st = c->move64(id, d, forward, false);
    if (st != PHPRNG_OK) return st;
    const uint64_t pm1 = kP64 - 1, r = d % pm1;
    h.x = forward ? add_u64_mod(h.x, r, pm1) : (h.x >= r ? h.x - r : h.x + (pm1 - r));
  } else {
    if (forward ? d > ~0ull - h.x : d > h.x) return c->fail(PHPRNG_E_RANGE, "jump beyond the position range");
    h.x = forward ? h.x + d : h.x - d;
  }
  h.k = forward ? h.k + d : h.k - d;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_set_state(phprng_ctx *c, uint32_t id, const phprng_state *st) {
  if (!c || !st || id >= c->inst.size()) return PHPRNG_E_INVALID;
  (void)hipSetDevice(c->device);
  HostInst &h = c->inst[id];
  if (h.sched == kSchedConstant) {
    if (st->m >= h.n || st->s != h.b) return c->fail(PHPRNG_E_INVALID, "bad state for a constant skip");
    Mont64 M(h.n);
    HostInst tmp = h;
    tmp.mbase = M.sub(st->m, M.mulmod(st->k % h.n, h.b));
    InstRec rec = c->make_record(tmp);
    hipError_t e = hipMemcpy(c->d_inst + id, &rec, sizeof rec, hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "instance upload");
    h.mbase = tmp.mbase;
    h.x = h.k = st->k;
    return PHPRNG_OK;
  }
  const SkipGroup &G = group(h.width);
  if (st->m >= h.n || st->s == 0 || st->s >= G.p) return c->fail(PHPRNG_E_INVALID, "bad state");
  const uint64_t pm1 = G.p - 1;
  const uint64_t t = G.dlog(st->s);
  if (h.width == 64) {
    phprng_status ws = c->write_m64(id, st->m);
    if (ws != PHPRNG_OK) return ws;
    h.x = t;
    h.k = st->k;
    return PHPRNG_OK;
  }
  const uint64_t q = st->k / pm1;
  const uint64_t x = q * pm1 + t;
  HostInst tmp = h;
  tmp.mbase = 0;
  uint64_t mu, su;
  c->state_at(tmp, x, &mu, &su);
  Mont64 M(h.n);
  const uint64_t mbase = M.sub(st->m, mu);
  tmp.mbase = mbase;
  InstRec rec = c->make_record(tmp);
  hipError_t e = hipMemcpy(c->d_inst + id, &rec, sizeof rec, hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "instance upload");
  h.mbase = mbase;
  h.x = x;
  h.k = st->k;
  return PHPRNG_OK;
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------

static phprng_status check_tuning(phprng_ctx *c, const phprng_tuning &v) {
  if (v.block_threads != 64 && v.block_threads != 128 && v.block_threads != 256 && v.block_threads != 512)
    return c->fail(PHPRNG_E_INVALID, "block_threads");
  if (v.blocks_per_cu < 1 || v.blocks_per_cu > 64) return c->fail(PHPRNG_E_INVALID, "blocks_per_cu");
  if (v.tiles_per_chunk < 1 || v.tiles_per_chunk > 64) return c->fail(PHPRNG_E_INVALID, "tiles_per_chunk");
  if (v.unroll != 1 && v.unroll != 2 && v.unroll != 4) return c->fail(PHPRNG_E_INVALID, "unroll");
  return PHPRNG_OK;
}

static phprng_tuning merge_tuning(const phprng_tuning &base, const phprng_tuning *t) {
  phprng_tuning v = base;
  if (t->block_threads) v.block_threads = t->block_threads;
  if (t->blocks_per_cu) v.blocks_per_cu = t->blocks_per_cu;
  if (t->tiles_per_chunk) v.tiles_per_chunk = t->tiles_per_chunk;
  if (t->unroll) v.unroll = t->unroll;
  return v;
}

extern "C" phprng_status phprng_set_tuning_class(phprng_ctx *c, int cls, const phprng_tuning *t) {
  if (!c || !t || cls < 0 || cls > 2) return PHPRNG_E_INVALID;
  const phprng_tuning v = merge_tuning(c->tuning[cls], t);
  phprng_status st = check_tuning(c, v);
  if (st != PHPRNG_OK) return st;
  c->tuning[cls] = v;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_tuning_class(phprng_ctx *c, int cls, phprng_tuning *t) {
  if (!c || !t || cls < 0 || cls > 2) return PHPRNG_E_INVALID;
  *t = c->tuning[cls];
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_set_tuning(phprng_ctx *c, const phprng_tuning *t) {
  if (!c || !t) return PHPRNG_E_INVALID;
  phprng_tuning v[3];
  for (int cls = 0; cls < 3; ++cls) {
    v[cls] = merge_tuning(c->tuning[cls], t);
    phprng_status st = check_tuning(c, v[cls]);
    if (st != PHPRNG_OK) return st;
  }
  for (int cls = 0; cls < 3; ++cls) c->tuning[cls] = v[cls];
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_tuning(phprng_ctx *c, phprng_tuning *t) {
  return phprng_get_tuning_class(c, PHPRNG_CLASS_W32, t);
}

extern "C" phprng_status phprng_autotune(phprng_ctx *c, uint64_t draws, phprng_tuning *best) {
  if (!c || draws == 0) return PHPRNG_E_INVALID;
  if (c->inst.empty()) return c->fail(PHPRNG_E_INVALID, "no instances");
  (void)hipSetDevice(c->device);
  const uint64_t ninst = std::min<uint64_t>(c->inst.size(), 4096);
  const uint64_t per = std::max<uint64_t>(draws / ninst, 1);
  std::vector<phprng_request> reqs(ninst);
  for (uint64_t i = 0; i < ninst; ++i) reqs[i] = phprng_request{(uint32_t)i, 0, per, i * per};
  const uint64_t cap = ninst * per;
  bool any64 = false, any32 = false;
  for (uint64_t i = 0; i < ninst; ++i) (c->inst[i].width == 64 ? any64 : any32) = true;
  const int cls = any64 ? (any32 ? kMixBoth : kMix64) : kMix32;
  double *d_r = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&d_r, cap * 8)) != hipSuccess) return c->hip_fail(e, "autotune alloc");
  // positions and (width 64) device messages are restored afterwards
  std::vector<std::pair<uint64_t, uint64_t>> saved(ninst);
  for (uint64_t i = 0; i < ninst; ++i) saved[i] = {c->inst[i].x, c->inst[i].k};
  std::vector<uint64_t> m64;
  phprng_status result = PHPRNG_OK;
  if (any64) {
    if ((result = c->sync_chain()) == PHPRNG_OK) {
      m64.resize(ninst);
      if ((e = hipMemcpy(m64.data(), c->d_m64, ninst * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        result = c->hip_fail(e, "autotune save");
    }
  }
  const phprng_tuning orig = c->tuning[cls];
  // the candidates are timed with events whatever the caller's setting
  const bool timing_was = c->timing_on;
  c->timing_on = true;
  // one timed call: median kernel time of `reps` calls of shape t
  auto run = [&](const phprng_tuning &t, int reps) -> double {
    c->tuning[cls] = t;
    std::vector<double> v;
    for (int rep = 0; rep < reps && result == PHPRNG_OK; ++rep) {
      for (uint64_t i = 0; i < ninst; ++i) std::tie(c->inst[i].x, c->inst[i].k) = saved[i];
      phprng_status st = phprng_generate(c, reqs.data(), ninst, nullptr, nullptr, d_r, cap, nullptr,
                                         PHPRNG_MODE_PERSISTENT);
      double ms = 0;
      if (st == PHPRNG_OK) st = phprng_last_kernel_ms(c, &ms);
      if (st != PHPRNG_OK) result = st;
      v.push_back(ms);
    }
    if (v.empty()) return 1e30;
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
  };
  phprng_tuning bestT = orig;
  if (result == PHPRNG_OK) {
    // bring the clocks up before timing anything
    auto t0 = std::chrono::steady_clock::now();
    while (result == PHPRNG_OK && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(300)) run(orig, 1);
    double best_ms = run(orig, 5);
    const int blocks[] = {256, 512, 128, 64};
    const int bpcs[] = {1, 2, 4, 8};
    const int tpcs[] = {1, 2, 4, 8, 16};
    const int unrolls[] = {1, 2, 4};
    for (int b : blocks)
      for (int bpc : bpcs)
        for (int tpc : tpcs)
          for (int u : unrolls) {
            if (b * bpc > 2048 || result != PHPRNG_OK) continue;
            const phprng_tuning t{b, bpc, tpc, u};
            const double ms = run(t, 3);
            if (ms < best_ms) {
              best_ms = ms;
              bestT = t;
            }
          }
    // confirm the winner against the starting shape with more repetitions
    if (result == PHPRNG_OK && run(bestT, 7) > run(orig, 7)) bestT = orig;
  }
  for (uint64_t i = 0; i < ninst; ++i) std::tie(c->inst[i].x, c->inst[i].k) = saved[i];
  if (any64 && !m64.empty()) {
    phprng_status s2 = c->sync_chain();
    if (s2 == PHPRNG_OK && (e = hipMemcpy(c->d_m64, m64.data(), ninst * 8, hipMemcpyHostToDevice)) != hipSuccess)
      s2 = c->hip_fail(e, "autotune restore");
    if (result == PHPRNG_OK) result = s2;
  }
  (void)hipDeviceSynchronize();
  (void)hipFree(d_r);
  c->tuning[cls] = result == PHPRNG_OK ? bestT : orig;
  if (result == PHPRNG_OK) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[TuneKey{c->arch, c->num_cus, cls}] = bestT;
  }
  if (best) *best = c->tuning[cls];
  c->timing_on = timing_was;
  return result;
}

// ---------------------------------------------------------------------------
// captured repeat draws
// ---------------------------------------------------------------------------

extern "C" phprng_status phprng_graph_create(phprng_ctx *c, const phprng_request *reqs, uint64_t nreq,
                                             uint32_t *out_c32, uint64_t *out_c64, double *out_r, uint64_t capacity,
                                             void *stream, phprng_graph **graph) {
  if (!c || !graph || nreq == 0 || !reqs) return PHPRNG_E_INVALID;
  *graph = nullptr;
  (void)stream;
  (void)hipSetDevice(c->device);
  {
    std::vector<uint8_t> used(c->inst.size(), 0);
    for (uint64_t i = 0; i < nreq; ++i) {
      if (reqs[i].instance < c->inst.size()) {
        if (used[reqs[i].instance]) return c->fail(PHPRNG_E_INVALID, "graph requests must name distinct instances");
        used[reqs[i].instance] = 1;
      }
    }
  }
  // plan once from the current positions (not reserved: every launch plans again)
  phprng_ctx::Slot *slot = nullptr;
  phprng_status st = c->take_slot(nreq, &slot);
  if (st != PHPRNG_OK) return st;
  Plan P;
  st = c->plan(reqs, nreq, capacity, PHPRNG_MODE_PERSISTENT, nullptr, slot->cap, slot->h_blk, &P);
  if (st != PHPRNG_OK) return st;
  std::unique_ptr<phprng_graph> g(new (std::nothrow) phprng_graph);
  if (!g) return PHPRNG_E_NOMEM;
  g->ctx = c;
  g->reqs.assign(reqs, reqs + nreq);
  g->nreq64 = P.nreq64;
  g->tpc = P.tpc;
  g->has64 = P.has64;
  // Each replay finds every instance's tile starts in whichever way its
  // position allows (the table, or the reduce and scan): a request takes
  // ceil(count / 1024) tiles the second way and at most one more the first.
  uint64_t cap64 = 1;
  for (uint64_t i = 0; i < nreq; ++i)
    if (lcg64(c->inst[reqs[i].instance])) cap64 += (reqs[i].count + kTile64 - 1) / kTile64 + 1;
  g->cap64 = cap64;
  hipError_t e;
  const uint64_t bytes = sizeof(BatchHdr) + nreq * sizeof(ReqRec);
  if ((e = hipMalloc(&g->d_blk, bytes)) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMalloc(&g->d_ctr, sizeof(WorkCtr))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMemset(g->d_ctr, 0, sizeof(WorkCtr))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMalloc(&g->d_t64, 3 * cap64 * sizeof(uint64_t))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming)) != hipSuccess) return c->hip_fail(e, "event");
  const phprng_tuning &T = c->tuning[P.cls];
  GenArgs A = c->args(g->d_blk, g->d_ctr, g->d_t64, cap64, nreq, out_c32, out_c64, out_r, P.tpc);
  hipStream_t cap_stream;
  if ((e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking)) != hipSuccess) return c->hip_fail(e, "stream");
  e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
  // all three tile-start kernels, on grids that fit any replay: each reads
  // from the replay's block which instances are its own
  const unsigned reduce_blocks = (unsigned)c->num_cus * 8;
  if (e == hipSuccess && P.nreq64 > 0) e = launch_tiles64_reduce(A, 4ull * reduce_blocks, reduce_blocks, cap_stream);
  if (e == hipSuccess && P.nreq64 > 0) e = launch_tiles64_table(A, P.nreq64, cap_stream);
  if (e == hipSuccess && P.nreq64 > 0) e = launch_tiles64_scan(A, P.nreq64, cap_stream);
  if (e == hipSuccess)
    e = launch_persistent(A, (unsigned)(c->num_cus * T.blocks_per_cu), T.block_threads, T.unroll, P.has64, cap_stream);
  hipError_t e2 = hipStreamEndCapture(cap_stream, &g->graph);
  (void)hipStreamDestroy(cap_stream);
  if (e != hipSuccess || e2 != hipSuccess) return c->hip_fail(e != hipSuccess ? e : e2, "graph capture");
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return c->hip_fail(e, "graph instantiate");
  *graph = g.release();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_graph_launch(phprng_graph *g, void *stream) {
  if (!g || !g->ctx) return PHPRNG_E_INVALID;
  phprng_ctx *c = g->ctx;
  (void)hipSetDevice(c->device);
  const uint64_t nreq = g->reqs.size();
  phprng_ctx::Slot *slot = nullptr;
  phprng_status st = c->take_slot(nreq, &slot);
  if (st != PHPRNG_OK) return st;
  // plan from the instances' current positions, whatever moved them since
  // the last launch (generate, jump, set_state)
  Plan P;
  uint64_t capacity = ~0ull;
  st = c->plan(g->reqs.data(), nreq, capacity, PHPRNG_MODE_PERSISTENT, &g->tpc, slot->cap, slot->h_blk, &P);
  if (st != PHPRNG_OK) return st;
  if (P.nreq64 != g->nreq64 || P.tiles64 > g->cap64)
    return c->fail(PHPRNG_E_INVALID, "graph requests no longer match their instances");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  // the previous launch must be done with the request block before it is rewritten
  if (g->launched && (e = hipStreamWaitEvent(s, g->done, 0)) != hipSuccess) return c->hip_fail(e, "graph wait");
  const uint64_t bytes = sizeof(BatchHdr) + nreq * sizeof(ReqRec);
  if ((e = hipMemcpyAsync(g->d_blk, slot->h_blk, bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return c->hip_fail(e, "request copy");
  if (g->nreq64 > 0 && c->chain_pending && (e = hipStreamWaitEvent(s, c->chain_ev, 0)) != hipSuccess)
    return c->hip_fail(e, "chain wait");
  if (c->timing_on && (e = hipEventRecord(slot->ev0, s)) != hipSuccess) return c->hip_fail(e, "event");
  if ((e = hipGraphLaunch(g->exec, s)) != hipSuccess) return c->hip_fail(e, "graph launch");
  if ((e = hipEventRecord(slot->ev1, s)) != hipSuccess) return c->hip_fail(e, "event");
  if ((e = hipEventRecord(g->done, s)) != hipSuccess) return c->hip_fail(e, "event");
  if (g->nreq64 > 0) {
    if ((e = hipEventRecord(c->chain_ev, s)) != hipSuccess) return c->hip_fail(e, "chain record");
    c->chain_pending = true;
  }
  g->launched = true;
  slot->busy = true;
  slot->timed = c->timing_on;
  c->last_timed = c->timing_on ? c->cur_slot : -1;
  c->commit_plan();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_graph_destroy(phprng_graph *g) {
  if (!g) return PHPRNG_E_INVALID;
  if (g->ctx) (void)hipSetDevice(g->ctx->device);
  (void)hipDeviceSynchronize();
  delete g;
  return PHPRNG_OK;
}
