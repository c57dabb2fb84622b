// Host runtime behind include/phprng.h: instance tables, seeding, the
// universal skip-prefix tables, request planning and kernel launches,
// jumps and state restore, captured repeat draws.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
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
  uint64_t mbase;  // m at internal index x = mbase + q p(p-1)/2 + U(r) mod n (constant skip: mbase + x b)
  uint64_t x;      // internal index of the current state
  int64_t kofs;    // reported position k = x - kofs
  uint32_t sched = kSchedSkipLcg;
  uint64_t b = 0;  // constant skip
};

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

}  // namespace

struct phprng_graph {
  phprng_ctx *ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HostReq *d_src = nullptr;  // requests; the graph's last node advances them
  ReqRec *d_req = nullptr;
  uint64_t *d_gbase = nullptr;
  PlanHdr *d_hdr = nullptr;
  std::vector<uint32_t> inst;
  std::vector<uint64_t> count;
};

struct phprng_ctx {
  int device = 0;
  int num_cus = 0;
  uint64_t max_instances = 0;
  std::vector<HostInst> inst;
  InstRec *d_inst = nullptr;
  LaneMul *d_lanemul = nullptr;
  // universal skip-prefix tables: host mirrors and device copies
  std::vector<uint64_t> u32;
  std::vector<uint32_t> s32;
  std::vector<u128> u64;
  std::vector<uint64_t> s64;
  uint64_t *d_u32 = nullptr;
  uint32_t *d_s32 = nullptr;
  uint64_t *d_u64lo = nullptr, *d_u64hi = nullptr, *d_s64 = nullptr;
  bool have64 = false;
  // Request staging: a ring of slots so that consecutive calls (possibly on
  // different streams) never overwrite a request list still in use.  A slot
  // is reused only after the event recorded behind its last kernel.
  struct Slot {
    HostReq *h_req = nullptr;            // pinned, mapped
    const HostReq *h_req_dev = nullptr;  // h_req's address for kernels
    ReqRec *d_req = nullptr;
    uint64_t *d_gbase = nullptr;         // ceil(cap / kPlanGroup) words
    uint64_t cap = 0;
    PlanHdr *d_hdr = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, done = nullptr;
    bool busy = false;
  };
  static constexpr int kSlots = 8;
  static constexpr uint64_t kMinSlotRequests = 8192;
  Slot slots[kSlots];
  int cur_slot = 0;
  int last_timed = -1;
  double acc_ms = 0;        // cumulative kernel time of recycled slots
  uint64_t acc_calls = 0;
  HostReq *h_req = nullptr;  // staging array of the slot being prepared
  // Per instance: its index in the touched list of the batch being prepared;
  // -1 between calls, so that a batch costs O(requests), not O(instances).
  std::vector<int64_t> where;
  phprng_tuning tuning{256, 4, 8, 4};
  std::string err;

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

  // U(r) = sum_{j=1}^{r} (a^j mod p) and a^r mod p, from the table entry at or
  // below r plus at most stride-1 host steps.
  void prefix(int width, uint64_t r, u128 *U, uint64_t *S) const {
    const SkipGroup &G = group(width);
    const uint64_t i = r / kTableStride;
    u128 u = width == 32 ? (u128)u32[i] : u64[i];
    uint64_t s = width == 32 ? (uint64_t)s32[i] : s64[i];
    for (uint64_t x = i * kTableStride; x < r; ++x) {
      s = G.mulmod(G.a, s);
      u += s;
    }
    *U = u;
    *S = s;
  }

  // State (m, s) at internal index x of instance h (eq. (7); constant skip:
  // m = m_0 + x b, s = b).
  void state_at(const HostInst &h, uint64_t x, uint64_t *m, uint64_t *s) const {
    if (h.sched == kSchedConstant) {
      Mont64 M(h.n);
      *m = M.add(h.mbase % h.n, M.mulmod(x % h.n, h.b));
      *s = h.b;
      return;
    }
    const SkipGroup &G = group(h.width);
    const uint64_t pm1 = G.p - 1;
    const uint64_t q = x / pm1, r = x % pm1;
    u128 U;
    prefix(h.width, r, &U, s);
    Mont64 M(h.n);
    const u128 full = ((u128)G.p * (G.p - 1)) / 2;
    uint64_t b = M.reduce128(full);
    uint64_t qb = M.mulmod(q % h.n, b);
    *m = M.add(M.add(h.mbase % h.n, M.reduce128(U)), qb);
  }

  uint64_t max_index(const HostInst &h) const {
    return (h.width == 32 || h.sched == kSchedConstant) ? ~0ull : kMaxPos64;
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
    hipError_t e = hipEventSynchronize(s.done);
    if (e != hipSuccess) return e;
    float f = 0;
    if (hipEventElapsedTime(&f, s.ev0, s.ev1) == hipSuccess) {
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
    hipError_t e;
    if (s.busy) {
      if ((e = retire(s)) != hipSuccess) return hip_fail(e, "slot wait");
    }
    if (!s.ev0) {
      if ((e = hipEventCreate(&s.ev0)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventCreate(&s.ev1)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipMalloc(&s.d_hdr, sizeof(PlanHdr))) != hipSuccess) return fail(PHPRNG_E_NOMEM, "plan header");
      // the plan kernel expects a zero completion counter and leaves it so
      if ((e = hipMemset(s.d_hdr, 0, sizeof(PlanHdr))) != hipSuccess) return hip_fail(e, "plan header");
    }
    if (nreq > s.cap) {
      // room for typical batches from the start: growing frees buffers,
      // which waits for the device
      uint64_t cap = std::max<uint64_t>({nreq, 2 * s.cap, kMinSlotRequests});
      if (s.d_req) (void)hipFree(s.d_req);
      if (s.d_gbase) (void)hipFree(s.d_gbase);
      if (s.h_req) (void)hipHostFree(s.h_req);
      s.d_req = nullptr;
      s.d_gbase = nullptr;
      s.h_req = nullptr;
      s.h_req_dev = nullptr;
      s.cap = 0;
      if ((e = hipMalloc(&s.d_req, cap * sizeof(ReqRec))) != hipSuccess)
        return fail(PHPRNG_E_NOMEM, "request buffer: %s", hipGetErrorString(e));
      if ((e = hipMalloc(&s.d_gbase, (cap + kPlanGroup - 1) / kPlanGroup * sizeof(uint64_t))) != hipSuccess)
        return fail(PHPRNG_E_NOMEM, "plan buffer: %s", hipGetErrorString(e));
      if ((e = hipHostMalloc(&s.h_req, cap * sizeof(HostReq), hipHostMallocMapped)) != hipSuccess)
        return fail(PHPRNG_E_NOMEM, "pinned request buffer: %s", hipGetErrorString(e));
      void *dp = nullptr;
      if ((e = hipHostGetDevicePointer(&dp, s.h_req, 0)) != hipSuccess || !dp)
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidValue, "pinned request buffer address");
      s.h_req_dev = static_cast<const HostReq *>(dp);
      s.cap = cap;
    }
    h_req = s.h_req;
    *out = &s;
    return PHPRNG_OK;
  }

  phprng_status build_table32();
  phprng_status build_table64();
};

phprng_status phprng_ctx::build_table32() {
  const uint64_t pm1 = (uint64_t)kP32 - 1;
  const uint64_t ne = (pm1 - 1) / kTableStride + 1;  // entries at 0, stride, ... <= p - 2
  uint64_t *d_sum = nullptr;
  uint32_t *d_start = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&d_sum, ne * sizeof(uint64_t))) != hipSuccess) return hip_fail(e, "table32 alloc");
  if ((e = hipMalloc(&d_start, ne * sizeof(uint32_t))) != hipSuccess) {
    (void)hipFree(d_sum);
    return hip_fail(e, "table32 alloc");
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
  prefix(32, pm1, &U, &S);
  if (U != ((u128)kP32 * pm1) / 2 || S != 1) {
    (void)hipFree(d_start);
    return fail(PHPRNG_E_DEVICE, "32-bit skip-prefix table failed its full-period check");
  }
  d_s32 = d_start;
  if ((e = hipMalloc(&d_u32, ne * sizeof(uint64_t))) != hipSuccess) return hip_fail(e, "table32 alloc");
  if ((e = hipMemcpy(d_u32, u32.data(), ne * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "table32 upload");
  return PHPRNG_OK;
}

phprng_status phprng_ctx::build_table64() {
  if (have64) return PHPRNG_OK;
  const uint64_t ne = kMaxPos64 / kTableStride;
  uint64_t *d_lo = nullptr, *d_hi = nullptr, *d_start = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&d_lo, ne * 8)) != hipSuccess) return hip_fail(e, "table64 alloc");
  if ((e = hipMalloc(&d_hi, ne * 8)) != hipSuccess) return hip_fail(e, "table64 alloc");
  if ((e = hipMalloc(&d_start, ne * 8)) != hipSuccess) return hip_fail(e, "table64 alloc");
  if ((e = launch_table_segments64(ne, d_lo, d_hi, d_start, nullptr)) != hipSuccess)
    return hip_fail(e, "table64 launch");
  std::vector<uint64_t> lo(ne), hi(ne);
  s64.resize(ne);
  if ((e = hipMemcpy(lo.data(), d_lo, ne * 8, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipMemcpy(hi.data(), d_hi, ne * 8, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipMemcpy(s64.data(), d_start, ne * 8, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "copy");
  u64.resize(ne);
  u128 acc = 0;
  for (uint64_t i = 0; i < ne; ++i) {
    u64[i] = acc;
    acc += ((u128)hi[i] << 64) | lo[i];
    lo[i] = (uint64_t)u64[i];
    hi[i] = (uint64_t)(u64[i] >> 64);
  }
  // Spot-check a few entries against host stepping from the previous entry.
  const SkipGroup &G = group(64);
  for (uint64_t i : {(uint64_t)1, ne / 3, ne - 1}) {
    u128 u = u64[i - 1];
    uint64_t s = s64[i - 1];
    for (uint64_t x = 0; x < kTableStride; ++x) {
      s = G.mulmod(G.a, s);
      u += s;
    }
    if (u != u64[i] || s != s64[i] || s != G.powmod(G.a, i * kTableStride))
      return fail(PHPRNG_E_DEVICE, "64-bit skip-prefix table failed its check at entry %llu", (unsigned long long)i);
  }
  if ((e = hipMemcpy(d_lo, lo.data(), ne * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "upload");
  if ((e = hipMemcpy(d_hi, hi.data(), ne * 8, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "upload");
  d_u64lo = d_lo;
  d_u64hi = d_hi;
  d_s64 = d_start;
  have64 = true;
  return PHPRNG_OK;
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
  std::unique_ptr<phprng_ctx> c(new (std::nothrow) phprng_ctx);
  if (!c) return PHPRNG_E_NOMEM;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PHPRNG_E_INVALID;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return PHPRNG_E_DEVICE;
  c->device = device;
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return PHPRNG_E_DEVICE;
  c->num_cus = prop.multiProcessorCount;
  c->max_instances = max_instances;
  if (hipMalloc(&c->d_inst, max_instances * sizeof(InstRec)) != hipSuccess) return PHPRNG_E_NOMEM;
  // lane start multipliers a^{l * run} mod p
  LaneMul lm;
  const SkipGroup &g32 = group(32), &g64 = group(64);
  for (int l = 0; l < 64; ++l) {
    lm.m32[l] = (uint32_t)g32.powmod(g32.a, (uint64_t)l * kRun);
    lm.m64[l] = g64.powmod(g64.a, (uint64_t)l * kRun);
  }
  if (hipMalloc(&c->d_lanemul, sizeof(LaneMul)) != hipSuccess) return PHPRNG_E_NOMEM;
  if (hipMemcpy(c->d_lanemul, &lm, sizeof lm, hipMemcpyHostToDevice) != hipSuccess) return PHPRNG_E_DEVICE;
  phprng_status st = c->build_table32();
  if (st != PHPRNG_OK) return st;
  *out = c.release();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_destroy(phprng_ctx *c) {
  if (!c) return PHPRNG_E_INVALID;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(c->d_inst);
  (void)hipFree(c->d_lanemul);
  (void)hipFree(c->d_u32);
  (void)hipFree(c->d_s32);
  (void)hipFree(c->d_u64lo);
  (void)hipFree(c->d_u64hi);
  (void)hipFree(c->d_s64);
  for (auto &s : c->slots) {
    (void)hipFree(s.d_req);
    (void)hipFree(s.d_gbase);
    if (s.h_req) (void)hipHostFree(s.h_req);
    (void)hipFree(s.d_hdr);
    if (s.ev0) (void)hipEventDestroy(s.ev0);
    if (s.ev1) (void)hipEventDestroy(s.ev1);
    if (s.done) (void)hipEventDestroy(s.done);
  }
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
  for (uint64_t i = 0; i < count; ++i) {
    phprng_status st = check_instance_impl(width, n[i], e[i]);
    if (st != PHPRNG_OK) return c->fail(st, "instance %llu rejected", (unsigned long long)i);
  }
  if (width == 64 && !c->have64) {
    phprng_status bs = c->build_table64();
    if (bs != PHPRNG_OK) return bs;
  }
  const SkipGroup &G = group(width);
  std::vector<HostInst> add(count);
  for (uint64_t i = 0; i < count; ++i) {
    phprng_status st = check_instance_impl(width, n[i], e[i]);
    if (st != PHPRNG_OK) return c->fail(st, "instance %llu rejected", (unsigned long long)i);
    const uint64_t mm0 = m0 ? m0[i] : 0, ss0 = s0 ? s0[i] : 1, kk = k0 ? k0[i] : 0;
    if (mm0 >= n[i] || ss0 == 0 || ss0 >= G.p) return c->fail(PHPRNG_E_INVALID, "bad m0/s0 at %llu", (unsigned long long)i);
    const uint64_t t0 = ss0 == 1 ? 0 : G.dlog(ss0);
    if (width == 64 && (t0 >= kMaxPos64 || kk >= kMaxPos64 - t0))
      return c->fail(PHPRNG_E_RANGE, "width-64 start beyond the supported range");
    if (width == 32 && kk > ~0ull - t0) return c->fail(PHPRNG_E_RANGE, "start index overflows");
    add[i] = HostInst{n[i], e[i], width, 0, t0 + kk, (int64_t)t0};
    // mbase such that the state at internal index t0 is (m0, s0): m0 - U(t0)
    if (t0 != 0 || mm0 != 0) {
      HostInst tmp = add[i];
      tmp.mbase = 0;
      uint64_t mu, su;
      c->state_at(tmp, t0, &mu, &su);
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
  if (width == 64 && k_hi > kMaxPos64) return c->fail(PHPRNG_E_RANGE, "width-64 start beyond the supported range");
  (void)hipSetDevice(c->device);
  std::vector<uint64_t> n(count), e(count), k(count);
  phprng_status st = draw_on_device(c, width, seed, count, e_set, e_len, k_lo, k_hi, n.data(), e.data(), k.data());
  if (st != PHPRNG_OK) return st;
  if (width == 64 && !c->have64) {
    st = c->build_table64();
    if (st != PHPRNG_OK) return st;
  }
  uint64_t *d_ne = nullptr;
  hipError_t he = hipMalloc(&d_ne, 2 * count * sizeof(uint64_t));
  if (he != hipSuccess) return c->hip_fail(he, "seed records");
  const uint64_t base = c->inst.size();
  he = hipMemcpy(d_ne, n.data(), count * 8, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(d_ne + count, e.data(), count * 8, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = launch_build_records(d_ne, d_ne + count, count, width, c->d_inst + base, nullptr);
  if (he == hipSuccess) he = hipDeviceSynchronize();
  (void)hipFree(d_ne);
  if (he != hipSuccess) return c->hip_fail(he, "seed records");
  for (uint64_t i = 0; i < count; ++i) {
    c->inst.push_back(HostInst{n[i], e[i], width, 0, k[i], 0});
    ids[i] = (uint32_t)(base + i);
  }
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
    HostInst h{n[i], e[i], width, mm0, k0 ? k0[i] : 0, 0};
    h.sched = kSchedConstant;
    h.b = b[i];
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
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_schedule(phprng_ctx *c, uint32_t id, int *sched, uint64_t *b) {
  if (!c || id >= c->inst.size()) return PHPRNG_E_INVALID;
  const HostInst &h = c->inst[id];
  if (sched) *sched = (int)h.sched;
  if (b) *b = h.b;
  return PHPRNG_OK;
}

namespace {

// Validate a request list and reserve positions.  Fills the slot's staging
// array (width-64 requests first, for load balance) and returns the new
// internal positions through `moves`; the caller applies them once every
// launch has been issued.
phprng_status prepare_requests(phprng_ctx *c, const phprng_request *reqs, uint64_t nreq, uint64_t capacity,
                               phprng_ctx::Slot **slot, bool *has64,
                               std::vector<std::pair<uint32_t, uint64_t>> *moves) {
  if (nreq > 0 && !reqs) return c->fail(PHPRNG_E_INVALID, "null request array");
  uint64_t n64 = 0;
  for (uint64_t i = 0; i < nreq; ++i) {
    const phprng_request &r = reqs[i];
    if (r.instance >= c->inst.size() || r.reserved != 0)
      return c->fail(PHPRNG_E_INVALID, "request %llu: bad instance", (unsigned long long)i);
    if (r.count > capacity || r.out_offset > capacity - r.count)
      return c->fail(PHPRNG_E_RANGE, "request %llu: output range beyond capacity", (unsigned long long)i);
    if (c->inst[r.instance].width == 64) ++n64;
  }
  *has64 = n64 > 0;
  // tentative positions, in request order
  std::vector<uint32_t> touched;
  std::vector<uint64_t> cur;
  if (c->where.size() < c->inst.size()) c->where.resize(c->inst.size(), -1);
  std::vector<int64_t> &where = c->where;
  struct Reset {  // back to -1 on every way out
    std::vector<int64_t> &w;
    const std::vector<uint32_t> &t;
    ~Reset() {
      for (uint32_t i : t) w[i] = -1;
    }
  } reset{where, touched};
  for (uint64_t i = 0; i < nreq; ++i) {
    const phprng_request &r = reqs[i];
    const HostInst &h = c->inst[r.instance];
    if (where[r.instance] < 0) {
      where[r.instance] = (int64_t)touched.size();
      touched.push_back(r.instance);
      cur.push_back(h.x);
    }
    uint64_t &x = cur[(size_t)where[r.instance]];
    if (r.count > c->max_index(h) - x)
      return c->fail(PHPRNG_E_RANGE, "request %llu: position beyond range", (unsigned long long)i);
    x += r.count;
  }
  phprng_status st = c->take_slot(std::max<uint64_t>(nreq, 1), slot);
  if (st != PHPRNG_OK) return st;
  for (size_t t = 0; t < touched.size(); ++t) cur[t] = c->inst[touched[t]].x;
  uint64_t w64 = 0, w32 = n64;
  for (uint64_t i = 0; i < nreq; ++i) {
    const phprng_request &r = reqs[i];
    const HostInst &h = c->inst[r.instance];
    uint64_t &x = cur[(size_t)where[r.instance]];
    HostReq rec;
    memset(&rec, 0, sizeof rec);
    rec.k = x;
    rec.count = r.count;
    rec.out_off = r.out_offset;
    rec.inst = r.instance;
    c->h_req[h.width == 64 ? w64++ : w32++] = rec;
    x += r.count;
  }
  moves->clear();
  for (size_t t = 0; t < touched.size(); ++t) moves->push_back({touched[t], cur[t]});
  return PHPRNG_OK;
}

}  // namespace

static GenArgs make_args(phprng_ctx *c, ReqRec *d_req, const uint64_t *d_gbase, PlanHdr *d_hdr, uint64_t nreq,
                         uint32_t *out_c32, uint64_t *out_c64, double *out_r, uint32_t tpc) {
  GenArgs A;
  A.inst = c->d_inst;
  A.req = d_req;
  A.gbase = d_gbase;
  A.hdr = d_hdr;
  A.nreq = nreq;
  A.tab = SkipTables{c->d_u32, c->d_s32, c->d_u64lo, c->d_u64hi, c->d_s64, c->u32.size(), c->s64.size()};
  A.lanemul = c->d_lanemul;
  A.out_c32 = out_c32;
  A.out_c64 = out_c64;
  A.out_r = out_r;
  A.tiles_per_chunk = tpc;
  return A;
}

extern "C" phprng_status phprng_generate(phprng_ctx *c, const phprng_request *reqs, uint64_t nreq, uint32_t *out_c32,
                                         uint64_t *out_c64, double *out_r, uint64_t capacity, void *stream,
                                         int mode) {
  if (!c) return PHPRNG_E_INVALID;
  if (mode != PHPRNG_MODE_PERSISTENT && mode != PHPRNG_MODE_PLAIN) return c->fail(PHPRNG_E_INVALID, "bad mode");
  if (nreq == 0) return PHPRNG_OK;
  (void)hipSetDevice(c->device);
  bool has64 = false;
  std::vector<std::pair<uint32_t, uint64_t>> moves;
  phprng_ctx::Slot *slot = nullptr;
  phprng_status st = prepare_requests(c, reqs, nreq, capacity, &slot, &has64, &moves);
  if (st != PHPRNG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const phprng_tuning &T = c->tuning;
  uint32_t tpc = mode == PHPRNG_MODE_PLAIN ? 1u : (uint32_t)T.tiles_per_chunk;
  // Upper bound on the tiles of the batch (a request touches at most
  // count / 2048 + 2 tiles, one more at a skip-period boundary).
  uint64_t tiles = 0;
  for (uint64_t i = 0; i < nreq; ++i)
    tiles += slot->h_req[i].count ? slot->h_req[i].count / kTile + 3 : 0;
  const uint64_t waves = (uint64_t)c->num_cus * T.blocks_per_cu * (T.block_threads / 64);
  // Small batches: shrink the chunk so that every resident wave gets work.
  while (tpc > 1 && tiles < 4 * waves * tpc) tpc >>= 1;
  // the plan reads the request list from the slot's pinned buffer directly
  hipError_t e = launch_plan(c->d_inst, slot->h_req_dev, slot->d_req, nreq, slot->d_gbase, slot->d_hdr, tpc, s);
  if (e != hipSuccess) return c->hip_fail(e, "plan");
  GenArgs A = make_args(c, slot->d_req, slot->d_gbase, slot->d_hdr, nreq, out_c32, out_c64, out_r, tpc);
  if ((e = hipEventRecord(slot->ev0, s)) != hipSuccess) return c->hip_fail(e, "event");
  if (mode == PHPRNG_MODE_PERSISTENT) {
    // no more blocks than the batch can keep busy
    const uint64_t wpb = (uint64_t)T.block_threads / 64;
    const uint64_t need = (tiles + tpc - 1) / tpc;
    const unsigned grid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)c->num_cus * T.blocks_per_cu, (need + wpb - 1) / wpb));
    e = launch_persistent(A, grid, T.block_threads, T.unroll, has64, s);
    if (e != hipSuccess) return c->hip_fail(e, "persistent launch");
  } else {
    for (uint64_t i = 0; i < nreq; ++i) {
      const HostReq &r = slot->h_req[i];
      const unsigned grid = r.count ? (unsigned)(r.count / kTile + 3) : 0u;
      e = launch_plain(A, i, grid, T.unroll, c->inst[r.inst].width == 64, s);
      if (e != hipSuccess) return c->hip_fail(e, "plain launch");
    }
  }
  if ((e = hipEventRecord(slot->ev1, s)) != hipSuccess) return c->hip_fail(e, "event");
  if ((e = hipEventRecord(slot->done, s)) != hipSuccess) return c->hip_fail(e, "event");
  slot->busy = true;
  c->last_timed = c->cur_slot;
  for (auto &mv : moves) c->inst[mv.first].x = mv.second;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_last_kernel_ms(phprng_ctx *c, double *ms) {
  if (!c || !ms) return PHPRNG_E_INVALID;
  if (c->last_timed < 0) return c->fail(PHPRNG_E_INVALID, "no timed launch yet");
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
  const HostInst &h = c->inst[id];
  uint64_t m, s;
  c->state_at(h, h.x, &m, &s);
  Mont64 M(h.n);
  out->m = m;
  out->s = s;
  out->c = M.powmod(m, h.e);
  out->k = (uint64_t)((int64_t)h.x - h.kofs);
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_position(phprng_ctx *c, uint32_t id, uint64_t *k) {
  if (!c || !k || id >= c->inst.size()) return PHPRNG_E_INVALID;
  const HostInst &h = c->inst[id];
  *k = (uint64_t)((int64_t)h.x - h.kofs);
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_jump(phprng_ctx *c, uint32_t id, int64_t delta) {
  if (!c || id >= c->inst.size()) return PHPRNG_E_INVALID;
  HostInst &h = c->inst[id];
  const uint64_t k = (uint64_t)((int64_t)h.x - h.kofs);
  if (delta < 0) {
    const uint64_t d = (uint64_t)(-(delta + 1)) + 1;
    if (d > k || d > h.x) return c->fail(PHPRNG_E_RANGE, "jump before position 0");
    h.x -= d;
  } else {
    const uint64_t d = (uint64_t)delta;
    if (d > c->max_index(h) - h.x) return c->fail(PHPRNG_E_RANGE, "jump beyond range");
    h.x += d;
  }
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_set_state(phprng_ctx *c, uint32_t id, const phprng_state *st) {
  if (!c || !st || id >= c->inst.size()) return PHPRNG_E_INVALID;
  HostInst &h = c->inst[id];
  if (h.sched == kSchedConstant) {
    if (st->m >= h.n || st->s != h.b) return c->fail(PHPRNG_E_INVALID, "bad state for a constant skip");
    Mont64 M(h.n);
    HostInst tmp = h;
    tmp.mbase = M.sub(st->m, M.mulmod(st->k % h.n, h.b));
    InstRec rec = c->make_record(tmp);
    (void)hipSetDevice(c->device);
    hipError_t e = hipMemcpy(c->d_inst + id, &rec, sizeof rec, hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "instance upload");
    h.mbase = tmp.mbase;
    h.x = st->k;
    h.kofs = 0;
    return PHPRNG_OK;
  }
  const SkipGroup &G = group(h.width);
  if (st->m >= h.n || st->s == 0 || st->s >= G.p) return c->fail(PHPRNG_E_INVALID, "bad state");
  const uint64_t pm1 = G.p - 1;
  const uint64_t t = G.dlog(st->s);
  uint64_t x;
  if (h.width == 32) {
    const uint64_t q = st->k / pm1;
    x = q * pm1 + t;
  } else {
    x = t;
    if (x >= kMaxPos64) return c->fail(PHPRNG_E_RANGE, "skip state beyond the width-64 index range");
  }
  HostInst tmp = h;
  tmp.mbase = 0;
  uint64_t mu, su;
  c->state_at(tmp, x, &mu, &su);
  Mont64 M(h.n);
  const uint64_t mbase = M.sub(st->m, mu);
  tmp.mbase = mbase;
  InstRec rec = c->make_record(tmp);
  (void)hipSetDevice(c->device);
  hipError_t e = hipMemcpy(c->d_inst + id, &rec, sizeof rec, hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "instance upload");
  h.mbase = mbase;
  h.x = x;
  h.kofs = (int64_t)(x - st->k);
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_set_tuning(phprng_ctx *c, const phprng_tuning *t) {
  if (!c || !t) return PHPRNG_E_INVALID;
  phprng_tuning v = c->tuning;
  if (t->block_threads) v.block_threads = t->block_threads;
  if (t->blocks_per_cu) v.blocks_per_cu = t->blocks_per_cu;
  if (t->tiles_per_chunk) v.tiles_per_chunk = t->tiles_per_chunk;
  if (t->unroll) v.unroll = t->unroll;
  if (v.block_threads != 64 && v.block_threads != 128 && v.block_threads != 256 && v.block_threads != 512)
    return c->fail(PHPRNG_E_INVALID, "block_threads");
  if (v.blocks_per_cu < 1 || v.blocks_per_cu > 64) return c->fail(PHPRNG_E_INVALID, "blocks_per_cu");
  if (v.tiles_per_chunk < 1 || v.tiles_per_chunk > 64) return c->fail(PHPRNG_E_INVALID, "tiles_per_chunk");
  if (v.unroll != 1 && v.unroll != 2 && v.unroll != 4) return c->fail(PHPRNG_E_INVALID, "unroll");
  c->tuning = v;
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_get_tuning(phprng_ctx *c, phprng_tuning *t) {
  if (!c || !t) return PHPRNG_E_INVALID;
  *t = c->tuning;
  return PHPRNG_OK;
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
  uint32_t *d_c32 = nullptr;
  uint64_t *d_c64 = nullptr;
  double *d_r = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&d_r, cap * 8)) != hipSuccess) return c->hip_fail(e, "autotune alloc");
  (void)any32;
  (void)any64;
  std::vector<uint64_t> saved(ninst);
  for (uint64_t i = 0; i < ninst; ++i) saved[i] = c->inst[i].x;
  const phprng_tuning orig = c->tuning;
  phprng_status result = PHPRNG_OK;
  // one timed call: median kernel time of `reps` calls of shape t
  auto run = [&](const phprng_tuning &t, int reps) -> double {
    c->tuning = t;
    std::vector<double> v;
    for (int rep = 0; rep < reps && result == PHPRNG_OK; ++rep) {
      for (uint64_t i = 0; i < ninst; ++i) c->inst[i].x = saved[i];
      phprng_status st =
          phprng_generate(c, reqs.data(), ninst, d_c32, d_c64, d_r, cap, nullptr, PHPRNG_MODE_PERSISTENT);
      double ms = 0;
      if (st == PHPRNG_OK) st = phprng_last_kernel_ms(c, &ms);
      if (st != PHPRNG_OK) result = st;
      v.push_back(ms);
    }
    if (v.empty()) return 1e30;
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
  };
  // bring the clocks up before timing anything
  auto t0 = std::chrono::steady_clock::now();
  while (result == PHPRNG_OK && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(300)) run(orig, 1);
  phprng_tuning bestT = orig;
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
  for (uint64_t i = 0; i < ninst; ++i) c->inst[i].x = saved[i];
  (void)hipFree(d_r);
  c->tuning = result == PHPRNG_OK ? bestT : orig;
  if (best) *best = c->tuning;
  return result;
}

// ---------------------------------------------------------------------------
// captured repeat draws
// ---------------------------------------------------------------------------

extern "C" phprng_status phprng_graph_create(phprng_ctx *c, const phprng_request *reqs, uint64_t nreq,
                                             uint32_t *out_c32, uint64_t *out_c64, double *out_r, uint64_t capacity,
                                             void *stream, phprng_graph **graph) {
  if (!c || !graph || nreq == 0) return PHPRNG_E_INVALID;
  *graph = nullptr;
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
  bool has64 = false;
  std::vector<std::pair<uint32_t, uint64_t>> moves;
  phprng_ctx::Slot *slot = nullptr;
  phprng_status st = prepare_requests(c, reqs, nreq, capacity, &slot, &has64, &moves);
  if (st != PHPRNG_OK) return st;
  // every launch advances each instance by its count: the first launch starts
  // at the current positions (prepare_requests recorded them in h_req)
  std::unique_ptr<phprng_graph> g(new (std::nothrow) phprng_graph);
  if (!g) return PHPRNG_E_NOMEM;
  g->ctx = c;
  hipError_t e;
  if ((e = hipMalloc(&g->d_src, nreq * sizeof(HostReq))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMalloc(&g->d_req, nreq * sizeof(ReqRec))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMalloc(&g->d_gbase, (nreq + kPlanGroup - 1) / kPlanGroup * sizeof(uint64_t))) != hipSuccess)
    return c->hip_fail(e, "graph alloc");
  if ((e = hipMalloc(&g->d_hdr, sizeof(PlanHdr))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMemset(g->d_hdr, 0, sizeof(PlanHdr))) != hipSuccess) return c->hip_fail(e, "graph alloc");
  if ((e = hipMemcpy(g->d_src, c->h_req, nreq * sizeof(HostReq), hipMemcpyHostToDevice)) != hipSuccess)
    return c->hip_fail(e, "graph upload");
  for (uint64_t i = 0; i < nreq; ++i) {
    g->inst.push_back(c->h_req[i].inst);
    g->count.push_back(c->h_req[i].count);
  }
  hipStream_t cap_stream;
  if ((e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking)) != hipSuccess) return c->hip_fail(e, "stream");
  const phprng_tuning &T = c->tuning;
  GenArgs A = make_args(c, g->d_req, g->d_gbase, g->d_hdr, nreq, out_c32, out_c64, out_r,
                        (uint32_t)T.tiles_per_chunk);
  e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess)
    e = launch_plan(c->d_inst, g->d_src, g->d_req, nreq, g->d_gbase, g->d_hdr, A.tiles_per_chunk, cap_stream);
  if (e == hipSuccess)
    e = launch_persistent(A, (unsigned)(c->num_cus * T.blocks_per_cu), T.block_threads, T.unroll, has64, cap_stream);
  if (e == hipSuccess) e = launch_advance(g->d_src, nreq, cap_stream);
  hipError_t e2 = hipStreamEndCapture(cap_stream, &g->graph);
  (void)hipStreamDestroy(cap_stream);
  if (e != hipSuccess || e2 != hipSuccess) return c->hip_fail(e != hipSuccess ? e : e2, "graph capture");
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return c->hip_fail(e, "graph instantiate");
  (void)stream;
  *graph = g.release();
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_graph_launch(phprng_graph *g, void *stream) {
  if (!g || !g->ctx) return PHPRNG_E_INVALID;
  phprng_ctx *c = g->ctx;
  (void)hipSetDevice(c->device);
  // range check before launching: each instance advances by its count
  for (size_t i = 0; i < g->inst.size(); ++i) {
    const HostInst &h = c->inst[g->inst[i]];
    if (g->count[i] > c->max_index(h) - h.x) return c->fail(PHPRNG_E_RANGE, "graph launch beyond range");
  }
  hipStream_t s = (hipStream_t)stream;
  phprng_ctx::Slot *slot = nullptr;
  phprng_status st = c->take_slot(1, &slot);
  if (st != PHPRNG_OK) return st;
  hipError_t e;
  if ((e = hipEventRecord(slot->ev0, s)) != hipSuccess) return c->hip_fail(e, "event");
  if ((e = hipGraphLaunch(g->exec, s)) != hipSuccess) return c->hip_fail(e, "graph launch");
  if ((e = hipEventRecord(slot->ev1, s)) != hipSuccess) return c->hip_fail(e, "event");
  if ((e = hipEventRecord(slot->done, s)) != hipSuccess) return c->hip_fail(e, "event");
  slot->busy = true;
  c->last_timed = c->cur_slot;
  for (size_t i = 0; i < g->inst.size(); ++i) c->inst[g->inst[i]].x += g->count[i];
  return PHPRNG_OK;
}

extern "C" phprng_status phprng_graph_destroy(phprng_graph *g) {
  if (!g) return PHPRNG_E_INVALID;
  if (g->ctx) (void)hipSetDevice(g->ctx->device);
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  (void)hipFree(g->d_src);
  (void)hipFree(g->d_req);
  (void)hipFree(g->d_gbase);
  (void)hipFree(g->d_hdr);
  delete g;
  return PHPRNG_OK;
}
