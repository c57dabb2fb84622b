// Host side of the statistical battery (the chi-square tests of the paper's
// Tests section): device histograms, the exact category laws, chi-square
// P-values, and the interstream interleave.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "battery.hpp"
#include "stats.hpp"
#include "phprng.h"

using namespace phprng::bat;
namespace ph = phprng::ph;

namespace {

constexpr int kKernelClasses = 6;    // hist, collision, runs, fft pass 1, fft pass 2, hist count + add
constexpr uint64_t kChunkBlocks = 128;  // blocks per inner pass (scratch: 1 GB of transform rows)

const uint32_t kCats[PHPRNG_TEST_COUNT] = {kFreqBins, kCells2, kCells3, kCells4, kCells5,
                                           kPokerCats, kCollCats, kRunsCats, kFourierCats};

// --- exact category laws ----------------------------------------------------

void poker_law(double *p) {
  // hands of five digits 0..9: all different, one pair, two pairs, three of a
  // kind, full house, four of a kind, five of a kind (counted among 10^5)
  const double ways[kPokerCats] = {10.0 * 9 * 8 * 7 * 6, 10.0 * 10 * 9 * 8 * 7, 15.0 * 10 * 9 * 8,
                                   10.0 * 10 * 9 * 8,     10.0 * 10 * 9,         5.0 * 10 * 9, 10.0};
  for (uint32_t i = 0; i < kPokerCats; ++i) p[i] = ways[i] / 1e5;
}

// Law of the number of collisions when kCollBalls balls fall into kCollUrns
// urns: after i balls with c collisions, ball i+1 hits one of the i - c
// occupied urns with probability (i - c) / urns.
void collision_law(double *p) {
  const int cmax = 600;
  std::vector<double> q(cmax + 2, 0.0), nq(cmax + 2);
  q[0] = 1.0;
  for (uint32_t i = 0; i < kCollBalls; ++i) {
    for (int c = 0; c <= cmax + 1; ++c) {
      const double occ = (double)i - c;
      const double hit = occ > 0 ? occ / kCollUrns : 0.0;
      nq[c] = q[c] * (1.0 - hit);
      if (c > 0) {
        const double pocc = (double)i - (c - 1);
        nq[c] += q[c - 1] * (pocc > 0 ? pocc / kCollUrns : 0.0);
      }
    }
    q.swap(nq);
  }
  double lo = 0, below_hi = 0;
  for (uint32_t c = 0; c <= kCollLo; ++c) lo += q[c];
  for (uint32_t c = 0; c < kCollHi; ++c) below_hi += q[c];
  p[0] = lo;
  for (uint32_t c = kCollLo + 1; c < kCollHi; ++c) p[c - kCollLo] = q[c];
  p[kCollCats - 1] = 1.0 - below_hi;
}

// Interior runs of length L in a block of M fair bits: (M - 1 - L) 2^-(L+1)
// expected; lengths 1..20 and the tail >= 21, normalised to a law.
void runs_law(double *p) {
  const double m = kBlock;
  double w[kRunsCats], sum = 0;
  for (uint32_t L = 1; L <= kRunsMax; ++L) w[L - 1] = (m - 1 - L) * std::ldexp(1.0, -(int)(L + 1));
  double tail = 0;
  for (uint32_t L = kRunsMax + 1; L + 1 < kBlock && L < 1100; ++L) tail += (m - 1 - L) * std::ldexp(1.0, -(int)(L + 1));
  w[kRunsCats - 1] = tail;
  for (uint32_t i = 0; i < kRunsCats; ++i) sum += w[i];
  for (uint32_t i = 0; i < kRunsCats; ++i) p[i] = w[i] / sum;
}

double normal_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Standard normal mass of bin u (covering [u/8, (u+1)/8) standard deviations)
// for u = -32 .. 31, plus the two tails beyond 4.
void fourier_law(double *p) {
  p[0] = normal_cdf(-kFourierHalf / 8.0);
  for (int u = -kFourierHalf; u < kFourierHalf; ++u) {
    const double m = u < 0 ? normal_cdf((u + 1) / 8.0) - normal_cdf(u / 8.0)
                           : normal_cdf(-u / 8.0) - normal_cdf(-(u + 1) / 8.0);
    p[u + kFourierHalf + 1] = m;
  }
  p[kFourierCats - 1] = p[0];
}

struct Pending {
  int cls;
  hipEvent_t a, b;
};

}  // namespace

struct phprng_battery {
  int device = 0;
  unsigned long long *d_hist = nullptr;  // all histograms, one allocation
  // partitioned histograms of the frequency and serial tests
  ph::PartSet parts{};
  BatteryParts bparts{};
  uint16_t *d_pdata = nullptr;
  uint32_t *d_pfill = nullptr, *d_pncell = nullptr, *d_pslices = nullptr;
  unsigned long long **d_phist = nullptr;
  unsigned long long *d_cat[PHPRNG_TEST_COUNT] = {};
  uint64_t *d_bits = nullptr;
  double2 *d_y = nullptr;
  double2 *d_tw = nullptr;  // w1024 | fineN | fineM
  double *d_probs = nullptr;  // poker | collision | runs | fourier
  Chi2Job *d_jobs = nullptr;
  double *d_chi2 = nullptr;
  unsigned long long *d_total = nullptr;
  unsigned long long *d_discard = nullptr;  // Fourier category replicas of phprng_battery_fourier calls
  // per-workgroup replicas [kRep][categories] of the small histograms
  unsigned long long *d_rep = nullptr;
  unsigned long long *rep[PHPRNG_TEST_COUNT] = {};
  Twiddles tw{};
  double fourier_scale = 0;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  double ms[kKernelClasses] = {};
  uint64_t launches[kKernelClasses] = {};
  std::string err;
};

namespace {

phprng_status fail(phprng_battery *b, phprng_status st, const char *fmt, ...) {
  if (b) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
  }
  return st;
}

phprng_status hip_fail(phprng_battery *b, hipError_t e, const char *what) {
  return fail(b, PHPRNG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

hipEvent_t take_event(phprng_battery *b) {
  if (!b->free_events.empty()) {
    hipEvent_t e = b->free_events.back();
    b->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold finished event pairs into the per-class totals; with `wait`, wait for all.
void resolve(phprng_battery *b, bool wait) {
  size_t keep = 0;
  for (size_t i = 0; i < b->pending.size(); ++i) {
    Pending &p = b->pending[i];
    bool done = wait ? hipEventSynchronize(p.b) == hipSuccess : hipEventQuery(p.b) == hipSuccess;
    if (done) {
      float t = 0;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        b->ms[p.cls] += t;
        b->launches[p.cls] += 1;
      }
      b->free_events.push_back(p.a);
      b->free_events.push_back(p.b);
    } else {
      b->pending[keep++] = p;
    }
  }
  b->pending.resize(keep);
}

template <class F>
phprng_status timed(phprng_battery *b, int cls, hipStream_t st, const char *what, F launch) {
  hipEvent_t a = take_event(b), c = take_event(b);
  if (a) (void)hipEventRecord(a, st);
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(b, e, what);
  if (a && c && hipEventRecord(c, st) == hipSuccess) {
    b->pending.push_back({cls, a, c});
  } else {
    if (a) b->free_events.push_back(a);
    if (c) b->free_events.push_back(c);
  }
  if (b->pending.size() > 1024) resolve(b, false);
  return PHPRNG_OK;
}

phprng_status check_blocks(phprng_battery *b, const double *r, uint64_t count) {
  if (!b) return PHPRNG_E_INVALID;
  if (count % kBlock) return fail(b, PHPRNG_E_INVALID, "count %llu is not a multiple of 2^20", (unsigned long long)count);
  if (count && (!r || (reinterpret_cast<uintptr_t>(r) & 15)))
    return fail(b, PHPRNG_E_INVALID, "uniforms must be a 16-byte aligned device array");
  return PHPRNG_OK;
}

}  // namespace

extern "C" {

phprng_status phprng_battery_create(phprng_battery **out, int device) {
  if (!out) return PHPRNG_E_INVALID;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return PHPRNG_E_DEVICE;
  auto *b = new (std::nothrow) phprng_battery;
  if (!b) return PHPRNG_E_NOMEM;
  b->device = device;
  uint64_t total = 0;
  for (int t = 0; t < PHPRNG_TEST_COUNT; ++t) total += kCats[t];
  const uint64_t nprob = kPokerCats + kCollCats + kRunsCats + kFourierCats;
  bool ok = hipMalloc(&b->d_hist, total * sizeof(unsigned long long)) == hipSuccess &&
            hipMalloc(&b->d_bits, kChunkBlocks * kWordsPerBlock * sizeof(uint64_t)) == hipSuccess &&
            hipMalloc(&b->d_y, kChunkBlocks * (uint64_t)kFftN * sizeof(double2)) == hipSuccess &&
            hipMalloc(&b->d_tw, 3 * 1024 * sizeof(double2)) == hipSuccess &&
            hipMalloc(&b->d_probs, nprob * sizeof(double)) == hipSuccess &&
            hipMalloc(&b->d_jobs, PHPRNG_TEST_COUNT * sizeof(Chi2Job)) == hipSuccess &&
            hipMalloc(&b->d_chi2, PHPRNG_TEST_COUNT * sizeof(double)) == hipSuccess &&
            hipMalloc(&b->d_total, PHPRNG_TEST_COUNT * sizeof(unsigned long long)) == hipSuccess &&
            hipMalloc(&b->d_discard, kRep * kFourierCats * sizeof(unsigned long long)) == hipSuccess &&
            hipMalloc(&b->d_rep, kRep * nprob * sizeof(unsigned long long)) == hipSuccess;
  if (!ok) {
    phprng_battery_destroy(b);
    return PHPRNG_E_NOMEM;
  }
  uint64_t off = 0;
  for (int t = 0; t < PHPRNG_TEST_COUNT; ++t) {
    b->d_cat[t] = b->d_hist + off;
    off += kCats[t];
  }
  b->rep[PHPRNG_TEST_POKER] = b->d_rep;
  b->rep[PHPRNG_TEST_COLLISION] = b->d_rep + kRep * kPokerCats;
  b->rep[PHPRNG_TEST_RUNS] = b->d_rep + kRep * (kPokerCats + kCollCats);
  b->rep[PHPRNG_TEST_FOURIER] = b->d_rep + kRep * (kPokerCats + kCollCats + kRunsCats);
  // partition space: the frequency and serial tests, 2^15 cells per partition
  std::vector<unsigned long long *> phist;
  std::vector<uint32_t> pncell;
  uint32_t npart = 0;
  for (int t = 0; t < kPartTests; ++t) {
    const uint32_t cells = kCats[PHPRNG_TEST_FREQUENCY + t];
    const uint32_t np = (cells + ph::kPartCells - 1) / ph::kPartCells;
    b->bparts.p0[t] = npart;
    for (uint32_t q = 0; q < np; ++q) {
      phist.push_back(b->d_cat[PHPRNG_TEST_FREQUENCY + t] + (uint64_t)q * ph::kPartCells);
      pncell.push_back(std::min<uint32_t>(ph::kPartCells, cells - q * ph::kPartCells));
    }
    npart += np;
  }
  if (npart > kMaxParts) {
    phprng_battery_destroy(b);
    return PHPRNG_E_INVALID;
  }
  // bucket room per sub-bucket and chunk: the frequency test's share of a
  // partition (2^22 keys for a chunk) over the sub-buckets, with a margin;
  // any surplus goes to atomics
  const uint32_t nsub = 8;
  const uint32_t cap = (uint32_t)(kChunkBlocks * kBlock / 32 / nsub * 5 / 4 + 4096) & ~7u;
  const uint32_t nslice = 2;
  static_assert((uint64_t)kMaxParts * 8 * ((kChunkBlocks * kBlock / 32 / 8 * 5 / 4 + 4096) & ~7u) < (1ull << 32),
                "32-bit bucket indexing");
  ok = hipMalloc(&b->d_pdata, (uint64_t)npart * nsub * cap * sizeof(uint16_t)) == hipSuccess &&
       hipMalloc(&b->d_pfill, npart * nsub * sizeof(uint32_t)) == hipSuccess &&
       hipMalloc(&b->d_pncell, npart * sizeof(uint32_t)) == hipSuccess &&
       hipMalloc(&b->d_pslices, (uint64_t)npart * nslice * ph::kPartCells * sizeof(uint32_t)) == hipSuccess &&
       hipMalloc(&b->d_phist, npart * sizeof(unsigned long long *)) == hipSuccess;
  if (!ok || hipMemcpy(b->d_phist, phist.data(), npart * sizeof(void *), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_pncell, pncell.data(), npart * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->d_pfill, 0, npart * nsub * sizeof(uint32_t)) != hipSuccess) {
    phprng_battery_destroy(b);
    return PHPRNG_E_NOMEM;
  }
  b->parts = ph::PartSet{b->d_pdata, b->d_pfill, b->d_phist, b->d_pncell, b->d_pslices, npart, cap, nslice, nsub};
  // roots of unity in extended precision, then rounded
  std::vector<double2> tw(3 * 1024);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int t = 0; t < 1024; ++t) {
    const long double a0 = two_pi * t / 1024.0L, a1 = two_pi * t / 524288.0L, a2 = two_pi * t / 1048576.0L;
    tw[t] = make_double2((double)cosl(a0), (double)sinl(a0));
    tw[1024 + t] = make_double2((double)cosl(a1), (double)sinl(a1));
    tw[2048 + t] = make_double2((double)cosl(a2), (double)sinl(a2));
  }
  std::vector<double> probs(nprob);
  poker_law(probs.data());
  collision_law(probs.data() + kPokerCats);
  runs_law(probs.data() + kPokerCats + kCollCats);
  fourier_law(probs.data() + kPokerCats + kCollCats + kRunsCats);
  Chi2Job jobs[PHPRNG_TEST_COUNT];
  for (int t = 0; t < PHPRNG_TEST_COUNT; ++t) jobs[t] = Chi2Job{b->d_cat[t], nullptr, kCats[t], 0};
  jobs[PHPRNG_TEST_POKER].probs = b->d_probs;
  jobs[PHPRNG_TEST_COLLISION].probs = b->d_probs + kPokerCats;
  jobs[PHPRNG_TEST_RUNS].probs = b->d_probs + kPokerCats + kCollCats;
  jobs[PHPRNG_TEST_FOURIER].probs = b->d_probs + kPokerCats + kCollCats + kRunsCats;
  if (hipMemcpy(b->d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_probs, probs.data(), nprob * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_jobs, jobs, sizeof jobs, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->d_hist, 0, total * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(b->d_rep, 0, kRep * nprob * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(b->d_discard, 0, kRep * kFourierCats * sizeof(unsigned long long)) != hipSuccess) {
    phprng_battery_destroy(b);
    return PHPRNG_E_DEVICE;
  }
  b->tw = Twiddles{b->d_tw, b->d_tw + 1024, b->d_tw + 2048};
  b->fourier_scale = 8.0 * std::sqrt(24.0);
  *out = b;
  return PHPRNG_OK;
}

phprng_status phprng_battery_destroy(phprng_battery *b) {
  if (!b) return PHPRNG_E_INVALID;
  (void)hipSetDevice(b->device);
  resolve(b, true);
  for (hipEvent_t e : b->free_events) (void)hipEventDestroy(e);
  void *bufs[] = {b->d_hist,  b->d_bits,  b->d_y,      b->d_tw,     b->d_probs,   b->d_jobs,   b->d_chi2,
                  b->d_total, b->d_discard, b->d_pdata, b->d_pfill, b->d_pncell, b->d_pslices, b->d_phist,
                  b->d_rep};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  delete b;
  return PHPRNG_OK;
}

const char *phprng_battery_last_error(const phprng_battery *b) { return b ? b->err.c_str() : ""; }

phprng_status phprng_battery_reset(phprng_battery *b, void *stream) {
  if (!b) return PHPRNG_E_INVALID;
  (void)hipSetDevice(b->device);
  uint64_t total = 0;
  for (int t = 0; t < PHPRNG_TEST_COUNT; ++t) total += kCats[t];
  const uint64_t nprob = kPokerCats + kCollCats + kRunsCats + kFourierCats;
  hipError_t e = hipMemsetAsync(b->d_hist, 0, total * sizeof(unsigned long long), (hipStream_t)stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->d_rep, 0, kRep * nprob * sizeof(unsigned long long), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(b, e, "reset");
  resolve(b, true);
  for (int i = 0; i < kKernelClasses; ++i) {
    b->ms[i] = 0;
    b->launches[i] = 0;
  }
  return PHPRNG_OK;
}

phprng_status phprng_battery_accumulate(phprng_battery *b, const double *r, uint64_t count, void *stream) {
  phprng_status s = check_blocks(b, r, count);
  if (s != PHPRNG_OK) return s;
  (void)hipSetDevice(b->device);
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nblocks = count / kBlock;
  for (uint64_t b0 = 0; b0 < nblocks; b0 += kChunkBlocks) {
    const uint64_t nb = nblocks - b0 < kChunkBlocks ? nblocks - b0 : kChunkBlocks;
    const double *src = r + b0 * kBlock;
    if ((s = timed(b, 0, st, "hist kernel",
                   [&] {
                     return launch_hist(src, nb, b->parts, b->bparts, b->rep[PHPRNG_TEST_POKER], b->d_bits, st);
                   })) != PHPRNG_OK ||
        (s = timed(b, 1, st, "collision kernel",
                   [&] { return launch_collision(src, nb, b->rep[PHPRNG_TEST_COLLISION], st); })) != PHPRNG_OK ||
        (s = timed(b, 2, st, "runs kernel",
                   [&] { return launch_runs(b->d_bits, nb, b->rep[PHPRNG_TEST_RUNS], st); })) != PHPRNG_OK ||
        (s = timed(b, 3, st, "fft pass 1", [&] { return launch_fft_pass1(src, nb, b->d_y, b->tw, st); })) != PHPRNG_OK ||
        (s = timed(b, 4, st, "fft pass 2", [&] {
           return launch_fft_pass2(b->d_y, nb, b->rep[PHPRNG_TEST_FOURIER], nullptr, b->tw, b->fourier_scale, st);
         })) != PHPRNG_OK ||
        (s = timed(b, 5, st, "histogram count", [&] {
           hipError_t e = ph::launch_count(b->parts, st);
           return e == hipSuccess ? ph::launch_add(b->parts, st) : e;
         })) != PHPRNG_OK)
      return s;
  }
  // the small histograms' replicas into their histograms
  if (nblocks) {
    for (int t : {PHPRNG_TEST_POKER, PHPRNG_TEST_COLLISION, PHPRNG_TEST_RUNS, PHPRNG_TEST_FOURIER}) {
      hipError_t e = launch_fold(b->rep[t], b->d_cat[t], kCats[t], st);
      if (e != hipSuccess) return hip_fail(b, e, "fold");
    }
  }
  return PHPRNG_OK;
}

phprng_status phprng_battery_fourier(phprng_battery *b, const double *r, uint64_t count, double *coef, void *stream) {
  phprng_status s = check_blocks(b, r, count);
  if (s != PHPRNG_OK) return s;
  if (count && !coef) return fail(b, PHPRNG_E_INVALID, "null coefficient array");
  (void)hipSetDevice(b->device);
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nblocks = count / kBlock;
  for (uint64_t b0 = 0; b0 < nblocks; b0 += kChunkBlocks) {
    const uint64_t nb = nblocks - b0 < kChunkBlocks ? nblocks - b0 : kChunkBlocks;
    hipError_t e = launch_fft_pass1(r + b0 * kBlock, nb, b->d_y, b->tw, st);
    if (e == hipSuccess)
      e = launch_fft_pass2(b->d_y, nb, b->d_discard, coef + b0 * kBlock, b->tw, b->fourier_scale, st);
    if (e != hipSuccess) return hip_fail(b, e, "fourier");
  }
  return PHPRNG_OK;
}

phprng_status phprng_battery_report(phprng_battery *b, phprng_test_result *out, void *stream) {
  if (!b || !out) return PHPRNG_E_INVALID;
  (void)hipSetDevice(b->device);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_chi2(b->d_jobs, PHPRNG_TEST_COUNT, b->d_chi2, b->d_total, st);
  double chi2[PHPRNG_TEST_COUNT];
  unsigned long long tot[PHPRNG_TEST_COUNT];
  if (e == hipSuccess) e = hipMemcpyAsync(chi2, b->d_chi2, sizeof chi2, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(tot, b->d_total, sizeof tot, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(b, e, "report");
  for (int t = 0; t < PHPRNG_TEST_COUNT; ++t) {
    out[t].chi2 = chi2[t];
    out[t].samples = tot[t];
    out[t].dof = kCats[t] - 1;
    double P = 0, Q = 0;
    if (tot[t]) {
      phprng::gamma_pq(0.5 * (double)out[t].dof, 0.5 * chi2[t], &P, &Q);
      out[t].p_value = P < Q ? P : Q;
    } else {
      out[t].p_value = 0;
      out[t].chi2 = 0;
    }
  }
  return PHPRNG_OK;
}

phprng_status phprng_battery_counts(phprng_battery *b, int test, uint64_t *out, uint64_t capacity, uint64_t *ncat,
                                    void *stream) {
  if (!b || test < 0 || test >= PHPRNG_TEST_COUNT) return PHPRNG_E_INVALID;
  if (ncat) *ncat = kCats[test];
  if (!out) return PHPRNG_OK;
  if (capacity < kCats[test]) return fail(b, PHPRNG_E_RANGE, "capacity below %u", kCats[test]);
  (void)hipSetDevice(b->device);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(out, b->d_cat[test], kCats[test] * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? PHPRNG_OK : hip_fail(b, e, "counts");
}

phprng_status phprng_battery_probabilities(int test, double *out, uint64_t capacity, uint64_t *ncat) {
  if (test < 0 || test >= PHPRNG_TEST_COUNT) return PHPRNG_E_INVALID;
  if (ncat) *ncat = kCats[test];
  if (!out) return PHPRNG_OK;
  if (capacity < kCats[test]) return PHPRNG_E_RANGE;
  switch (test) {
    case PHPRNG_TEST_POKER: poker_law(out); break;
    case PHPRNG_TEST_COLLISION: collision_law(out); break;
    case PHPRNG_TEST_RUNS: runs_law(out); break;
    case PHPRNG_TEST_FOURIER: fourier_law(out); break;
    default:
      for (uint32_t i = 0; i < kCats[test]; ++i) out[i] = 1.0 / kCats[test];
  }
  return PHPRNG_OK;
}

phprng_status phprng_battery_timing(phprng_battery *b, double *ms, uint64_t *launches) {
  if (!b) return PHPRNG_E_INVALID;
  (void)hipSetDevice(b->device);
  resolve(b, true);
  for (int i = 0; i < kKernelClasses; ++i) {
    if (ms) ms[i] = b->ms[i];
    if (launches) launches[i] = b->launches[i];
  }
  return PHPRNG_OK;
}

phprng_status phprng_chi2_pvalue(double chi2, double dof, double *p) {
  if (!p || !(dof > 0) || !(chi2 >= 0)) return PHPRNG_E_INVALID;
  double P = 0, Q = 0;
  phprng::gamma_pq(0.5 * dof, 0.5 * chi2, &P, &Q);
  *p = P < Q ? P : Q;
  return PHPRNG_OK;
}

phprng_status phprng_interleave(const double *in, double *out, uint64_t nstreams, uint64_t length, void *stream) {
  if (nstreams == 0 || length == 0) return PHPRNG_OK;
  if (!in || !out || in == out) return PHPRNG_E_INVALID;
  if ((nstreams + 63) / 64 > 65535 || (length + 63) / 64 > 0x7fffffffull) return PHPRNG_E_RANGE;
  return launch_interleave(in, out, nstreams, length, (hipStream_t)stream) == hipSuccess ? PHPRNG_OK
                                                                                         : PHPRNG_E_DEVICE;
}

}  // extern "C"
