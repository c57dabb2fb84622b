// gfx950 kernels for the Pohlig-Hellman parameter-split generator:
//   - skip-prefix table segments (eq. (7b) building blocks),
//   - the request planner (tile/chunk bookkeeping for a batch),
//   - batched generation (algorithm (9)) as a persistent work-stealing grid
//     or as one plain grid per request,
//   - the position advance used by captured repeat draws.
//
// Work decomposition.  A tile is 2048 consecutive draws of one instance whose
// starting state index is a multiple of 2048 within the skip period (the
// universal table holds the skip-prefix sum U and the skip a^r there).  One
// wave computes a tile in three passes over its LDS row block:
//   A. lane l steps the skip generator over its run of 32 draws, keeps the
//      skips in LDS and sums them;
//   B. a wave scan of the run sums gives each lane its starting message; the
//      lane accumulates its run's messages into LDS (eq. (3a));
//   C. lanes read the messages back in draw order (lane l takes draws
//      i*64 + l), encrypt (eq. (1)), form R and store both coalesced.
// A chunk is a run of consecutive tiles of one request; a wave carries the
// state from one tile to the next within a chunk.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "arith.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace phprng {

constexpr int kRow = kRun + 1;  // padded LDS row (conflict-free for both access orders)
static_assert((kTilesPerPeriod32 & (kTilesPerPeriod32 - 1)) == 0, "tiles per period is a power of two");
constexpr int kTileShift32 = 20;
static_assert((1ull << kTileShift32) == kTilesPerPeriod32, "tile shift");

// ---------------------------------------------------------------------------
// skip-prefix table segments
// ---------------------------------------------------------------------------

// Segment i: start skip a^{i*stride} and the sum of the next `stride` skips.
__global__ void __launch_bounds__(256) table_segments32(uint64_t nseg, uint64_t *seg_sum, uint32_t *seg_start) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nseg) return;
  uint32_t s = dev::powmod_p31(kA32, i * kTableStride);
  seg_start[i] = s;
  uint64_t sum = 0;
  for (uint64_t j = 0; j < kTableStride; ++j) {
    s = dev::mulmod_p31(kA32, s);
    sum += s;
  }
  seg_sum[i] = sum;
}

__global__ void __launch_bounds__(256) table_segments64(uint64_t nseg, uint64_t *seg_lo, uint64_t *seg_hi,
                                                        uint64_t *seg_start) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nseg) return;
  uint64_t s = dev::powmod_p61(kA64, i * kTableStride);
  seg_start[i] = s;
  uint64_t lo = 0, hi = 0;
  for (uint64_t j = 0; j < kTableStride; ++j) {
    s = dev::mulmod_p61(kA64, s);
    uint64_t t = lo + s;
    hi += (t < lo) ? 1 : 0;
    lo = t;
  }
  seg_lo[i] = lo;
  seg_hi[i] = hi;
}

// ---------------------------------------------------------------------------
// instance seeding on the device
// ---------------------------------------------------------------------------

// flags[i] = 1 when output j0 + i of the seeding stream, read as a candidate
// modulus (lo + x mod 2^w) | 1 of the width's range, is prime.
__global__ void __launch_bounds__(256) seed_prime_flags(uint64_t seed, uint64_t j0, uint64_t count, int width,
                                                        uint8_t *flags) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t x = dev::splitmix64_at(seed, j0 + i);
  bool p;
  if (width == 32) {
    const uint32_t n = (uint32_t)((1ull << 31) + (x & ((1ull << 31) - 1))) | 1u;
    p = dev::is_prime32_dev(n);
  } else {
    const uint64_t n = ((1ull << 62) + (x & ((1ull << 62) - 1))) | 1ull;
    p = dev::is_prime64_dev(n);
  }
  flags[i] = p ? 1 : 0;
}

// Instance records for base-state instances (m_0 = 0, s_0 = 1) of one width:
// the same constants the host computes (Montgomery inverse, R^2, R^e, the
// full-period skip sum times R^2, binary64 n + 1 and its reciprocal).
__global__ void __launch_bounds__(256) build_records(const uint64_t *n_arr, const uint64_t *e_arr, uint64_t count,
                                                     int width, InstRec *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t n = n_arr[i], e = e_arr[i];
  InstRec rec;
  memset(&rec, 0, sizeof rec);
  rec.n = n;
  rec.e = e;
  rec.width = (uint32_t)width;
  int eb = 0;
  for (uint64_t v = e; v; v >>= 1) ++eb;
  rec.ebits = (uint32_t)eb;
  rec.ekind = (e == 3 || e == 5 || e == 9 || e == 17) ? (uint32_t)e : 0u;
  rec.sched = kSchedSkipLcg;
  rec.den = (double)(n + 1);
  if (width == 32) {
    const uint32_t n32 = (uint32_t)n, ninv = dev::inv32(n32);
    const uint32_t one = 0u - n32;
    uint32_t r2 = one;
    for (int k = 0; k < 32; ++k) r2 = dev::addmod32(r2, r2, n32);
    // R^e: the Montgomery power of R (Montgomery form R^2) is R^{e+1}; one more REDC
    const uint32_t re1 = dev::mpow32(r2, e, one, n32, ninv);
    rec.ninv = ninv;
    rec.r2 = r2;
    rec.kcorr = dev::mont32(re1, 1u, n32, ninv);
    // p(p-1)/2 mod n, then times R^2: mont(b, R^3) with R^3 = mont(R^2, R^2)
    const uint64_t full = ((uint64_t)kP32 * ((uint64_t)kP32 - 1)) / 2;
    const uint32_t b = dev::mont32(dev::redc32(full, n32, ninv), r2, n32, ninv);
    rec.br2 = dev::mont32(b, dev::mont32(r2, r2, n32, ninv), n32, ninv);
    rec.rcp = 1.0 / (double)(n + 1);
  } else {
    const uint64_t ninv = dev::inv64(n);
    uint64_t one = 0ull - n;
    while (one >= n) one -= n;
    uint64_t r2 = one;
    for (int k = 0; k < 64; ++k) r2 = dev::addmod64(r2, r2, n);
    const uint64_t re1 = dev::mpow64(r2, e, one, n, ninv);
    rec.ninv = ninv;
    rec.r2 = r2;
    rec.kcorr = dev::mont64(re1, 1ull, n, ninv);
    rec.br2 = 0;
    rec.rcp = 1.0 / rec.den;
  }
  out[i] = rec;
}

// ---------------------------------------------------------------------------
// planner
// ---------------------------------------------------------------------------

// Global tile index of the tile whose draws include the draw made from state
// index x.
__device__ __forceinline__ uint64_t tile_of(uint64_t x, bool w64) {
  if (w64) return x / kTile;
  uint64_t q = x / ((uint64_t)kP32 - 1);
  uint64_t r = x - q * ((uint64_t)kP32 - 1);
  return (q << kTileShift32) | (r / kTile);
}

// Inclusive scan of v over a workgroup of kPlanGroup threads; *total gets the
// sum.  ws: LDS scratch of kPlanGroup / 64 words.  Starts and ends with a barrier.
__device__ __forceinline__ uint64_t plan_scan(uint64_t v, uint64_t *ws, uint64_t *total) {
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  uint64_t incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t u = dev::shfl_up_u64(incl, d);
    if ((int)lane >= d) incl += u;
  }
  if (lane == 63) ws[w] = incl;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (uint32_t j = 0; j < kPlanGroup / 64; ++j) {
    before += j < w ? ws[j] : 0;
    all += ws[j];
  }
  *total = all;
  __syncthreads();
  return before + incl;
}

// One workgroup per kPlanGroup requests.  The host-written requests are read
// with system-scope loads (src is pinned host memory, or device memory for
// graph replays); per request the first tile, tile count and chunk count are
// found, scanned inside the group, and the group's total goes to gbase.  The
// last workgroup to finish turns gbase into exclusive prefixes, stores the
// batch total, and clears the work counter and its own completion counter.
__global__ void __launch_bounds__(kPlanGroup) plan_kernel(const InstRec *inst, const HostReq *src, ReqRec *req,
                                                          uint64_t nreq, uint64_t *gbase, PlanHdr *hdr,
                                                          uint32_t tiles_per_chunk) {
  constexpr uint32_t kWords = sizeof(HostReq) / 8;
  __shared__ uint64_t words[kPlanGroup * kWords];
  __shared__ uint64_t ws[kPlanGroup / 64];
  __shared__ uint32_t last;
  const uint32_t tid = threadIdx.x;
  const uint64_t r0 = (uint64_t)blockIdx.x * kPlanGroup;
  const uint32_t nin = (uint32_t)min((uint64_t)kPlanGroup, nreq - r0);
  // consecutive lanes read consecutive words: whole lines over the bus
  const uint64_t *sw = reinterpret_cast<const uint64_t *>(src + r0);
  for (uint32_t i = tid; i < nin * kWords; i += kPlanGroup)
    words[i] = __hip_atomic_load(sw + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __syncthreads();
  ReqRec R{};
  if (tid < nin) {
    R.k = words[tid * kWords];
    R.count = words[tid * kWords + 1];
    R.out_off = words[tid * kWords + 2];
    R.inst = (uint32_t)words[tid * kWords + 3];
    const InstRec &I = inst[R.inst];
    const bool w64 = I.width == 64 || I.sched == kSchedConstant;  // no skip period to respect
    if (R.count > 0) {
      R.g1 = tile_of(R.k, w64);
      R.ntiles = tile_of(R.k + R.count - 1, w64) - R.g1 + 1;
    }
    R.nchunks = (uint32_t)((R.ntiles + tiles_per_chunk - 1) / tiles_per_chunk);
  }
  uint64_t gtotal;
  const uint64_t incl = plan_scan(R.nchunks, ws, &gtotal);
  if (tid < nin) {
    R.chunk_base = incl - R.nchunks;
    req[r0 + tid] = R;
  }
  if (tid == 0) {
    gbase[blockIdx.x] = gtotal;
    __threadfence();
    last = atomicAdd(&hdr->done, 1u) == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // last workgroup: exclusive scan of the group totals, in place
  const uint32_t ng = gridDim.x;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < ng; base += kPlanGroup) {
    const uint32_t j = base + tid;
    const uint64_t v = j < ng ? __hip_atomic_load(gbase + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    uint64_t rtotal;
    const uint64_t in = plan_scan(v, ws, &rtotal);
    if (j < ng) gbase[j] = carry + in - v;
    carry += rtotal;
  }
  if (tid == 0) {
    hdr->total_chunks = carry;
    hdr->counter = 0;
    hdr->done = 0;
  }
}

// Graph replays: every request continues where it ended.
__global__ void __launch_bounds__(256) advance_kernel(HostReq *req, uint64_t nreq) {
  uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nreq) req[r].k += req[r].count;
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------

// Which outputs a pass writes (bit 0: ciphertexts, bit 1: uniforms).
enum { kOutC = 1, kOutR = 2 };

struct Enc32 {
  uint32_t n, ninv, kc;
  uint64_t e;
  int ebits;
  double den, rcp;
};

// Pass C, width 32: draw t = i*64 + lane of the tile lives at LDS row t / 32,
// column t % 32.  MASKED tiles write only t in [t_lo, t_hi).
template <int UNROLL, int EK, int OUT, bool MASKED>
__device__ __forceinline__ void passC32(const uint32_t *L, uint32_t lane, const Enc32 &K, uint32_t *c32, double *rr,
                                        uint32_t t_lo, uint32_t t_hi) {
  const uint32_t *src = L + (lane >> 5) * kRow + (lane & 31);
  const uint32_t span = t_hi - t_lo;
#pragma unroll UNROLL
  for (int i = 0; i < kRun; ++i) {
    const uint32_t m = src[i * 2 * kRow];
    if (!MASKED || ((uint32_t)i * 64u + lane - t_lo < span)) {
      const uint32_t c = dev::encrypt32<EK>(m, K.n, K.ninv, K.kc, K.e, K.ebits);
      if (OUT & kOutC) c32[i * 64] = c;
      if (OUT & kOutR) rr[i * 64] = dev::uniform32(c, K.den, K.rcp);
    }
  }
}

template <int UNROLL, int EK, bool MASKED>
__device__ __forceinline__ void passC32_out(const uint32_t *L, uint32_t lane, const Enc32 &K, uint32_t *c32,
                                            double *rr, uint32_t t_lo, uint32_t t_hi) {
  if (c32 && rr) passC32<UNROLL, EK, kOutC | kOutR, MASKED>(L, lane, K, c32, rr, t_lo, t_hi);
  else if (rr) passC32<UNROLL, EK, kOutR, MASKED>(L, lane, K, c32, rr, t_lo, t_hi);
  else if (c32) passC32<UNROLL, EK, kOutC, MASKED>(L, lane, K, c32, rr, t_lo, t_hi);
}

template <int UNROLL, bool MASKED>
__device__ __forceinline__ void passC32_e(int ekind, const uint32_t *L, uint32_t lane, const Enc32 &K, uint32_t *c32,
                                          double *rr, uint32_t t_lo, uint32_t t_hi) {
  switch (ekind) {
    case 9: passC32_out<UNROLL, 9, MASKED>(L, lane, K, c32, rr, t_lo, t_hi); break;
    case 17: passC32_out<UNROLL, 17, MASKED>(L, lane, K, c32, rr, t_lo, t_hi); break;
    case 3: passC32_out<UNROLL, 3, MASKED>(L, lane, K, c32, rr, t_lo, t_hi); break;
    case 5: passC32_out<UNROLL, 5, MASKED>(L, lane, K, c32, rr, t_lo, t_hi); break;
    default: passC32_out<UNROLL, 0, MASKED>(L, lane, K, c32, rr, t_lo, t_hi); break;
  }
}

template <int UNROLL>
__device__ void run_chunk32(const GenArgs &A, const InstRec &I, const ReqRec &R, uint64_t chunk, uint32_t *L,
                            uint32_t lane) {
  const uint32_t n = (uint32_t)I.n, ninv = (uint32_t)I.ninv, kc = (uint32_t)I.kcorr, r2 = (uint32_t)I.r2;
  const uint32_t br2 = (uint32_t)I.br2;
  const uint64_t e = I.e;
  const int ebits = (int)I.ebits, ekind = (int)I.ekind;
  const double den = I.den, rcp = I.rcp;
  const uint64_t pm1 = (uint64_t)kP32 - 1;
  const uint32_t lane_mul = A.lanemul->m32[lane];
  const uint32_t one = dev::opaque_one();

  const uint64_t g_begin = R.g1 + chunk * A.tiles_per_chunk;
  const uint64_t g_end = min(g_begin + A.tiles_per_chunk, R.g1 + R.ntiles);
  uint32_t m_t = 0, s_t = 0;
  bool carried = false;
  for (uint64_t g = g_begin; g < g_end; ++g) {
    const uint64_t q = g >> kTileShift32;
    const uint32_t j = (uint32_t)(g & (kTilesPerPeriod32 - 1));
    const uint64_t x0 = q * pm1 + (uint64_t)j * kTile;
    if (!carried || j == 0) {
      // state at x0 from the universal table (eq. (7)):
      // m = mbase + q p(p-1)/2 + U(j*2048) mod n,  s = a^{j*2048} mod p
      const uint64_t u = A.tab.u32[j];
      s_t = A.tab.s32[j];
      uint32_t mu = dev::mont32(dev::redc32(u + I.mbase, n, ninv), r2, n, ninv);
      uint32_t mq = dev::mont32(dev::redc32(q, n, ninv), br2, n, ninv);
      m_t = dev::addmod32(mu, mq, n);
    }
    // ---- pass A: skips of this lane's run, their sum
    uint32_t *row = L + lane * kRow;
    uint32_t s = dev::mulmod_p31(s_t, lane_mul);
    uint64_t sum = 0;
#pragma unroll 8
    for (int i = 0; i < kRun; ++i) {
      s = dev::mulmod_p31(kA32, s);
      row[i] = s;
      sum = dev::acc_u32(sum, s, one);
    }
    // ---- pass B: exclusive wave scan of run sums -> run start message
    uint64_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint64_t v = dev::shfl_up_u64(incl, d);
      if ((int)lane >= d) incl += v;
    }
    uint32_t m = dev::mont32(dev::redc32(incl - sum + m_t, n, ninv), r2, n, ninv);
#pragma unroll 8
    for (int i = 0; i < kRun; ++i) {
      m = dev::addmod32(m, row[i], n);
      row[i] = m;
    }
    // state at the end of the tile (lane 63's last message and skip)
    m_t = (uint32_t)__shfl((int)m, 63, 64);
    s_t = (uint32_t)__shfl((int)s, 63, 64);
    carried = true;
    dev::wave_lds_sync();
    // ---- pass C: encrypt in draw order
    const uint64_t tile_first = x0;  // draw t of this tile comes from state index x0 + t
    const uint64_t req_end = R.k + R.count;  // one past the last state index used
    uint32_t t_lo = R.k > tile_first ? (uint32_t)(R.k - tile_first) : 0u;
    uint64_t hi1 = req_end - tile_first;
    uint64_t hi2 = pm1 - (uint64_t)j * kTile;
    uint64_t hi = min(min(hi1, hi2), (uint64_t)kTile);
    uint32_t t_hi = (uint32_t)hi;
    const int64_t base = (int64_t)R.out_off + (int64_t)(tile_first - R.k) + (int64_t)lane;
    uint32_t *c32 = A.out_c32 ? A.out_c32 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    const Enc32 K{n, ninv, kc, e, ebits, den, rcp};
    if (t_lo == 0 && t_hi == (uint32_t)kTile)
      passC32_e<UNROLL, false>(ekind, L, lane, K, c32, rr, t_lo, t_hi);
    else
      passC32_e<1, true>(ekind, L, lane, K, c32, rr, t_lo, t_hi);
    dev::wave_lds_sync();
  }
}

struct Enc64 {
  uint64_t n, ninv, kc, e;
  int ebits;
  double den, rcp;
};

template <int UNROLL, int EK, int OUT, bool MASKED>
__device__ __forceinline__ void passC64(const uint64_t *L, uint32_t lane, const Enc64 &K, uint64_t *c64, double *rr,
                                        uint32_t t_lo, uint32_t t_hi) {
  const uint64_t *src = L + (lane >> 5) * kRow + (lane & 31);
  const uint32_t span = t_hi - t_lo;
#pragma unroll UNROLL
  for (int i = 0; i < kRun; ++i) {
    const uint64_t m = src[i * 2 * kRow];
    if (!MASKED || ((uint32_t)i * 64u + lane - t_lo < span)) {
      const uint64_t c = dev::encrypt64<EK>(m, K.n, K.ninv, K.kc, K.e, K.ebits);
      if (OUT & kOutC) c64[i * 64] = c;
      if (OUT & kOutR) rr[i * 64] = dev::uniform64(c, K.den, K.rcp);
    }
  }
}

template <int UNROLL, int EK, bool MASKED>
__device__ __forceinline__ void passC64_out(const uint64_t *L, uint32_t lane, const Enc64 &K, uint64_t *c64,
                                            double *rr, uint32_t t_lo, uint32_t t_hi) {
  if (c64 && rr) passC64<UNROLL, EK, kOutC | kOutR, MASKED>(L, lane, K, c64, rr, t_lo, t_hi);
  else if (rr) passC64<UNROLL, EK, kOutR, MASKED>(L, lane, K, c64, rr, t_lo, t_hi);
  else if (c64) passC64<UNROLL, EK, kOutC, MASKED>(L, lane, K, c64, rr, t_lo, t_hi);
}

template <int UNROLL, bool MASKED>
__device__ __forceinline__ void passC64_e(int ekind, const uint64_t *L, uint32_t lane, const Enc64 &K, uint64_t *c64,
                                          double *rr, uint32_t t_lo, uint32_t t_hi) {
  switch (ekind) {
    case 9: passC64_out<UNROLL, 9, MASKED>(L, lane, K, c64, rr, t_lo, t_hi); break;
    case 17: passC64_out<UNROLL, 17, MASKED>(L, lane, K, c64, rr, t_lo, t_hi); break;
    case 3: passC64_out<UNROLL, 3, MASKED>(L, lane, K, c64, rr, t_lo, t_hi); break;
    case 5: passC64_out<UNROLL, 5, MASKED>(L, lane, K, c64, rr, t_lo, t_hi); break;
    default: passC64_out<UNROLL, 0, MASKED>(L, lane, K, c64, rr, t_lo, t_hi); break;
  }
}

template <int UNROLL>
__device__ void run_chunk64(const GenArgs &A, const InstRec &I, const ReqRec &R, uint64_t chunk, uint64_t *L,
                            uint32_t lane) {
  const uint64_t n = I.n, ninv = I.ninv, kc = I.kcorr, r2 = I.r2;
  const uint64_t e = I.e;
  const int ebits = (int)I.ebits, ekind = (int)I.ekind;
  const double den = I.den;
  const uint64_t lane_mul = A.lanemul->m64[lane];

  const uint64_t g_begin = R.g1 + chunk * A.tiles_per_chunk;
  const uint64_t g_end = min(g_begin + A.tiles_per_chunk, R.g1 + R.ntiles);
  uint64_t m_t = 0, s_t = 0;
  bool carried = false;
  for (uint64_t g = g_begin; g < g_end; ++g) {
    const uint64_t x0 = g * kTile;  // width-64 indices never reach the end of the skip period
    if (!carried) {
      dev::W128 u;
      u.lo = A.tab.u64_lo[g];
      u.hi = A.tab.u64_hi[g];
      s_t = A.tab.s64[g];
      uint64_t mu = dev::mont64(dev::redc64(u, n, ninv), r2, n, ninv);
      m_t = dev::addmod64(mu, I.mbase, n);
    }
    uint64_t *row = L + lane * kRow;
    uint64_t s = dev::mulmod_p61(s_t, lane_mul);
    uint64_t sum = 0;
#pragma unroll 4
    for (int i = 0; i < kRun; ++i) {
      s = dev::mulmod_p61(kA64, s);
      row[i] = s;
      sum = dev::addmod64(sum, s, n);
    }
    uint64_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint64_t v = dev::shfl_up_u64(incl, d);
      if ((int)lane >= d) incl = dev::addmod64(incl, v, n);
    }
    // exclusive prefix = incl - sum (mod n)
    uint64_t pre = incl >= sum ? incl - sum : incl + (n - sum);
    uint64_t m = dev::addmod64(m_t, pre, n);
#pragma unroll 4
    for (int i = 0; i < kRun; ++i) {
      m = dev::addmod64(m, row[i], n);
      row[i] = m;
    }
    m_t = dev::shfl_u64(m, 63);
    s_t = dev::shfl_u64(s, 63);
    carried = true;
    dev::wave_lds_sync();
    const uint64_t req_end = R.k + R.count;
    uint32_t t_lo = R.k > x0 ? (uint32_t)(R.k - x0) : 0u;
    uint64_t hi = min(req_end - x0, (uint64_t)kTile);
    uint32_t t_hi = (uint32_t)hi;
    const int64_t base = (int64_t)R.out_off + (int64_t)(x0 - R.k) + (int64_t)lane;
    uint64_t *c64 = A.out_c64 ? A.out_c64 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    const Enc64 K{n, ninv, kc, e, ebits, den, I.rcp};
    if (t_lo == 0 && t_hi == (uint32_t)kTile)
      passC64_e<UNROLL, false>(ekind, L, lane, K, c64, rr, t_lo, t_hi);
    else
      passC64_e<1, true>(ekind, L, lane, K, c64, rr, t_lo, t_hi);
    dev::wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// constant / unit skip (Sec. II): m at state index x is mbase + x b mod n, so
// lane l of a tile starts at state x0 + 1 + l and steps by 64 b mod n; no
// skip generator, no prefix, no LDS.
// ---------------------------------------------------------------------------

template <int UNROLL, int EK, int OUT, bool MASKED>
__device__ __forceinline__ void passCS32(uint32_t m, uint32_t step, uint32_t lane, const Enc32 &K, uint32_t *c32,
                                         double *rr, uint32_t t_lo, uint32_t t_hi) {
  const uint32_t span = t_hi - t_lo;
#pragma unroll UNROLL
  for (int i = 0; i < kRun; ++i) {
    if (!MASKED || ((uint32_t)i * 64u + lane - t_lo < span)) {
      const uint32_t c = dev::encrypt32<EK>(m, K.n, K.ninv, K.kc, K.e, K.ebits);
      if (OUT & kOutC) c32[i * 64] = c;
      if (OUT & kOutR) rr[i * 64] = dev::uniform32(c, K.den, K.rcp);
    }
    m = dev::addmod32(m, step, K.n);
  }
}

template <int UNROLL, int EK, bool MASKED>
__device__ __forceinline__ void passCS32_out(uint32_t m, uint32_t step, uint32_t lane, const Enc32 &K,
                                             uint32_t *c32, double *rr, uint32_t t_lo, uint32_t t_hi) {
  if (c32 && rr) passCS32<UNROLL, EK, kOutC | kOutR, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi);
  else if (rr) passCS32<UNROLL, EK, kOutR, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi);
  else if (c32) passCS32<UNROLL, EK, kOutC, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi);
}

template <int UNROLL, bool MASKED>
__device__ __forceinline__ void passCS32_e(int ekind, uint32_t m, uint32_t step, uint32_t lane, const Enc32 &K,
                                           uint32_t *c32, double *rr, uint32_t t_lo, uint32_t t_hi) {
  switch (ekind) {
    case 9: passCS32_out<UNROLL, 9, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi); break;
    case 17: passCS32_out<UNROLL, 17, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi); break;
    case 3: passCS32_out<UNROLL, 3, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi); break;
    case 5: passCS32_out<UNROLL, 5, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi); break;
    default: passCS32_out<UNROLL, 0, MASKED>(m, step, lane, K, c32, rr, t_lo, t_hi); break;
  }
}

template <int UNROLL>
__device__ void run_chunk32_cs(const GenArgs &A, const InstRec &I, const ReqRec &R, uint64_t chunk, uint32_t lane) {
  const uint32_t n = (uint32_t)I.n, ninv = (uint32_t)I.ninv;
  const Enc32 K{n, ninv, (uint32_t)I.kcorr, I.e, (int)I.ebits, I.den, I.rcp};
  const uint32_t bR2 = (uint32_t)I.bR2, step = (uint32_t)I.b64, mbase = (uint32_t)I.mbase;
  const uint64_t g_begin = R.g1 + chunk * A.tiles_per_chunk;
  const uint64_t g_end = min(g_begin + A.tiles_per_chunk, R.g1 + R.ntiles);
  for (uint64_t g = g_begin; g < g_end; ++g) {
    const uint64_t x0 = g * kTile;
    // lane's first state index v = x0 + 1 + lane; v b mod n by Montgomery:
    // bring hi(v) below n, then REDC(v) times b R^2
    const uint64_t v = x0 + 1 + lane;
    uint32_t vh = (uint32_t)(v >> 32);
    vh = vh >= n ? vh - n : vh;
    const uint64_t vr = ((uint64_t)vh << 32) | (uint32_t)v;
    const uint32_t m = dev::addmod32(mbase, dev::mont32(dev::redc32(vr, n, ninv), bR2, n, ninv), n);
    const uint64_t req_end = R.k + R.count;
    const uint32_t t_lo = R.k > x0 ? (uint32_t)(R.k - x0) : 0u;
    const uint32_t t_hi = (uint32_t)min(req_end - x0, (uint64_t)kTile);
    const int64_t base = (int64_t)R.out_off + (int64_t)(x0 - R.k) + (int64_t)lane;
    uint32_t *c32 = A.out_c32 ? A.out_c32 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    if (t_lo == 0 && t_hi == (uint32_t)kTile)
      passCS32_e<UNROLL, false>((int)I.ekind, m, step, lane, K, c32, rr, t_lo, t_hi);
    else
      passCS32_e<1, true>((int)I.ekind, m, step, lane, K, c32, rr, t_lo, t_hi);
  }
}

template <int UNROLL, int EK, int OUT, bool MASKED>
__device__ __forceinline__ void passCS64(uint64_t m, uint64_t step, uint32_t lane, const Enc64 &K, uint64_t *c64,
                                         double *rr, uint32_t t_lo, uint32_t t_hi) {
  const uint32_t span = t_hi - t_lo;
#pragma unroll UNROLL
  for (int i = 0; i < kRun; ++i) {
    if (!MASKED || ((uint32_t)i * 64u + lane - t_lo < span)) {
      const uint64_t c = dev::encrypt64<EK>(m, K.n, K.ninv, K.kc, K.e, K.ebits);
      if (OUT & kOutC) c64[i * 64] = c;
      if (OUT & kOutR) rr[i * 64] = dev::uniform64(c, K.den, K.rcp);
    }
    m = dev::addmod64(m, step, K.n);
  }
}

template <int UNROLL, int EK, bool MASKED>
__device__ __forceinline__ void passCS64_out(uint64_t m, uint64_t step, uint32_t lane, const Enc64 &K,
                                             uint64_t *c64, double *rr, uint32_t t_lo, uint32_t t_hi) {
  if (c64 && rr) passCS64<UNROLL, EK, kOutC | kOutR, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi);
  else if (rr) passCS64<UNROLL, EK, kOutR, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi);
  else if (c64) passCS64<UNROLL, EK, kOutC, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi);
}

template <int UNROLL, bool MASKED>
__device__ __forceinline__ void passCS64_e(int ekind, uint64_t m, uint64_t step, uint32_t lane, const Enc64 &K,
                                           uint64_t *c64, double *rr, uint32_t t_lo, uint32_t t_hi) {
  switch (ekind) {
    case 9: passCS64_out<UNROLL, 9, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi); break;
    case 17: passCS64_out<UNROLL, 17, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi); break;
    case 3: passCS64_out<UNROLL, 3, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi); break;
    case 5: passCS64_out<UNROLL, 5, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi); break;
    default: passCS64_out<UNROLL, 0, MASKED>(m, step, lane, K, c64, rr, t_lo, t_hi); break;
  }
}

template <int UNROLL>
__device__ void run_chunk64_cs(const GenArgs &A, const InstRec &I, const ReqRec &R, uint64_t chunk, uint32_t lane) {
  const uint64_t n = I.n, ninv = I.ninv;
  const Enc64 K{n, ninv, I.kcorr, I.e, (int)I.ebits, I.den, I.rcp};
  const uint64_t g_begin = R.g1 + chunk * A.tiles_per_chunk;
  const uint64_t g_end = min(g_begin + A.tiles_per_chunk, R.g1 + R.ntiles);
  for (uint64_t g = g_begin; g < g_end; ++g) {
    const uint64_t x0 = g * kTile;
    dev::W128 v;
    v.lo = x0 + 1 + lane;  // hi word 0 < n, so REDC applies
    v.hi = 0;
    const uint64_t m = dev::addmod64(I.mbase, dev::mont64(dev::redc64(v, n, ninv), I.bR2, n, ninv), n);
    const uint64_t req_end = R.k + R.count;
    const uint32_t t_lo = R.k > x0 ? (uint32_t)(R.k - x0) : 0u;
    const uint32_t t_hi = (uint32_t)min(req_end - x0, (uint64_t)kTile);
    const int64_t base = (int64_t)R.out_off + (int64_t)(x0 - R.k) + (int64_t)lane;
    uint64_t *c64 = A.out_c64 ? A.out_c64 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    if (t_lo == 0 && t_hi == (uint32_t)kTile)
      passCS64_e<UNROLL, false>((int)I.ekind, m, I.b64, lane, K, c64, rr, t_lo, t_hi);
    else
      passCS64_e<1, true>((int)I.ekind, m, I.b64, lane, K, c64, rr, t_lo, t_hi);
  }
}

// First chunk of request r in the batch.
__device__ __forceinline__ uint64_t chunk_base_of(const GenArgs &A, uint64_t r) {
  return A.gbase[r / kPlanGroup] + A.req[r].chunk_base;
}

// Wave-cooperative search: the request r whose first chunk is <= c < the next
// request's (the last such r when empty requests share a first chunk).
__device__ __forceinline__ uint64_t find_request(const GenArgs &A, uint64_t c, uint32_t lane) {
  uint64_t lo = 0, hi = A.nreq;
  while (hi - lo > 1) {
    uint64_t step = (hi - lo + 63) / 64;
    uint64_t idx = lo + (uint64_t)lane * step;
    bool le = idx < hi && chunk_base_of(A, idx) <= c;
    uint64_t mask = __ballot(le);
    uint64_t k = (uint64_t)__popcll(mask);
    lo = lo + (k - 1) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

template <bool HAS64>
struct WaveLds {
  using T = typename std::conditional<HAS64, uint64_t, uint32_t>::type;
  static constexpr int kWords = 64 * kRow;
};

template <int BLOCK, int UNROLL, bool HAS64>
__global__ void __launch_bounds__(BLOCK) gen_persistent(GenArgs A) {
  using LT = typename WaveLds<HAS64>::T;
  __shared__ LT lds[BLOCK / 64][WaveLds<HAS64>::kWords];
  const uint32_t lane = dev::lane_id();
  const uint32_t wave = dev::uniform_u32(threadIdx.x / 64);  // wave-uniform: keeps chunk math scalar
  LT *L = lds[wave];
  const uint64_t total = dev::uniform_u64(A.hdr->total_chunks);
  // The first chunk of every wave is its global wave index; later chunks come
  // from the shared counter, offset by the number of waves.  Small batches
  // therefore need no atomics, and large ones avoid the start-up burst.
  const uint32_t nwaves = gridDim.x * (BLOCK / 64);
  uint64_t c = (uint64_t)blockIdx.x * (BLOCK / 64) + wave;
  for (;;) {
    if (c >= total) break;
    const uint64_t r = dev::uniform_u64(find_request(A, c, lane));
    const ReqRec R = dev::const_load(A.req + r);
    const InstRec I = dev::const_load(A.inst + R.inst);
    const uint64_t chunk = c - (dev::const_load(A.gbase + r / kPlanGroup) + R.chunk_base);
    if (I.sched == kSchedConstant) {
      if (HAS64 && I.width == 64) run_chunk64_cs<UNROLL>(A, I, R, chunk, lane);
      else run_chunk32_cs<UNROLL>(A, I, R, chunk, lane);
    } else if (HAS64 && I.width == 64) {
      run_chunk64<UNROLL>(A, I, R, chunk, reinterpret_cast<uint64_t *>(L), lane);
    } else {
      run_chunk32<UNROLL>(A, I, R, chunk, reinterpret_cast<uint32_t *>(L), lane);
    }
    uint32_t next = 0;
    if (lane == 0) next = atomicAdd(&A.hdr->counter, 1u);
    c = (uint64_t)nwaves + dev::uniform_u32((uint32_t)__shfl((int)next, 0, 64));
  }
}

// One grid per request: block b (one wave) takes chunk b of request `r`.
template <int UNROLL, bool HAS64>
__global__ void __launch_bounds__(64) gen_plain(GenArgs A, uint64_t r) {
  using LT = typename WaveLds<HAS64>::T;
  __shared__ LT lds[WaveLds<HAS64>::kWords];
  const uint32_t lane = dev::lane_id();
  const ReqRec R = dev::const_load(A.req + r);
  if ((uint64_t)blockIdx.x >= R.nchunks) return;
  const InstRec I = dev::const_load(A.inst + R.inst);
  if (I.sched == kSchedConstant) {
    if (HAS64 && I.width == 64) run_chunk64_cs<UNROLL>(A, I, R, blockIdx.x, lane);
    else run_chunk32_cs<UNROLL>(A, I, R, blockIdx.x, lane);
  } else if (HAS64 && I.width == 64) {
    run_chunk64<UNROLL>(A, I, R, blockIdx.x, reinterpret_cast<uint64_t *>(lds), lane);
  } else {
    run_chunk32<UNROLL>(A, I, R, blockIdx.x, reinterpret_cast<uint32_t *>(lds), lane);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

hipError_t launch_table_segments32(uint64_t nseg, uint64_t *seg_sum, uint32_t *seg_start, hipStream_t st) {
  unsigned blocks = (unsigned)((nseg + 255) / 256);
  hipLaunchKernelGGL(table_segments32, dim3(blocks), dim3(256), 0, st, nseg, seg_sum, seg_start);
  return hipGetLastError();
}

hipError_t launch_table_segments64(uint64_t nseg, uint64_t *seg_lo, uint64_t *seg_hi, uint64_t *seg_start,
                                   hipStream_t st) {
  unsigned blocks = (unsigned)((nseg + 255) / 256);
  hipLaunchKernelGGL(table_segments64, dim3(blocks), dim3(256), 0, st, nseg, seg_lo, seg_hi, seg_start);
  return hipGetLastError();
}

hipError_t launch_seed_prime_flags(uint64_t seed, uint64_t j0, uint64_t count, int width, uint8_t *flags,
                                   hipStream_t st) {
  unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(seed_prime_flags, dim3(blocks), dim3(256), 0, st, seed, j0, count, width, flags);
  return hipGetLastError();
}

hipError_t launch_build_records(const uint64_t *n, const uint64_t *e, uint64_t count, int width, InstRec *out,
                                hipStream_t st) {
  unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(build_records, dim3(blocks), dim3(256), 0, st, n, e, count, width, out);
  return hipGetLastError();
}

hipError_t launch_plan(const InstRec *inst, const HostReq *src, ReqRec *req, uint64_t nreq, uint64_t *gbase,
                       PlanHdr *hdr, uint32_t tiles_per_chunk, hipStream_t st) {
  if (nreq == 0) return hipErrorInvalidValue;
  const uint64_t groups = (nreq + kPlanGroup - 1) / kPlanGroup;
  if (groups > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(plan_kernel, dim3((unsigned)groups), dim3(kPlanGroup), 0, st, inst, src, req, nreq, gbase, hdr,
                     tiles_per_chunk);
  return hipGetLastError();
}

hipError_t launch_advance(HostReq *req, uint64_t nreq, hipStream_t st) {
  if (nreq == 0) return hipSuccess;
  unsigned blocks = (unsigned)((nreq + 255) / 256);
  hipLaunchKernelGGL(advance_kernel, dim3(blocks), dim3(256), 0, st, req, nreq);
  return hipGetLastError();
}

template <int BLOCK, int UNROLL, bool HAS64>
static void launch_p(const GenArgs &A, unsigned grid, hipStream_t st) {
  hipLaunchKernelGGL((gen_persistent<BLOCK, UNROLL, HAS64>), dim3(grid), dim3(BLOCK), 0, st, A);
}

template <int BLOCK, bool HAS64>
static bool launch_pu(const GenArgs &A, unsigned grid, int unroll, hipStream_t st) {
  switch (unroll) {
    case 1: launch_p<BLOCK, 1, HAS64>(A, grid, st); return true;
    case 2: launch_p<BLOCK, 2, HAS64>(A, grid, st); return true;
    case 4: launch_p<BLOCK, 4, HAS64>(A, grid, st); return true;
    default: return false;
  }
}

template <bool HAS64>
static bool launch_pb(const GenArgs &A, unsigned grid, int block, int unroll, hipStream_t st) {
  switch (block) {
    case 64: return launch_pu<64, HAS64>(A, grid, unroll, st);
    case 128: return launch_pu<128, HAS64>(A, grid, unroll, st);
    case 256: return launch_pu<256, HAS64>(A, grid, unroll, st);
    case 512: return launch_pu<512, HAS64>(A, grid, unroll, st);
    default: return false;
  }
}

hipError_t launch_persistent(const GenArgs &A, unsigned grid, int block, int unroll, bool has64, hipStream_t st) {
  bool ok = has64 ? launch_pb<true>(A, grid, block, unroll, st) : launch_pb<false>(A, grid, block, unroll, st);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_plain(const GenArgs &A, uint64_t r, unsigned grid, int unroll, bool has64, hipStream_t st) {
  if (grid == 0) return hipSuccess;
  if (has64) {
    if (unroll == 4) hipLaunchKernelGGL((gen_plain<4, true>), dim3(grid), dim3(64), 0, st, A, r);
    else if (unroll == 2) hipLaunchKernelGGL((gen_plain<2, true>), dim3(grid), dim3(64), 0, st, A, r);
    else hipLaunchKernelGGL((gen_plain<1, true>), dim3(grid), dim3(64), 0, st, A, r);
  } else {
    if (unroll == 4) hipLaunchKernelGGL((gen_plain<4, false>), dim3(grid), dim3(64), 0, st, A, r);
    else if (unroll == 2) hipLaunchKernelGGL((gen_plain<2, false>), dim3(grid), dim3(64), 0, st, A, r);
    else hipLaunchKernelGGL((gen_plain<1, false>), dim3(grid), dim3(64), 0, st, A, r);
  }
  return hipGetLastError();
}

}  // namespace phprng
