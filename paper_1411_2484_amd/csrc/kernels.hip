// gfx950 kernels for the Pohlig-Hellman parameter-split generator:
//   - skip-prefix table segments (eq. (7b) building blocks),
//   - width-64 tile starts, from the 64-bit table for instances that stay
//     in its range, else from the requests' own skip sums (reduce, then a
//     scan per instance); both commit the instance's message,
//   - batched generation (algorithm (9)) as a persistent work-stealing grid
//     or as one plain grid per request,
//   - width-64 positioning and jumps (eq. (7) sums on the device),
//   - the fixed scratch of the allocation-free entry point.
//
// Width-32 tiles are 2048 consecutive draws of one instance whose starting
// state index is a multiple of 2048 within the skip period: the universal
// table holds the skip-prefix sum U and the skip a^r there.  Width-64 tiles
// are 1024 draws, starting at multiples of 1024 skip logarithms (table
// entries) or counted from the first draw of their request (reduce and
// scan).  One wave computes a tile in
// three passes over its LDS row block:
//   A. lane l steps the skip generator over its run of draws, keeps the
//      skips in LDS and sums them;
//   B. a wave scan of the run sums gives each lane its starting message; the
//      lane accumulates its run's messages into LDS (eq. (3a));
//   C. lanes read the messages back in draw order (lane l takes draws
//      i*64 + l), encrypt (eq. (1)), form R and store both coalesced.
// A chunk is a run of consecutive tiles of one request; a wave carries the
// state from one tile to the next within a chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "arith.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace phprng {

constexpr int kRow32 = kRun32 + 1;  // padded LDS rows (conflict-free for both access orders)
constexpr int kRow64 = kRun64 + 1;
static_assert((kTilesPerPeriod32 & (kTilesPerPeriod32 - 1)) == 0, "tiles per period is a power of two");
constexpr int kTileShift32 = 20;
static_assert((1ull << kTileShift32) == kTilesPerPeriod32, "tile shift");
// LDS words (64-bit) per wave: the width-32 block, or the larger width-64 one.
constexpr int kLdsWords32 = (64 * kRow32 + 1) / 2;  // 1056
constexpr int kLdsWords64 = 64 * kRow64;            // 1088

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
  uint64_t s = dev::powmod_p61(kA64, i * kTab64Stride);
  seg_start[i] = s;
  uint64_t lo = 0, hi = 0;
  for (uint64_t j = 0; j < kTab64Stride; ++j) {
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
// width-64 skip sums from the positioning table (eq. (7b))
// ---------------------------------------------------------------------------

// U(t) mod n for t < kTab64Range: the table entry at or below t plus at most
// kTab64Stride - 1 steps of the skip generator, then the 128-bit sum reduced
// mod n.
__device__ uint64_t table_prefix64(const uint64_t *u_lo, const uint64_t *u_hi, const uint64_t *u_s, uint64_t t,
                                   uint64_t n, uint64_t ninv, uint64_t r2) {
  const uint64_t i = t / kTab64Stride;
  uint64_t lo = u_lo[i], hi = u_hi[i], s = u_s[i];
  for (uint64_t x = i * kTab64Stride; x < t; ++x) {
    s = dev::mulmod_p61(kA64, s);
    const uint64_t v = lo + s;
    hi += v < lo ? 1 : 0;
    lo = v;
  }
  // hi < 2^30 < n, so REDC applies; times R^2 undoes the 2^-64
  dev::W128 w;
  w.lo = lo;
  w.hi = hi;
  return dev::mont64(dev::redc64(w, n, ninv), r2, n, ninv);
}

// m64[ids[i]] = m0[i] + U(ta[i]) - U(tb[i]) mod n, for skip logarithms
// ta, tb < kTab64Range (one thread per instance).  With ta = t0 + k0 and
// tb = t0 this is the message at position k0 of an instance whose state at
// position 0 is (m0, a^t0) (eq. (7b)); a jump by d from skip log t takes
// ta = t + d, tb = t (backward: ta = t - d).
__global__ void __launch_bounds__(256) position64_kernel(const InstRec *inst, const uint32_t *ids, const uint64_t *m0,
                                                         const uint64_t *ta, const uint64_t *tb, uint64_t count,
                                                         const uint64_t *u_lo, const uint64_t *u_hi,
                                                         const uint64_t *u_s, uint64_t *m64) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const InstRec &I = inst[ids[i]];
  const uint64_t n = I.n, ninv = I.ninv, r2 = I.r2;
  const uint64_t a = ta ? ta[i] : 0, b = tb ? tb[i] : 0;
  const uint64_t ua = a ? table_prefix64(u_lo, u_hi, u_s, a, n, ninv, r2) : 0;
  const uint64_t ub = b ? table_prefix64(u_lo, u_hi, u_s, b, n, ninv, r2) : 0;
  const uint64_t m = dev::addmod64(m0 ? m0[i] : 0, ua, n);
  m64[ids[i]] = m >= ub ? m - ub : m + (n - ub);
}

// ---------------------------------------------------------------------------
// width-64 tile starts: reduce, then scan per instance
// ---------------------------------------------------------------------------

// Wave-cooperative search over a sorted key: the last index r in [0, nreq)
// with key(r) <= c (the last such r when empty requests share a key).
template <typename Key>
__device__ __forceinline__ uint64_t wave_search(uint64_t nreq, uint64_t c, uint32_t lane, Key key) {
  uint64_t lo = 0, hi = nreq;
  while (hi - lo > 1) {
    const uint64_t step = (hi - lo + 63) / 64;
    const uint64_t idx = lo + (uint64_t)lane * step;
    const bool le = idx < hi && key(idx) <= c;
    const uint64_t mask = __ballot(le);
    const uint64_t k = (uint64_t)__popcll(mask);
    lo = lo + (k - 1) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

// Sum, mod n, of the skips of lane `lane`'s run of kRun64 draws in a tile
// that starts with skip s_tile and holds `len` draws; every lane gets the
// tile total.
__device__ __forceinline__ uint64_t tile_skip_sum64(uint64_t s_tile, uint64_t lane_mul, uint32_t len, uint64_t n,
                                                    uint32_t lane) {
  uint64_t s = dev::mulmod_p61(s_tile, lane_mul);
  uint64_t sum = 0;
  const uint32_t first = lane * kRun64;
#pragma unroll 4
  for (int i = 0; i < kRun64; ++i) {
    s = dev::mulmod_p61(kA64, s);
    if (first + (uint32_t)i < len) sum = dev::addmod64(sum, s, n);
  }
  return dev::wave_sum_mod(sum, n);
}

// Draws in tile j of a width-64 request: 1024, or what is left in its last
// tile.  Written with a 32-bit test of the tile index: a wave-uniform 64-bit
// "rem < 1024 ? rem : 1024" has been compiled for gfx950 into a select that
// reads a stale SCC after the branch on the same comparison, which gave 1024
// for every last tile.
__device__ __forceinline__ uint32_t tile_len64(const ReqRec &R, uint32_t j, uint32_t head = 0) {
  // one past the request's last draw, counted from the first tile's start
  const uint32_t last = (uint32_t)(R.count + head - (uint64_t)(R.ntiles - 1) * kTile64);
  return j + 1 == R.ntiles ? last : (uint32_t)kTile64;
}

// One wave per reduce unit (grid-stride): up to hdr->reduce_tiles consecutive
// tiles of one width-64 request.  For each tile j of a request starting at
// skip log t it writes the skip before the tile, a^{t + 1024 j} mod p (a
// power for the unit's first tile, then carried from tile to tile), and the
// sum of the tile's skips mod n.
__global__ void __launch_bounds__(256) reduce64_kernel(GenArgs A) {
  const uint32_t lane = dev::lane_id();
  const uint32_t wave = dev::uniform_u32(threadIdx.x / 64);
  const uint64_t units = dev::uniform_u64(dev::const_load(&A.hdr->units64));
  const uint64_t nreq64 = dev::uniform_u64(dev::const_load(&A.hdr->nreq64));
  const uint32_t rt = dev::uniform_u32((uint32_t)dev::const_load(&A.hdr->reduce_tiles));
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / 64);
  const uint64_t lane_mul = A.lanemul->m64[lane];
  const uint64_t pm1 = kP64 - 1;
  for (uint64_t u = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave; u < units; u += nwaves) {
    const uint64_t r =
        dev::uniform_u64(wave_search(nreq64, u, lane, [&](uint64_t i) { return A.req[i].rbase; }));
    const ReqRec R = dev::const_load(A.req + r);
    const uint64_t n = dev::const_load(&A.inst[R.inst].n);
    const uint32_t j0 = (uint32_t)(u - R.rbase) * rt;
    const uint32_t j1 = R.ntiles - j0 > rt ? j0 + rt : R.ntiles;
    uint64_t lg = R.x + (uint64_t)j0 * kTile64;  // x < p - 1 and j * 1024 < 2^42: one subtraction wraps it
    if (lg >= pm1) lg -= pm1;
    uint64_t s_tile = dev::wave_pow_p61(A.lanemul->pow64, lg, lane);
    const uint64_t a8 = A.lanemul->pow64[3];  // a^8
    for (uint32_t j = j0; j < j1; ++j) {
      const uint32_t len = tile_len64(R, j);
      uint64_t sum;
      uint64_t s = dev::mulmod_p61(s_tile, lane_mul);  // skip before the lane's run
      if (len == kTile64) {
        // The run as two independent chains of 8 skips (more work in flight
        // per lane).  Eight skips below 2^61 sum below 2^64 < 4n, so each
        // chain is summed in plain 64-bit adds and reduced once.
        uint64_t s2 = dev::mulmod_p61(s, a8);
        uint64_t g1 = 0, g2 = 0;
#pragma unroll
        for (int i = 0; i < kRun64 / 2; ++i) {
          s = dev::mulmod_p61(kA64, s);
          s2 = dev::mulmod_p61(kA64, s2);
          g1 += s;
          g2 += s2;
        }
        sum = dev::addmod64(dev::mod_below_4n(g1, n), dev::mod_below_4n(g2, n), n);
        s = s2;
      } else {
        // the request's last tile: only draws below len count
        const uint32_t first = lane * kRun64;
        sum = 0;
#pragma unroll 4
        for (int i = 0; i < kRun64; ++i) {
          s = dev::mulmod_p61(kA64, s);
          if (first + (uint32_t)i < len) sum = dev::addmod64(sum, s, n);
        }
      }
      sum = dev::wave_sum_mod(sum, n);
      if (lane == 0) {
        A.t64.s[R.g1 + j] = s_tile;
        A.t64.sum[R.g1 + j] = sum;
      }
      s_tile = dev::shfl_u64(s, 63);  // the skip after the tile's last draw
    }
  }
}

// ---------------------------------------------------------------------------
// width-64 tile starts from the table (batches whose draws all lie below
// kTab64Range)
// ---------------------------------------------------------------------------

// A table entry U(i * kTab64Stride) (128 bits, read as w) reduced mod n:
// U < 2^95 < n 2^64, so one REDC and a product with R^2 give it.  n is the
// same in every lane of the wave.
__device__ __forceinline__ uint64_t table_u_mod64(dev::W128 w, uint64_t n, uint64_t ninv, uint64_t r2) {
  return dev::mont64_uniform(dev::redc64_uniform(w, n, ninv), r2, n, ninv);
}

// U(x) mod n and U(y) mod n for x, y < kTab64Range by the whole wave: the
// entry at or below each plus the (at most kTab64Stride - 1) skips after
// it, lane l taking the 16 skip indices from T + 16 l + 1.  The table reads
// of both positions are issued before either is used, and the two skip
// chains run side by side.  Every lane gets both results.
__device__ void wave_prefix64_pair(const SkipTables &T, uint64_t x, uint64_t y, uint64_t n, uint64_t ninv,
                                   uint64_t r2, uint64_t lane_mul, uint32_t lane, uint64_t *ux, uint64_t *uy) {
  const uint64_t ix = x / kTab64Stride, iy = y / kTab64Stride;
  const uint32_t rx = (uint32_t)(x - ix * kTab64Stride), ry = (uint32_t)(y - iy * kTab64Stride);
  const uint64_t sx0 = dev::const_load(T.s64 + ix), sy0 = dev::const_load(T.s64 + iy);
  const dev::W128 wx{dev::const_load(T.u64lo + ix), dev::const_load(T.u64hi + ix)};
  const dev::W128 wy{dev::const_load(T.u64lo + iy), dev::const_load(T.u64hi + iy)};
  uint64_t sx = dev::mulmod_p61(sx0, lane_mul), sy = dev::mulmod_p61(sy0, lane_mul);
  uint64_t sumx = 0, sumy = 0;
  const uint32_t first = lane * kRun64;
#pragma unroll 4
  for (int k = 0; k < kRun64; ++k) {
    sx = dev::mulmod_p61(kA64, sx);
    sy = dev::mulmod_p61(kA64, sy);
    if (first + (uint32_t)k < rx) sumx = dev::addmod64(sumx, sx, n);
    if (first + (uint32_t)k < ry) sumy = dev::addmod64(sumy, sy, n);
  }
  *ux = dev::addmod64(table_u_mod64(wx, n, ninv, r2), dev::wave_sum_mod(sumx, n), n);
  *uy = dev::addmod64(table_u_mod64(wy, n, ninv, r2), dev::wave_sum_mod(sumy, n), n);
}

// One wave per width-64 request; the first request of each instance in the
// batch whose tiles start at table entries (seg count > 0 and kSegTable)
// serves all of that instance's requests.  With m the
// instance's committed message at skip log x (its first request's start),
// mbase = m - U(x) mod n gives the message at any skip log t of the range as
// mbase + U(t) (eq. (7b)).  Each tile of the requests starts at a table
// entry, so its skip a^t and message come straight from the table.  The
// wave then commits the message after the instance's last draw in the batch.
__global__ void __launch_bounds__(64) tab64_kernel(GenArgs A) {
  const uint32_t lane = dev::lane_id();
  const ReqRec R0 = dev::const_load(A.req + blockIdx.x);
  const uint32_t seg = R0.seg & kSegCount;
  if (seg == 0 || !(R0.seg & kSegTable)) return;
  const InstRec &I = A.inst[R0.inst];
  const uint64_t n = dev::const_load(&I.n), ninv = dev::const_load(&I.ninv), r2 = dev::const_load(&I.r2);
  const uint64_t lane_mul = A.lanemul->m64[lane];
  const uint64_t m0 = dev::uniform_u64(A.m64[R0.inst]);
  // U at the instance's first and last positions in the batch
  const ReqRec RL = dev::const_load(A.req + blockIdx.x + seg - 1);
  uint64_t u0, ue;
  wave_prefix64_pair(A.tab, R0.x, RL.x + RL.count, n, ninv, r2, lane_mul, lane, &u0, &ue);
  const uint64_t mbase = m0 >= u0 ? m0 - u0 : m0 + (n - u0);
  for (uint32_t q = 0; q < seg; ++q) {
    const ReqRec R = dev::const_load(A.req + blockIdx.x + q);
    const uint64_t e0 = R.x / kTab64Stride;
    // the table reads of kTabGroup tiles per lane are issued before any of
    // them is used, so their latencies overlap (a long request has up to
    // 16 tiles per lane)
    constexpr int kTabGroup = 8;
    for (uint32_t j0 = 0; j0 < R.ntiles; j0 += 64 * kTabGroup) {
      // lanes past the request's last tile compute on zeros and store nothing
      uint64_t sv[kTabGroup] = {}, ulo[kTabGroup] = {}, uhi[kTabGroup] = {};
#pragma unroll
      for (int k = 0; k < kTabGroup; ++k) {
        const uint32_t j = j0 + 64 * k + lane;
        if (j < R.ntiles) {
          sv[k] = dev::const_load(A.tab.s64 + e0 + j);
          ulo[k] = dev::const_load(A.tab.u64lo + e0 + j);
          uhi[k] = dev::const_load(A.tab.u64hi + e0 + j);
        }
      }
      uint64_t mv[kTabGroup];
#pragma unroll
      for (int k = 0; k < kTabGroup; ++k) {
        // mbase + U(1024 e) mod n
        mv[k] = dev::addmod64(mbase, table_u_mod64({ulo[k], uhi[k]}, n, ninv, r2), n);
      }
#pragma unroll
      for (int k = 0; k < kTabGroup; ++k) {
        const uint32_t j = j0 + 64 * k + lane;
        if (j < R.ntiles) {
          A.t64.s[R.g1 + j] = sv[k];
          A.t64.m[R.g1 + j] = mv[k];
        }
      }
    }
  }
  if (lane == 0) A.m64[R0.inst] = dev::addmod64(mbase, ue, n);
}

// Scan per instance: one workgroup per width-64 request; the first request
// of each instance in the batch (seg > 0) turns the tile sums of all of that
// instance's requests into tile-start messages, starting from the
// instance's committed message, and commits the message after the last
// draw.  The instance's requests hold consecutive tiles.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;

__global__ void __launch_bounds__(kScanThreads) scan64_kernel(GenArgs A) {
  __shared__ uint64_t wtot[kScanThreads / 64];
  const uint64_t r = blockIdx.x;
  const ReqRec R = dev::const_load(A.req + r);
  const uint32_t seg = R.seg & kSegCount;
  if (seg == 0 || (R.seg & kSegTable)) return;
  const ReqRec L = dev::const_load(A.req + r + seg - 1);
  const uint64_t n = dev::const_load(&A.inst[R.inst].n);
  const uint64_t t0 = R.g1, t1 = L.g1 + L.ntiles;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint64_t carry = A.m64[R.inst];
  for (uint64_t base = t0; base < t1; base += (uint64_t)kScanThreads * kScanPer) {
    const uint64_t first = base + (uint64_t)tid * kScanPer;
    uint64_t v[kScanPer];
    uint64_t tot = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      v[q] = first + q < t1 ? A.t64.sum[first + q] : 0;
      tot = dev::addmod64(tot, v[q], n);
    }
    // exclusive prefix of the thread totals over the workgroup
    const uint64_t ex = dev::wave_exclusive_mod(tot, n, lane);
    if (lane == 63) wtot[w] = dev::addmod64(ex, tot, n);
    __syncthreads();
    uint64_t before = carry, all = carry;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
      if (k < (int)w) before = dev::addmod64(before, wtot[k], n);
      all = dev::addmod64(all, wtot[k], n);
    }
    __syncthreads();
    uint64_t m = dev::addmod64(before, ex, n);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      if (first + q < t1) A.t64.m[first + q] = m;
      m = dev::addmod64(m, v[q], n);
    }
    carry = all;
  }
  if (tid == 0) A.m64[R.inst] = carry;
}

// ---------------------------------------------------------------------------
// width-64 jumps off the table: sum of `count` consecutive skips
// ---------------------------------------------------------------------------

// partial[w] = sum, mod n, of the skips a^{t+1+i} mod p for the blocks of
// 1024 draws i in [1024 b, 1024 (b + 1)) ∩ [0, count) that wave w takes
// (b = w, w + nwaves, ...).
__global__ void __launch_bounds__(256) skip_total64_kernel(uint64_t t, uint64_t count, uint64_t n,
                                                           const LaneMul *lm, uint64_t *partial) {
  const uint32_t lane = dev::lane_id();
  const uint32_t wave = dev::uniform_u32(threadIdx.x / 64);
  const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / 64);
  const uint64_t pm1 = kP64 - 1;
  const uint64_t lane_mul = lm->m64[lane];
  const uint64_t nblk = (count + kTile64 - 1) / kTile64;
  uint64_t acc = 0;
  for (uint64_t b = w; b < nblk; b += nwaves) {
    const uint64_t off = (b * kTile64) % pm1;
    uint64_t lg = t + off;
    if (lg >= pm1) lg -= pm1;
    const uint64_t s0 = dev::wave_pow_p61(lm->pow64, lg, lane);
    // the last block holds what is left (an equality test: see tile_len64)
    const uint32_t len = b + 1 == nblk ? (uint32_t)(count - (nblk - 1) * kTile64) : (uint32_t)kTile64;
    acc = dev::addmod64(acc, tile_skip_sum64(s0, lane_mul, len, n, lane), n);
  }
  if (lane == 0) partial[w] = acc;
}

// *m = *m + sign * (sum of the partials + extra) mod n (one wave).
__global__ void __launch_bounds__(64) skip_total64_apply(const uint64_t *partial, uint64_t nparts, uint64_t n,
                                                         uint64_t extra, int sign, uint64_t *m) {
  const uint32_t lane = threadIdx.x;
  uint64_t acc = 0;
  for (uint64_t i = lane; i < nparts; i += 64) acc = dev::addmod64(acc, partial[i], n);
  acc = dev::wave_sum_mod(acc, n);
  acc = dev::addmod64(acc, extra, n);
  if (lane == 0) {
    const uint64_t v = *m;
    *m = sign > 0 ? dev::addmod64(v, acc, n) : (v >= acc ? v - acc : v + (n - acc));
  }
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
  const uint32_t *src = L + (lane >> 5) * kRow32 + (lane & 31);
  const uint32_t span = t_hi - t_lo;
#pragma unroll UNROLL
  for (int i = 0; i < kRun32; ++i) {
    const uint32_t m = src[i * 2 * kRow32];
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
    const uint64_t x0 = q * pm1 + (uint64_t)j * kTile32;
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
    uint32_t *row = L + lane * kRow32;
    uint32_t s = dev::mulmod_p31(s_t, lane_mul);
    uint64_t sum = 0;
#pragma unroll 8
    for (int i = 0; i < kRun32; ++i) {
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
    for (int i = 0; i < kRun32; ++i) {
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
    const uint64_t req_end = R.x + R.count;  // one past the last state index used
    uint32_t t_lo = R.x > tile_first ? (uint32_t)(R.x - tile_first) : 0u;
    uint64_t hi1 = req_end - tile_first;
    uint64_t hi2 = pm1 - (uint64_t)j * kTile32;
    uint64_t hi = min(min(hi1, hi2), (uint64_t)kTile32);
    uint32_t t_hi = (uint32_t)hi;
    const int64_t base = (int64_t)R.out_off + (int64_t)(tile_first - R.x) + (int64_t)lane;
    uint32_t *c32 = A.out_c32 ? A.out_c32 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    const Enc32 K{n, ninv, kc, e, ebits, den, rcp};
    if (t_lo == 0 && t_hi == (uint32_t)kTile32)
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

// Pass C, width 64: draw t = i*64 + lane lives at LDS row t / 16, column
// t % 16, i.e. row 4 i + lane / 16.  MASKED tiles write only t_lo <= t < t_hi.
template <int UNROLL, int EK, int OUT, bool MASKED>
__device__ __forceinline__ void passC64(const uint64_t *L, uint32_t lane, const Enc64 &K, uint64_t *c64, double *rr,
                                        uint32_t t_lo, uint32_t t_hi) {
  const uint64_t *src = L + (lane >> 4) * kRow64 + (lane & 15);
  const uint32_t span = t_hi - t_lo;
#pragma unroll UNROLL
  for (int i = 0; i < kRun64; ++i) {
    const uint64_t m = src[i * 4 * kRow64];
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

// Width 64: tile j of the request covers its draws [1024 j, 1024 (j + 1)),
// or, when the instance's tiles start at table entries, the skip logarithms
// (1024 (e0 + j), 1024 (e0 + j + 1)] with e0 = x / 1024, of which the first
// tile skips the part before the request.  The state before the chunk's
// first tile comes from the scan or the table kernel; later tiles continue
// from lane 63's last state.
template <int UNROLL>
__device__ void run_chunk64(const GenArgs &A, const InstRec &I, const ReqRec &R, uint64_t chunk, uint64_t *L,
                            uint32_t lane) {
  const uint64_t n = I.n, ninv = I.ninv, kc = I.kcorr;
  const uint64_t e = I.e;
  const int ebits = (int)I.ebits, ekind = (int)I.ekind;
  const double den = I.den;
  const uint64_t lane_mul = A.lanemul->m64[lane];

  const uint32_t j_begin = (uint32_t)chunk * A.tiles_per_chunk;
  const uint32_t j_end = min(j_begin + A.tiles_per_chunk, R.ntiles);
  const bool tab = (R.seg & kSegTable) != 0;
  // draw t of tile j is request draw (first draw of tile j) + t; at table
  // entries the first tile starts x mod 1024 draws before the request
  const uint32_t head = tab ? (uint32_t)(R.x & (kTab64Stride - 1)) : 0u;
  uint64_t m_t = dev::uniform_u64(dev::const_load(A.t64.m + R.g1 + j_begin));
  uint64_t s_t = dev::uniform_u64(dev::const_load(A.t64.s + R.g1 + j_begin));
  for (uint32_t j = j_begin; j < j_end; ++j) {
    // ---- pass A
    uint64_t *row = L + lane * kRow64;
    uint64_t s = dev::mulmod_p61(s_t, lane_mul);
    // eight skips below 2^61 sum below 2^64 < 4n: plain adds, one reduction per half run
    uint64_t g1 = 0, g2 = 0;
#pragma unroll 4
    for (int i = 0; i < kRun64 / 2; ++i) {
      s = dev::mulmod_p61(kA64, s);
      row[i] = s;
      g1 += s;
    }
#pragma unroll 4
    for (int i = kRun64 / 2; i < kRun64; ++i) {
      s = dev::mulmod_p61(kA64, s);
      row[i] = s;
      g2 += s;
    }
    const uint64_t sum = dev::addmod64(dev::mod_below_4n(g1, n), dev::mod_below_4n(g2, n), n);
    // ---- pass B
    uint64_t m = dev::addmod64(m_t, dev::wave_exclusive_mod(sum, n, lane), n);
#pragma unroll 4
    for (int i = 0; i < kRun64; ++i) {
      m = dev::addmod64(m, row[i], n);
      row[i] = m;
    }
    m_t = dev::shfl_u64(m, 63);
    s_t = dev::shfl_u64(s, 63);
    dev::wave_lds_sync();
    // ---- pass C
    const uint32_t t_lo = j == 0 ? head : 0u;
    const uint32_t t_hi = tile_len64(R, j, head);
    const int64_t base = (int64_t)R.out_off + (int64_t)j * kTile64 - (int64_t)head + (int64_t)lane;
    uint64_t *c64 = A.out_c64 ? A.out_c64 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    const Enc64 K{n, ninv, kc, e, ebits, den, I.rcp};
    if (t_lo == 0 && t_hi == (uint32_t)kTile64)
      passC64_e<UNROLL, false>(ekind, L, lane, K, c64, rr, 0u, t_hi);
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
  for (int i = 0; i < kTileCS / 64; ++i) {
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
    const uint64_t x0 = g * kTileCS;
    // lane's first state index v = x0 + 1 + lane; v b mod n by Montgomery:
    // bring hi(v) below n, then REDC(v) times b R^2
    const uint64_t v = x0 + 1 + lane;
    uint32_t vh = (uint32_t)(v >> 32);
    vh = vh >= n ? vh - n : vh;
    const uint64_t vr = ((uint64_t)vh << 32) | (uint32_t)v;
    const uint32_t m = dev::addmod32(mbase, dev::mont32(dev::redc32(vr, n, ninv), bR2, n, ninv), n);
    const uint64_t req_end = R.x + R.count;
    const uint32_t t_lo = R.x > x0 ? (uint32_t)(R.x - x0) : 0u;
    const uint32_t t_hi = (uint32_t)min(req_end - x0, (uint64_t)kTileCS);
    const int64_t base = (int64_t)R.out_off + (int64_t)(x0 - R.x) + (int64_t)lane;
    uint32_t *c32 = A.out_c32 ? A.out_c32 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    if (t_lo == 0 && t_hi == (uint32_t)kTileCS)
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
  for (int i = 0; i < kTileCS / 64; ++i) {
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
    const uint64_t x0 = g * kTileCS;
    dev::W128 v;
    v.lo = x0 + 1 + lane;  // hi word 0 < n, so REDC applies
    v.hi = 0;
    const uint64_t m = dev::addmod64(I.mbase, dev::mont64(dev::redc64(v, n, ninv), I.bR2, n, ninv), n);
    const uint64_t req_end = R.x + R.count;
    const uint32_t t_lo = R.x > x0 ? (uint32_t)(R.x - x0) : 0u;
    const uint32_t t_hi = (uint32_t)min(req_end - x0, (uint64_t)kTileCS);
    const int64_t base = (int64_t)R.out_off + (int64_t)(x0 - R.x) + (int64_t)lane;
    uint64_t *c64 = A.out_c64 ? A.out_c64 + base : nullptr;
    double *rr = A.out_r ? A.out_r + base : nullptr;
    if (t_lo == 0 && t_hi == (uint32_t)kTileCS)
      passCS64_e<UNROLL, false>((int)I.ekind, m, I.b64, lane, K, c64, rr, t_lo, t_hi);
    else
      passCS64_e<1, true>((int)I.ekind, m, I.b64, lane, K, c64, rr, t_lo, t_hi);
  }
}

// One chunk of request r.
template <int UNROLL, bool HAS64>
__device__ __forceinline__ void run_chunk(const GenArgs &A, const ReqRec &R, uint64_t chunk, uint64_t *L,
                                          uint32_t lane) {
  const InstRec I = dev::const_load(A.inst + R.inst);
  if (I.sched == kSchedConstant) {
    if (HAS64 && I.width == 64) run_chunk64_cs<UNROLL>(A, I, R, chunk, lane);
    else run_chunk32_cs<UNROLL>(A, I, R, chunk, lane);
  } else if (HAS64 && I.width == 64) {
    run_chunk64<UNROLL>(A, I, R, chunk, L, lane);
  } else {
    run_chunk32<UNROLL>(A, I, R, chunk, reinterpret_cast<uint32_t *>(L), lane);
  }
}

template <int BLOCK, int UNROLL, bool HAS64>
__global__ void __launch_bounds__(BLOCK) gen_persistent(GenArgs A) {
  __shared__ uint64_t lds[BLOCK / 64][HAS64 ? kLdsWords64 : kLdsWords32];
  const uint32_t lane = dev::lane_id();
  const uint32_t wave = dev::uniform_u32(threadIdx.x / 64);  // wave-uniform: keeps chunk math scalar
  uint64_t *L = lds[wave];
  const uint64_t total = dev::uniform_u64(dev::const_load(&A.hdr->total_chunks));
  // The first chunk of every wave is its global wave index; later chunks come
  // from the shared counter, offset by the number of waves.  Small batches
  // therefore need no atomics, and large ones avoid the start-up burst.
  const uint32_t nwaves = gridDim.x * (BLOCK / 64);
  uint64_t c = (uint64_t)blockIdx.x * (BLOCK / 64) + wave;
  // Every wave grabs until a grab fails, so there are total - nwaves
  // successful grabs and one failed grab per wave: the grabs return
  // 0 .. total - 1, and the one returning total - 1 is the last of all.  Its
  // wave puts the counter back to zero for the next launch.  A batch with no
  // more chunks than waves never touches the counter.  (One call site of
  // run_chunk: a second one gets the whole chunk code outlined into a call.)
  const bool grab = total > nwaves;
  for (;;) {
    if (c >= total) break;
    const uint64_t r =
        dev::uniform_u64(wave_search(A.nreq, c, lane, [&](uint64_t i) { return A.req[i].chunk_base; }));
    const ReqRec R = dev::const_load(A.req + r);
    run_chunk<UNROLL, HAS64>(A, R, c - R.chunk_base, L, lane);
    if (!grab) break;
    uint32_t next = 0;
    if (lane == 0) {
      next = atomicAdd(&A.ctr->counter, 1u);
      if ((uint64_t)next == total - 1) __hip_atomic_store(&A.ctr->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    c = (uint64_t)nwaves + dev::uniform_u32((uint32_t)__shfl((int)next, 0, 64));
  }
}

// One grid per request: block b (one wave) takes chunk b of request `r`.
template <int UNROLL, bool HAS64>
__global__ void __launch_bounds__(64) gen_plain(GenArgs A, uint64_t r) {
  __shared__ uint64_t lds[HAS64 ? kLdsWords64 : kLdsWords32];
  const uint32_t lane = dev::lane_id();
  const ReqRec R = dev::const_load(A.req + r);
  if ((uint64_t)blockIdx.x >= R.nchunks) return;
  run_chunk<UNROLL, HAS64>(A, R, blockIdx.x, lds, lane);
}

// ---------------------------------------------------------------------------
// fixed scratch of the allocation-free entry point
// ---------------------------------------------------------------------------

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it takes the device address once per device
// (scratch_address) and uses that.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

__global__ void __launch_bounds__(64) clear_words(uint32_t *p, uint32_t nwords) {
  for (uint32_t i = threadIdx.x; i < nwords; i += 64) p[i] = 0;
}

hipError_t scratch_address(int device, void **ptr) {
  clear_launch_error();
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    // the work counter must start at zero; every launch leaves it so
    hipLaunchKernelGGL(clear_words, dim3(1), dim3(64), 0, nullptr, static_cast<uint32_t *>(p),
                       (uint32_t)(kScratchClearBytes / 4));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

hipError_t launch_table_segments32(uint64_t nseg, uint64_t *seg_sum, uint32_t *seg_start, hipStream_t st) {
  clear_launch_error();
  unsigned blocks = (unsigned)((nseg + 255) / 256);
  hipLaunchKernelGGL(table_segments32, dim3(blocks), dim3(256), 0, st, nseg, seg_sum, seg_start);
  return hipGetLastError();
}

hipError_t launch_table_segments64(uint64_t nseg, uint64_t *seg_lo, uint64_t *seg_hi, uint64_t *seg_start,
                                   hipStream_t st) {
  clear_launch_error();
  unsigned blocks = (unsigned)((nseg + 255) / 256);
  hipLaunchKernelGGL(table_segments64, dim3(blocks), dim3(256), 0, st, nseg, seg_lo, seg_hi, seg_start);
  return hipGetLastError();
}

hipError_t launch_seed_prime_flags(uint64_t seed, uint64_t j0, uint64_t count, int width, uint8_t *flags,
                                   hipStream_t st) {
  clear_launch_error();
  unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(seed_prime_flags, dim3(blocks), dim3(256), 0, st, seed, j0, count, width, flags);
  return hipGetLastError();
}

hipError_t launch_build_records(const uint64_t *n, const uint64_t *e, uint64_t count, int width, InstRec *out,
                                hipStream_t st) {
  clear_launch_error();
  unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(build_records, dim3(blocks), dim3(256), 0, st, n, e, count, width, out);
  return hipGetLastError();
}

hipError_t launch_position64(const InstRec *inst, const uint32_t *ids, const uint64_t *m0, const uint64_t *ta,
                             const uint64_t *tb, uint64_t count, const uint64_t *u_lo, const uint64_t *u_hi,
                             const uint64_t *u_s, uint64_t *m64, hipStream_t st) {
  clear_launch_error();
  if (count == 0) return hipSuccess;
  unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(position64_kernel, dim3(blocks), dim3(256), 0, st, inst, ids, m0, ta, tb, count, u_lo, u_hi, u_s,
                     m64);
  return hipGetLastError();
}

hipError_t launch_tiles64_reduce(const GenArgs &A, uint64_t units64, unsigned max_blocks, hipStream_t st) {
  clear_launch_error();
  if (units64 == 0) return hipSuccess;
  const uint64_t want = (units64 + 3) / 4;
  const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, max_blocks));
  hipLaunchKernelGGL(reduce64_kernel, dim3(blocks), dim3(256), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_tiles64_table(const GenArgs &A, uint64_t nreq64, hipStream_t st) {
  clear_launch_error();
  if (nreq64 == 0) return hipSuccess;
  if (nreq64 > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tab64_kernel, dim3((unsigned)nreq64), dim3(64), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_tiles64_scan(const GenArgs &A, uint64_t nreq64, hipStream_t st) {
  clear_launch_error();
  if (nreq64 == 0) return hipSuccess;
  if (nreq64 > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan64_kernel, dim3((unsigned)nreq64), dim3(kScanThreads), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_skip_total64(uint64_t t, uint64_t count, uint64_t n, const LaneMul *lm, uint64_t *partial,
                               unsigned blocks, uint64_t extra, int sign, uint64_t *m, hipStream_t st) {
  clear_launch_error();
  if (blocks == 0) return hipErrorInvalidValue;
  if (count > 0) {
    hipLaunchKernelGGL(skip_total64_kernel, dim3(blocks), dim3(256), 0, st, t, count, n, lm, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(skip_total64_apply, dim3(1), dim3(64), 0, st, partial, count > 0 ? (uint64_t)blocks * 4 : 0, n,
                     extra, sign, m);
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
  clear_launch_error();
  bool ok = has64 ? launch_pb<true>(A, grid, block, unroll, st) : launch_pb<false>(A, grid, block, unroll, st);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_plain(const GenArgs &A, uint64_t r, unsigned grid, int unroll, bool has64, hipStream_t st) {
  clear_launch_error();
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
