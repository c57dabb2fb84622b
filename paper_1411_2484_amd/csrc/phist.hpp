// Partitioned histograms for gfx950.  A global atomic per histogram entry
// runs at the device's atomic rate (about 2.7e10 per second, whatever the
// scope or locality), so large histograms are built in three stages:
//   1. scatter (inside the producing kernel): a workgroup ranks its keys by
//      partition (2^15 cells each) with LDS atomics, reserves room in every
//      partition's bucket with one global atomic per partition, and writes
//      the 15-bit cell offsets (uint16) into the buckets;
//   2. count: one workgroup per (partition, slice of its bucket) counts the
//      offsets in a 128 KB LDS histogram and stores the counts;
//   3. add: the per-slice counts are summed into the uint64 histogram and the
//      bucket fill counters are cleared for the next round.
// Atomics on one address serialise (about 5e7 per second), and every
// workgroup reserves in every partition, so each partition's bucket is split
// into nsub sub-buckets with fill counters of their own, and a workgroup
// reserves in sub-bucket blockIdx.x % nsub.  A sub-bucket that runs full
// sends its surplus keys straight to the histogram with global atomics, so
// the result is exact for any key distribution.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace phprng {
namespace ph {

constexpr int kPartBits = 15;
constexpr uint32_t kPartCells = 1u << kPartBits;
constexpr uint32_t kNoKey = 0xffffffffu;

// npart * nsub * cap < 2^32: the scatter indexes the data with 32 bits.
struct PartSet {
  uint16_t *data;                     // [npart][nsub][cap] cell offsets (16-byte aligned, cap a multiple of 8)
  uint32_t *fill;                     // [npart][nsub] entries written this round
  unsigned long long *const *hist;    // [npart] first cell of each partition in its histogram
  const uint32_t *ncell;              // [npart] cells of each partition (<= 2^15)
  uint32_t *slices;                   // [npart][nslice][2^15] stage-2 counts
  uint32_t npart, cap, nslice, nsub;  // cap: entries per sub-bucket; nsub a power of two <= 256
};

// Stage 1 for keys held in registers: key[it] of thread t is item t + it * NT;
// keys are (partition << 15) | offset with partition in [p0, p0 + np), or
// kNoKey.  The keys are sorted by partition in LDS before they leave, so that
// the bucket writes of a wave fall in one or two contiguous runs instead of
// one narrow store per partition.  cnt, off and base are LDS arrays of np
// words, stage an LDS array of NT * K words; np <= 8 * 64.  Ends with a barrier.
template <int NT, int K>
__device__ __forceinline__ void scatter_staged(const uint32_t (&key)[K], const PartSet &P, uint32_t p0, uint32_t np,
                                               uint32_t *cnt, uint32_t *off, uint32_t *base, uint32_t *stage) {
  for (uint32_t i = threadIdx.x; i < np; i += NT) cnt[i] = 0;
  __syncthreads();
  uint32_t rank[K];
#pragma unroll
  for (int it = 0; it < K; ++it)
    rank[it] = key[it] != kNoKey ? atomicAdd(&cnt[(key[it] >> kPartBits) - p0], 1u) : 0u;
  __syncthreads();
  // bucket reservations by all threads at once (one round trip of returning
  // global atomics), and the exclusive scan of the counts by the first wave
  // (up to 8 per lane)
  __shared__ uint32_t total;
  const uint32_t sub = blockIdx.x & (P.nsub - 1);
  for (uint32_t i = threadIdx.x; i < np; i += NT) {
    const uint32_t c = cnt[i];
    base[i] = c ? atomicAdd(&P.fill[(p0 + i) * P.nsub + sub], c) : 0u;
  }
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x;
    const uint32_t per = (np + 63) / 64;
    uint32_t local = 0;
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = lane * per + k;
      if (i < np) local += cnt[i];
    }
    uint32_t incl = local;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(incl, d);
      if ((int)lane >= d) incl += v;
    }
    uint32_t run = incl - local;
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = lane * per + k;
      if (i < np) {
        off[i] = run;
        run += cnt[i];
      }
    }
    if (lane == 63) total = incl;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < K; ++it)
    if (key[it] != kNoKey) stage[off[(key[it] >> kPartBits) - p0] + rank[it]] = key[it];
  // meanwhile, per partition: base becomes the data index of the staged key
  // at position 0 (index = base + staged position, modulo 2^32), and cnt the
  // staged position where the keys that do not fit the sub-bucket begin
  for (uint32_t i = threadIdx.x; i < np; i += NT) {
    const uint32_t b = base[i], o = off[i], c = cnt[i];
    const uint32_t room = P.cap > b ? P.cap - b : 0u;
    base[i] = ((p0 + i) * P.nsub + sub) * P.cap + b - o;
    cnt[i] = o + (c < room ? c : room);
  }
  __syncthreads();
  const uint32_t n = total;
  for (uint32_t i = threadIdx.x; i < n; i += NT) {
    const uint32_t k = stage[i];
    const uint32_t q = (k >> kPartBits) - p0;
    const uint32_t o = k & (kPartCells - 1);
    if (i < cnt[q])
      P.data[base[q] + i] = (uint16_t)o;
    else
      atomicAdd(&P.hist[p0 + q][o], 1ull);
  }
  __syncthreads();
}

hipError_t launch_count(const PartSet &P, hipStream_t st);
hipError_t launch_add(const PartSet &P, hipStream_t st);

}  // namespace ph
}  // namespace phprng
