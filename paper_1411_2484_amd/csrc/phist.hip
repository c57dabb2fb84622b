// Stages 2 and 3 of the partitioned histograms (phist.hpp).
#include "phist.hpp"

#include "arith.hpp"

namespace phprng {
namespace ph {

namespace {

// One workgroup per (partition, slice): count slice s of every sub-bucket
// of the partition in LDS and store the partition's counts for the slice.
__global__ __launch_bounds__(1024) void count_kernel(PartSet P) {
  __shared__ uint32_t c[kPartCells];
  const uint32_t p = blockIdx.x / P.nslice, s = blockIdx.x % P.nslice;
  for (uint32_t i = threadIdx.x; i < kPartCells; i += 1024) c[i] = 0;
  __syncthreads();
  for (uint32_t sb = 0; sb < P.nsub; ++sb) {
    const uint32_t f = P.fill[p * P.nsub + sb];
    const uint32_t fill = f < P.cap ? f : P.cap;
    // slice bounds on 8-entry (16-byte) boundaries, the last slice takes the tail
    const uint32_t lo = (uint32_t)((uint64_t)fill * s / P.nslice) & ~7u;
    const uint32_t hi = s + 1 == P.nslice ? fill : (uint32_t)((uint64_t)fill * (s + 1) / P.nslice) & ~7u;
    const uint16_t *d = P.data + ((uint64_t)p * P.nsub + sb) * P.cap;  // cap is a multiple of 8
    // 16-byte loads, kU of them in flight per thread before any is counted:
    // a loop that waits for each load pays the full memory latency per step
    constexpr uint32_t kU = 8;
    const uint4 *dv = reinterpret_cast<const uint4 *>(d);
    const uint32_t vend = hi / 8;
    for (uint32_t v0 = lo / 8 + threadIdx.x; v0 < vend; v0 += 1024 * kU) {
      uint4 w[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        const uint32_t v = v0 + 1024 * u;
        w[u] = v < vend ? dv[v] : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        if (v0 + 1024 * u >= vend) break;
        const uint32_t q[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          atomicAdd(&c[q[k] & 0xffffu], 1u);
          atomicAdd(&c[q[k] >> 16], 1u);
        }
      }
    }
    for (uint32_t i = (hi & ~7u) + threadIdx.x; i < hi; i += 1024) atomicAdd(&c[d[i]], 1u);
  }
  __syncthreads();
  uint32_t *out = P.slices + ((uint64_t)p * P.nslice + s) * kPartCells;
  const uint32_t nc = P.ncell[p];
  for (uint32_t i = threadIdx.x; i < nc; i += 1024) out[i] = c[i];
}

// hist[p][j] += sum over slices; the first nsub threads of each partition
// clear its fill counters (stage 2 has finished reading them).
__global__ __launch_bounds__(256) void add_kernel(PartSet P) {
  const uint32_t p = blockIdx.x / (kPartCells / 256);
  const uint32_t j = (blockIdx.x % (kPartCells / 256)) * 256 + threadIdx.x;
  if (j < P.nsub) P.fill[p * P.nsub + j] = 0;
  if (j >= P.ncell[p]) return;
  const uint32_t *in = P.slices + (uint64_t)p * P.nslice * kPartCells + j;
  unsigned long long s = 0;
  for (uint32_t k = 0; k < P.nslice; ++k) s += in[(uint64_t)k * kPartCells];
  if (s) P.hist[p][j] += s;
}

}  // namespace

hipError_t launch_count(const PartSet &P, hipStream_t st) {
  clear_launch_error();
  count_kernel<<<dim3(P.npart * P.nslice), dim3(1024), 0, st>>>(P);
  return hipGetLastError();
}

hipError_t launch_add(const PartSet &P, hipStream_t st) {
  clear_launch_error();
  add_kernel<<<dim3(P.npart * (kPartCells / 256)), dim3(256), 0, st>>>(P);
  return hipGetLastError();
}

}  // namespace ph
}  // namespace phprng
