// Full-period local pattern analysis of Sec. III on gfx950: the histogram of
// the D-1 ciphertexts that follow every first point of a window, over every
// skip of the period, and its chi-square against the uniform model.
//
// Over one period every pair (m_k, s_k) occurs once, so the windows whose
// first point c lies in [x0, x0 + l0) are enumerated by c and the skip s of
// the next step: m = c^d mod n, then (m + s)^e, (m + s + (a s mod p))^e, ...
// One workgroup takes one first point and 16384 consecutive skips; each
// thread decrypts its first point once (a 32-bit exponent chain) and then
// runs the cheap forward chain per skip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "arith.hpp"
#include "hostmath.hpp"
#include "phprng.h"
#include "stats.hpp"

namespace phprng {
namespace pat {

constexpr uint32_t kChunk = 256 * 64;  // skips per workgroup
constexpr uint64_t kMaxCells = 1ull << 28;
constexpr unsigned kChiBlocks = 1024;
constexpr uint64_t kMaxGroups = 1ull << 22;  // workgroups per pattern launch

struct PatArgs {
  uint32_t n, ninv, kc, kd;  // kc = 2^(32 e) mod n, kd = 2^(32 d) mod n
  uint64_t e, d;
  int ebits, dbits;
  uint32_t x0, bins;
  uint64_t s_lo, s_hi, nchunks;
  double binscale;  // RN(bins / n)
  unsigned long long *hist;
};

// floor(c bins / n): a binary64 estimate within one of the answer, then one
// exact integer correction.
__device__ __forceinline__ uint32_t cell_bin(uint32_t c, const PatArgs &A) {
  uint32_t q = (uint32_t)((double)c * A.binscale);
  const uint64_t x = (uint64_t)c * A.bins;
  const uint64_t qn = (uint64_t)q * A.n;
  if (qn > x)
    --q;
  else if (qn + A.n <= x)
    ++q;
  return q;
}

template <int EK, int D>
__global__ __launch_bounds__(256) void pattern_kernel(PatArgs A) {
  const uint64_t i = blockIdx.x / A.nchunks;
  const uint64_t ch = blockIdx.x - i * A.nchunks;
  const uint32_t m = dev::encrypt32<0>(A.x0 + (uint32_t)i, A.n, A.ninv, A.kd, A.d, A.dbits);
  const uint64_t s0 = A.s_lo + ch * kChunk + threadIdx.x;
  for (uint32_t it = 0; it < kChunk / 256; ++it) {
    const uint64_t s = s0 + (uint64_t)it * 256;
    if (s >= A.s_hi) break;
    uint32_t sk = (uint32_t)s;
    uint32_t mk = dev::addmod32(m, sk, A.n);
    uint32_t cell = cell_bin(dev::encrypt32<EK>(mk, A.n, A.ninv, A.kc, A.e, A.ebits), A);
#pragma unroll
    for (int j = 2; j < D; ++j) {
      sk = dev::mulmod_p31(sk, kA32);
      mk = dev::addmod32(mk, sk, A.n);
      cell = cell * A.bins + cell_bin(dev::encrypt32<EK>(mk, A.n, A.ninv, A.kc, A.e, A.ebits), A);
    }
    atomicAdd(&A.hist[cell], 1ull);
  }
}

// chi^2 against E = T prod_j (w_{b_j} / n), w_b = ceil((b+1) n / B) - ceil(b n / B):
// per-block partial sums in a fixed order, then one block over the partials.
__global__ __launch_bounds__(256) void pattern_chi2_kernel(const unsigned long long *hist, uint64_t ncell, int dim,
                                                           uint64_t bins, uint64_t n, double tuples,
                                                           double *part, unsigned long long *part_tot) {
  __shared__ double sd[256];
  __shared__ unsigned long long su[256];
  double acc = 0.0;
  unsigned long long tot = 0;
  for (uint64_t cell = (uint64_t)blockIdx.x * 256 + threadIdx.x; cell < ncell; cell += (uint64_t)gridDim.x * 256) {
    double ex = tuples;
    uint64_t rest = cell, div = 1;
    for (int j = 2; j < dim; ++j) div *= bins;
    for (int j = 1; j < dim; ++j) {  // most significant digit first
      const uint64_t b = rest / div;
      rest -= b * div;
      div = div > 1 ? div / bins : 1;
      const uint64_t lo = (b * n + bins - 1) / bins, hi = ((b + 1) * n + bins - 1) / bins;
      ex *= (double)(hi - lo) / (double)n;
    }
    const unsigned long long o = hist[cell];
    const double dlt = (double)o - ex;
    acc += dlt * dlt / ex;
    tot += o;
  }
  sd[threadIdx.x] = acc;
  su[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      su[threadIdx.x] += su[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sd[0];
    part_tot[blockIdx.x] = su[0];
  }
}

__global__ __launch_bounds__(256) void pattern_sum_kernel(double *part, unsigned long long *part_tot, unsigned np) {
  __shared__ double sd[256];
  __shared__ unsigned long long su[256];
  double acc = 0.0;
  unsigned long long tot = 0;
  for (unsigned i = threadIdx.x; i < np; i += 256) {
    acc += part[i];
    tot += part_tot[i];
  }
  sd[threadIdx.x] = acc;
  su[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      su[threadIdx.x] += su[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[0] = sd[0];
    part_tot[0] = su[0];
  }
}

template <int EK>
hipError_t launch_dim(const PatArgs &A, unsigned grid, int dim, hipStream_t st) {
  switch (dim) {
    case 2: pattern_kernel<EK, 2><<<grid, 256, 0, st>>>(A); break;
    case 3: pattern_kernel<EK, 3><<<grid, 256, 0, st>>>(A); break;
    case 4: pattern_kernel<EK, 4><<<grid, 256, 0, st>>>(A); break;
    default: pattern_kernel<EK, 5><<<grid, 256, 0, st>>>(A); break;
  }
  return hipGetLastError();
}

int bit_length(uint64_t x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

phprng_status validate(const phprng_pattern *P, uint64_t *ncell) {
  if (!P) return PHPRNG_E_INVALID;
  phprng_status st = phprng_check_instance(32, P->n, P->e);
  if (st != PHPRNG_OK) return st;
  if (P->dim < 2 || P->dim > 5 || P->bins < 1) return PHPRNG_E_INVALID;
  uint64_t cells = 1;
  for (uint32_t j = 1; j < P->dim; ++j) {
    cells *= P->bins;
    if (cells > kMaxCells) return PHPRNG_E_RANGE;
  }
  if (P->l0 < 1 || P->x0 >= P->n || P->l0 > P->n - P->x0) return PHPRNG_E_RANGE;
  if (P->s_lo < 1 || P->s_hi <= P->s_lo || P->s_hi > kP32) return PHPRNG_E_RANGE;
  *ncell = cells;
  return PHPRNG_OK;
}

}  // namespace pat
}  // namespace phprng

using namespace phprng;

extern "C" {

phprng_status phprng_pattern_histogram(const phprng_pattern *P, uint64_t *hist, void *stream) {
  uint64_t ncell = 0;
  phprng_status st = pat::validate(P, &ncell);
  if (st != PHPRNG_OK) return st;
  if (!hist) return PHPRNG_E_INVALID;
  pat::PatArgs A;
  const uint32_t n = (uint32_t)P->n;
  A.n = n;
  uint32_t inv = n;
  for (int i = 0; i < 5; ++i) inv *= 2u - n * inv;
  A.ninv = inv;
  Mont64 M(P->n);
  const uint64_t R = (1ull << 32) % P->n;
  A.e = P->e;
  A.d = inverse_mod(P->e, P->n - 1);
  A.kc = (uint32_t)M.powmod(R, A.e);
  A.kd = (uint32_t)M.powmod(R, A.d);
  A.ebits = pat::bit_length(A.e);
  A.dbits = pat::bit_length(A.d);
  A.x0 = (uint32_t)P->x0;
  A.bins = P->bins;
  A.s_lo = P->s_lo;
  A.s_hi = P->s_hi;
  A.nchunks = (P->s_hi - P->s_lo + pat::kChunk - 1) / pat::kChunk;
  A.binscale = (double)P->bins / (double)P->n;
  A.hist = reinterpret_cast<unsigned long long *>(hist);
  // one launch per batch of first points, each within 2^22 workgroups (a
  // dispatch counts its work-items in 32 bits)
  const uint64_t per_launch = std::max<uint64_t>(1, pat::kMaxGroups / A.nchunks);
  hipStream_t s = (hipStream_t)stream;
  for (uint64_t i0 = 0; i0 < P->l0; i0 += per_launch) {
    const uint64_t cnt = std::min<uint64_t>(per_launch, P->l0 - i0);
    pat::PatArgs B = A;
    B.x0 = (uint32_t)(P->x0 + i0);
    const unsigned grid = (unsigned)(cnt * A.nchunks);
    hipError_t e;
    switch (P->e) {
      case 3: e = pat::launch_dim<3>(B, grid, P->dim, s); break;
      case 5: e = pat::launch_dim<5>(B, grid, P->dim, s); break;
      case 9: e = pat::launch_dim<9>(B, grid, P->dim, s); break;
      case 17: e = pat::launch_dim<17>(B, grid, P->dim, s); break;
      default: e = pat::launch_dim<0>(B, grid, P->dim, s); break;
    }
    if (e != hipSuccess) return PHPRNG_E_DEVICE;
  }
  return PHPRNG_OK;
}

phprng_status phprng_pattern_chi2(const phprng_pattern *P, const uint64_t *hist, double *chi2, double *p_value,
                                  uint64_t *total, void *stream) {
  uint64_t ncell = 0;
  phprng_status st = pat::validate(P, &ncell);
  if (st != PHPRNG_OK) return st;
  if (!hist) return PHPRNG_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = (unsigned)std::min<uint64_t>(pat::kChiBlocks, (ncell + 255) / 256);
  void *scratch = nullptr;
  hipError_t e = hipMallocAsync(&scratch, blocks * 16, s);
  if (e != hipSuccess) return PHPRNG_E_NOMEM;
  double *part = (double *)scratch;
  unsigned long long *ptot = (unsigned long long *)((char *)scratch + blocks * 8);
  const double tuples = (double)P->l0 * (double)(P->s_hi - P->s_lo);
  pat::pattern_chi2_kernel<<<blocks, 256, 0, s>>>(reinterpret_cast<const unsigned long long *>(hist), ncell,
                                                   (int)P->dim, P->bins, P->n, tuples, part, ptot);
  pat::pattern_sum_kernel<<<1, 256, 0, s>>>(part, ptot, blocks);
  double c2 = 0;
  unsigned long long tot = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&c2, part, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&tot, ptot, 8, hipMemcpyDeviceToHost, s);
  hipError_t fe = hipFreeAsync(scratch, s);
  if (e == hipSuccess) e = fe;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return PHPRNG_E_DEVICE;
  if (chi2) *chi2 = c2;
  if (total) *total = tot;
  if (p_value) {
    double Pl = 0, Q = 0;
    gamma_pq(0.5 * (double)(ncell - 1), 0.5 * c2, &Pl, &Q);
    *p_value = ncell > 1 ? (Pl < Q ? Pl : Q) : 0.0;
  }
  return PHPRNG_OK;
}

}  // extern "C"
