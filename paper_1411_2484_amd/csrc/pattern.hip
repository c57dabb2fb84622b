// Full-period local pattern analysis of Sec. II, Figs. 3-4 on gfx950: the histogram of
// the D-1 ciphertexts that follow every first point of a window, over every
// skip of the period, and its chi-square against the uniform model.
//
// Over one period every pair (m_k, s_k) occurs once, so the windows whose
// first point c lies in [x0, x0 + l0) are enumerated by c and the skip s of
// the next step: m = c^d mod n, then (m + s)^e, (m + s + (a s mod p))^e, ...
// One workgroup takes one first point and 16384 consecutive skips; each
// thread decrypts its first point once (a 32-bit exponent chain) and then
// runs the cheap forward chain per skip.  The cells go through partitioned
// histograms (phist.hpp): a global atomic per tuple would cap the rate at the
// device's atomic throughput.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "arith.hpp"
#include "hostmath.hpp"
#include "phprng.h"
#include "phist.hpp"
#include "stats.hpp"

namespace phprng {
namespace pat {

constexpr uint32_t kChunk = 256 * 64;  // skips per workgroup
constexpr uint32_t kHalf = 256 * 32;   // skips whose keys a workgroup holds in registers at once
constexpr uint32_t kMaxParts = 512;
constexpr uint64_t kMaxCells = (uint64_t)kMaxParts << ph::kPartBits;  // 2^24
constexpr uint64_t kRoundKeys = 1ull << 30;  // keys per bucket round
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
__global__ __launch_bounds__(256) void pattern_kernel(PatArgs A, ph::PartSet P) {
  __shared__ uint32_t cnt[kMaxParts], off[kMaxParts], base[kMaxParts];
  __shared__ uint32_t stage[kHalf];
  const uint64_t i = blockIdx.x / A.nchunks;
  const uint64_t ch = blockIdx.x - i * A.nchunks;
  const uint32_t m = dev::encrypt32<0>(A.x0 + (uint32_t)i, A.n, A.ninv, A.kd, A.d, A.dbits);
  for (uint32_t half = 0; half < kChunk / kHalf; ++half) {
    const uint64_t s0 = A.s_lo + ch * kChunk + half * kHalf + threadIdx.x;
    uint32_t key[kHalf / 256];
#pragma unroll
    for (uint32_t it = 0; it < kHalf / 256; ++it) {
      const uint64_t s = s0 + (uint64_t)it * 256;
      uint32_t sk = (uint32_t)(s < A.s_hi ? s : A.s_lo);  // lanes past the range compute a valid dummy
      uint32_t mk = dev::addmod32(m, sk, A.n);
      uint32_t cell = cell_bin(dev::encrypt32<EK>(mk, A.n, A.ninv, A.kc, A.e, A.ebits), A);
#pragma unroll
      for (int j = 2; j < D; ++j) {
        sk = dev::mulmod_p31(sk, kA32);
        mk = dev::addmod32(mk, sk, A.n);
        cell = cell * A.bins + cell_bin(dev::encrypt32<EK>(mk, A.n, A.ninv, A.kc, A.e, A.ebits), A);
      }
      key[it] = s < A.s_hi ? cell : ph::kNoKey;
    }
    ph::scatter_staged<256, kHalf / 256>(key, P, 0, P.npart, cnt, off, base, stage);
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
hipError_t launch_dim(const PatArgs &A, const ph::PartSet &P, unsigned grid, int dim, hipStream_t st) {
  clear_launch_error();
  switch (dim) {
    case 2: pattern_kernel<EK, 2><<<grid, 256, 0, st>>>(A, P); break;
    case 3: pattern_kernel<EK, 3><<<grid, 256, 0, st>>>(A, P); break;
    case 4: pattern_kernel<EK, 4><<<grid, 256, 0, st>>>(A, P); break;
    default: pattern_kernel<EK, 5><<<grid, 256, 0, st>>>(A, P); break;
  }
  return hipGetLastError();
}

hipError_t launch_ek(const PatArgs &A, const ph::PartSet &P, unsigned grid, int dim, uint64_t e, hipStream_t st) {
  switch (e) {
    case 3: return launch_dim<3>(A, P, grid, dim, st);
    case 5: return launch_dim<5>(A, P, grid, dim, st);
    case 9: return launch_dim<9>(A, P, grid, dim, st);
    case 17: return launch_dim<17>(A, P, grid, dim, st);
    default: return launch_dim<0>(A, P, grid, dim, st);
  }
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
  // Rounds of at most 2^30 keys (and 2^22 workgroups): a round is a batch of
  // first points over the whole skip range, or one first point over a slice
  // of it.  Each round scatters its keys into the partition buckets, then
  // the buckets are counted into the histogram.
  const uint64_t srange = P->s_hi - P->s_lo;
  const uint64_t s_step = srange > pat::kRoundKeys ? pat::kRoundKeys : srange;
  const uint64_t fp_per_round = std::max<uint64_t>(
      1, std::min({P->l0, pat::kRoundKeys / s_step, pat::kMaxGroups / ((s_step + pat::kChunk - 1) / pat::kChunk)}));
  const uint64_t round_keys = fp_per_round * s_step;
  const uint32_t npart = (uint32_t)((ncell + ph::kPartCells - 1) / ph::kPartCells);
  const uint32_t nslice = std::max<uint32_t>(1, 512 / npart);
  const uint32_t nsub = 8;
  // bucket room: the expected share of a full partition over its sub-buckets
  // plus a margin (any surplus is added with atomics)
  const uint64_t share = (round_keys * std::min<uint64_t>(ph::kPartCells, ncell) + ncell - 1) / ncell;
  const uint64_t sub_share = (share + nsub - 1) / nsub;
  const uint32_t cap = (uint32_t)std::min<uint64_t>(sub_share + sub_share / 4 + 4096, 0xfffffff0ull) & ~7u;
  if ((uint64_t)npart * nsub * cap >= (1ull << 32)) return PHPRNG_E_RANGE;  // 32-bit bucket indexing
  const uint64_t bytes_data = ((uint64_t)npart * nsub * cap * 2 + 255) / 256 * 256;
  const uint64_t bytes_slices = (uint64_t)npart * nslice * ph::kPartCells * 4;
  // table: hist pointers[npart] | fill[npart][nsub] | ncell[npart]
  const uint64_t bytes = bytes_data + bytes_slices + (uint64_t)npart * (8 + 4 * nsub + 4);
  hipStream_t s = (hipStream_t)stream;
  void *mem = nullptr;
  if (hipMallocAsync(&mem, bytes, s) != hipSuccess) return PHPRNG_E_NOMEM;
  char *cm = (char *)mem;
  ph::PartSet PS;
  PS.data = (uint16_t *)cm;
  PS.slices = (uint32_t *)(cm + bytes_data);
  // the pointer table first, at a 256-byte aligned offset
  unsigned long long **hist_d = (unsigned long long **)(cm + bytes_data + bytes_slices);
  PS.fill = (uint32_t *)(hist_d + npart);
  uint32_t *ncell_d = PS.fill + (uint64_t)npart * nsub;
  PS.ncell = ncell_d;
  PS.hist = hist_d;
  PS.npart = npart;
  PS.cap = cap;
  PS.nslice = nslice;
  PS.nsub = nsub;
  std::vector<uint32_t> tab32((uint64_t)npart * (nsub + 1), 0);  // fill = 0 | ncell
  std::vector<unsigned long long *> tabp(npart);
  for (uint32_t q = 0; q < npart; ++q) {
    tab32[(uint64_t)npart * nsub + q] =
        (uint32_t)std::min<uint64_t>(ph::kPartCells, ncell - (uint64_t)q * ph::kPartCells);
    tabp[q] = reinterpret_cast<unsigned long long *>(hist) + (uint64_t)q * ph::kPartCells;
  }
  hipError_t e = hipMemcpyAsync(PS.fill, tab32.data(), tab32.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hist_d, tabp.data(), npart * sizeof(void *), hipMemcpyHostToDevice, s);
  for (uint64_t i0 = 0; e == hipSuccess && i0 < P->l0; i0 += fp_per_round) {
    const uint64_t cnt = std::min<uint64_t>(fp_per_round, P->l0 - i0);
    for (uint64_t s_lo = P->s_lo; e == hipSuccess && s_lo < P->s_hi; s_lo += s_step) {
      pat::PatArgs B = A;
      B.x0 = (uint32_t)(P->x0 + i0);
      B.s_lo = s_lo;
      B.s_hi = std::min<uint64_t>(s_lo + s_step, P->s_hi);
      B.nchunks = (B.s_hi - B.s_lo + pat::kChunk - 1) / pat::kChunk;
      e = pat::launch_ek(B, PS, (unsigned)(cnt * B.nchunks), P->dim, P->e, s);
      if (e == hipSuccess) e = ph::launch_count(PS, s);
      if (e == hipSuccess) e = ph::launch_add(PS, s);
    }
  }
  // the host tables above must outlive their asynchronous copies
  hipError_t se = hipStreamSynchronize(s);
  hipError_t fe = hipFreeAsync(mem, s);
  if (e == hipSuccess) e = se;
  if (e == hipSuccess) e = fe;
  return e == hipSuccess ? PHPRNG_OK : PHPRNG_E_DEVICE;
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
  phprng::clear_launch_error();
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
