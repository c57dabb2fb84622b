// gfx950 kernels of the statistical battery (the chi-square tests of the
// paper's Tests section): histograms of the frequency, serial, poker,
// collision, runs and Fourier tests over blocks of 2^20 uniforms, the
// chi-square reduction, and the interstream interleave.
#include "battery.hpp"

namespace phprng {
namespace bat {

namespace {

// Bin of a uniform among B equal bins, clamped so that R = 1.0 (possible for
// 64-bit moduli) falls in the last one.
__device__ __forceinline__ uint32_t bin_of(double x, uint32_t b) {
  const uint32_t u = (uint32_t)floor(x * (double)b);
  return u < b ? u : b - 1;
}

// Poker hand category from the number of equal pairs among the five digits:
// 0 all different, 1 one pair, 2 two pairs, 3 three of a kind, 4 full house,
// 6 four of a kind, 10 five of a kind.
__device__ __forceinline__ uint32_t poker_cat(const uint32_t d[5]) {
  uint32_t pairs = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int k = i + 1; k < 5; ++k) pairs += d[i] == d[k];
  return pairs <= 4 ? pairs : (pairs == 6 ? 5u : 6u);
}

// Keys of one test for one tile, held in registers for the partitioned
// histogram: item j = threadIdx.x + it * 256 is the j-th D-tuple of the tile
// (D = 1: the j-th uniform), its key the partition-space offset of the test
// plus its cell (first element most significant).
template <int D, uint32_t B, int K>
__device__ __forceinline__ void tuple_keys(const double *t, uint32_t len, uint32_t key0, uint32_t *key) {
  const uint32_t ntup = len / D;
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const uint32_t j = threadIdx.x + it * 256;
    uint32_t cell = 0;
    if (j < ntup) {
#pragma unroll
      for (int i = 0; i < D; ++i) cell = cell * B + bin_of(t[j * D + i], B);
    }
    key[it] = j < ntup ? key0 + cell : ph::kNoKey;
  }
}

// Registers per thread for the keys of one tile: 15 + 8 + 5 + 4 + 3.
constexpr int kK1 = kHistTile / 256, kK2 = (kHistTile / 2 + 255) / 256, kK3 = (kHistTile / 3 + 255) / 256;
constexpr int kK4 = (kHistTile / 4 + 255) / 256, kK5 = (kHistTile / 5 + 255) / 256;
constexpr int kKeys = kK1 + kK2 + kK3 + kK4 + kK5;

// One tile of one block: frequency and serial D = 2..5 keys into the
// partitioned histograms, the poker histogram, and the bits R > 1/2 packed
// one 64-bit word per 64 uniforms (for the runs test).
__global__ __launch_bounds__(256) void hist_kernel(const double *__restrict__ r, ph::PartSet P, BatteryParts bp,
                                                   unsigned long long *poker_hist, uint64_t *__restrict__ bits) {
  // the tile of uniforms, later reused as the key staging area of the scatter
  __shared__ __align__(16) uint32_t buf[kKeys * 256];
  static_assert(kKeys * 256 * 4 >= kHistTile * 8, "staging area must hold the tile");
  __shared__ uint32_t poker[kPokerCats];
  __shared__ uint32_t cnt[kMaxParts], poff[kMaxParts], base[kMaxParts];
  double *t = reinterpret_cast<double *>(buf);
  const uint32_t tile = blockIdx.x % kHistTilesPerBlock;
  const uint64_t blk = blockIdx.x / kHistTilesPerBlock;
  const uint32_t off = tile * kHistTile;
  const uint32_t len = (kBlock - off) < kHistTile ? (kBlock - off) : kHistTile;  // 3840 or 256
  const uint64_t base_i = blk * kBlock + off;
  if (threadIdx.x < kPokerCats) poker[threadIdx.x] = 0;
  // len is a multiple of 256, so every wave covers 64 consecutive uniforms per step
  for (uint32_t i = threadIdx.x; i < len; i += 256) {
    const double x = r[base_i + i];
    t[i] = x;
    const uint64_t word = __ballot(x > 0.5);
    if ((threadIdx.x & 63) == 0) bits[(base_i + i) >> 6] = word;
  }
  __syncthreads();
  const uint32_t nhand = len / 5;
  for (uint32_t j = threadIdx.x; j < nhand; j += 256) {
    uint32_t d[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = bin_of(t[j * 5 + i], 10);
    atomicAdd(&poker[poker_cat(d)], 1u);
  }
  // all five tests' keys of the tile in registers, then one scatter over the
  // partition space (its first barrier orders the last reads of the tile
  // before the staging area is overwritten)
  uint32_t key[kKeys];
  tuple_keys<1, kFreqBins, kK1>(t, len, bp.p0[0] << ph::kPartBits, key);
  tuple_keys<2, kAxis2, kK2>(t, len, bp.p0[1] << ph::kPartBits, key + kK1);
  tuple_keys<3, kAxis3, kK3>(t, len, bp.p0[2] << ph::kPartBits, key + kK1 + kK2);
  tuple_keys<4, kAxis4, kK4>(t, len, bp.p0[3] << ph::kPartBits, key + kK1 + kK2 + kK3);
  tuple_keys<5, kAxis5, kK5>(t, len, bp.p0[4] << ph::kPartBits, key + kK1 + kK2 + kK3 + kK4);
  ph::scatter_staged<256, kKeys>(key, P, 0, P.npart, cnt, poff, base, buf);
  if (threadIdx.x < kPokerCats && poker[threadIdx.x])
    atomicAdd(&poker_hist[threadIdx.x], (unsigned long long)poker[threadIdx.x]);
}

// One collision trial per workgroup: 2^14 uniforms into 2^20 urns held as a
// 128 KB bitmap in LDS; a ball that finds its bit already set is a collision.
__global__ __launch_bounds__(1024) void collision_kernel(const double *__restrict__ r, unsigned long long *hist) {
  __shared__ uint32_t bm[kCollUrns / 32];
  __shared__ uint32_t total;
  const double *src = r + (uint64_t)blockIdx.x * kCollBalls;
  for (uint32_t i = threadIdx.x; i < kCollUrns / 32; i += 1024) bm[i] = 0;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  uint32_t coll = 0;
  for (uint32_t i = threadIdx.x; i < kCollBalls; i += 1024) {
    const uint32_t u = bin_of(src[i], kCollUrns);
    const uint32_t bit = 1u << (u & 31);
    const uint32_t old = atomicOr(&bm[u >> 5], bit);
    coll += (old & bit) ? 1u : 0u;
  }
  for (int s = 32; s > 0; s >>= 1) coll += __shfl_xor(coll, s);
  if ((threadIdx.x & 63) == 0) atomicAdd(&total, coll);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t c = total < kCollLo ? kCollLo : (total > kCollHi ? kCollHi : total);
    atomicAdd(&hist[c - kCollLo], 1ull);
  }
}

// One thread per 64-bit word of run bits: every run that starts in the word
// (a position whose bit differs from its predecessor's) is measured up to the
// next change, scanning later words of the block if needed; runs that reach
// the end of the block, and the block's first run, are not interior and are
// not counted.
__global__ __launch_bounds__(256) void runs_kernel(const uint64_t *__restrict__ bits, uint64_t nwords,
                                                   unsigned long long *hist) {
  __shared__ uint32_t h[kRunsCats];
  if (threadIdx.x < kRunsCats) h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (w < nwords) {
    const uint32_t wi = (uint32_t)(w & (kWordsPerBlock - 1));
    const uint64_t word = bits[w];
    const uint64_t prev = wi ? (bits[w - 1] >> 63) : (word & 1);
    uint64_t ch = word ^ ((word << 1) | prev);
    while (ch) {
      const uint32_t i = __builtin_ctzll(ch);
      ch &= ch - 1;
      uint32_t len = 0;
      if (ch) {
        len = __builtin_ctzll(ch) - i;
      } else {
        uint32_t run = 64 - i;
        uint64_t pw = word;
        bool found = false;
        for (uint32_t wj = wi + 1; wj < kWordsPerBlock; ++wj) {
          const uint64_t nw = bits[w + (wj - wi)];
          const uint64_t c2 = nw ^ ((nw << 1) | (pw >> 63));
          if (c2) {
            len = run + __builtin_ctzll(c2);
            found = true;
            break;
          }
          run += 64;
          pw = nw;
        }
        if (!found) break;
      }
      atomicAdd(&h[(len < kRunsCats ? len : kRunsCats) - 1], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < kRunsCats && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place decimation-in-frequency transform with the positive exponent on
// NCOL columns of length LEN (512 or 1024) held in LDS (column c at re/im +
// c * STRIDE): radix-4 stages, then one radix-2 stage when LEN is not a power
// of 4.  Position p ends up holding frequency out_freq<LEN>(p).
template <int LEN, int NCOL, int STRIDE, int NT>
__device__ void lds_fft(double *re, double *im, const double2 *__restrict__ w1024) {
  for (int len = LEN; len >= 4; len >>= 2) {
    const int q = len >> 2;
    const int step = 1024 / len;
    for (int b = threadIdx.x; b < NCOL * (LEN / 4); b += NT) {
      const int col = b / (LEN / 4);
      const int bb = b % (LEN / 4);
      const int i = bb % q;
      const int p0 = col * STRIDE + (bb / q) * len + i;
      const double a0r = re[p0], a0i = im[p0];
      const double a1r = re[p0 + q], a1i = im[p0 + q];
      const double a2r = re[p0 + 2 * q], a2i = im[p0 + 2 * q];
      const double a3r = re[p0 + 3 * q], a3i = im[p0 + 3 * q];
      const double b0r = a0r + a2r, b0i = a0i + a2i;
      const double b1r = a0r - a2r, b1i = a0i - a2i;
      const double b2r = a1r + a3r, b2i = a1i + a3i;
      const double b3r = -(a1i - a3i), b3i = a1r - a3r;  // i (a1 - a3)
      re[p0] = b0r + b2r;
      im[p0] = b0i + b2i;
      const double2 y1 = cmul(make_double2(b1r + b3r, b1i + b3i), w1024[i * step]);
      const double2 y2 = cmul(make_double2(b0r - b2r, b0i - b2i), w1024[2 * i * step]);
      const double2 y3 = cmul(make_double2(b1r - b3r, b1i - b3i), w1024[3 * i * step]);
      re[p0 + q] = y1.x;
      im[p0 + q] = y1.y;
      re[p0 + 2 * q] = y2.x;
      im[p0 + 2 * q] = y2.y;
      re[p0 + 3 * q] = y3.x;
      im[p0 + 3 * q] = y3.y;
    }
    __syncthreads();
  }
  if ((LEN & 0x55555555) == 0) {  // LEN = 2 * 4^k: last stage is radix 2
    for (int b = threadIdx.x; b < NCOL * (LEN / 2); b += NT) {
      const int p0 = (b / (LEN / 2)) * STRIDE + 2 * (b % (LEN / 2));
      const double a0r = re[p0], a0i = im[p0], a1r = re[p0 + 1], a1i = im[p0 + 1];
      re[p0] = a0r + a1r;
      im[p0] = a0i + a1i;
      re[p0 + 1] = a0r - a1r;
      im[p0 + 1] = a0i - a1i;
    }
    __syncthreads();
  }
}

template <int LEN>
__device__ __forceinline__ int out_freq(int p) {
  int k = 0, mul = 1, len = LEN;
  while (len >= 4) {
    const int q = len >> 2;
    k += (p / q) * mul;
    p %= q;
    mul *= 4;
    len = q;
  }
  if (len == 2) k += p * mul;
  return k;
}

template <int LEN>
__device__ __forceinline__ int pos_of(int k) {
  int p = 0, len = LEN;
  while (len >= 4) {
    const int q = len >> 2;
    p += (k & 3) * q;
    k >>= 2;
    len = q;
  }
  if (len == 2) p += k;
  return p;
}

constexpr int kP1Stride = kFftN1 + 2;  // LDS column stride (doubles), spreads banks

// Pass 1 of the four-step transform of z_n = (x_2n - 1/2) + i (x_2n+1 - 1/2),
// n = 1024 j1 + j2: the 512-point transforms over j1 of kFftCols columns j2,
// times exp(2 pi i j2 k1 / 2^19), written as rows Y[k1][j2].
__global__ __launch_bounds__(256) void fft_pass1_kernel(const double *__restrict__ r, double2 *__restrict__ y,
                                                        Twiddles tw) {
  __shared__ double re[kFftCols * kP1Stride], im[kFftCols * kP1Stride];
  const uint64_t blk = blockIdx.x / kFftPass1Groups;
  const uint32_t c0 = (blockIdx.x % kFftPass1Groups) * kFftCols;
  const double2 *src = reinterpret_cast<const double2 *>(r + blk * kBlock);
  for (uint32_t e = threadIdx.x; e < kFftCols * kFftN1; e += 256) {
    const uint32_t j1 = e / kFftCols, col = e % kFftCols;
    const double2 v = src[(uint64_t)j1 * kFftN2 + c0 + col];
    re[col * kP1Stride + j1] = v.x - 0.5;
    im[col * kP1Stride + j1] = v.y - 0.5;
  }
  __syncthreads();
  lds_fft<kFftN1, kFftCols, kP1Stride, 256>(re, im, tw.w1024);
  double2 *dst = y + blk * (uint64_t)kFftN;
  for (uint32_t e = threadIdx.x; e < kFftCols * kFftN1; e += 256) {
    const uint32_t p = e / kFftCols, col = e % kFftCols;
    const uint32_t k1 = out_freq<kFftN1>(p);
    const uint32_t j2 = c0 + col;
    const uint32_t t = j2 * k1;  // < 2^19
    const double2 w = cmul(tw.fineN[t & 1023], tw.w1024[2 * (t >> 10)]);
    dst[(uint64_t)k1 * kFftN2 + j2] = cmul(make_double2(re[col * kP1Stride + p], im[col * kP1Stride + p]), w);
  }
}

__device__ __forceinline__ uint32_t fourier_cat(double v, double scale) {
  const double u = floor(v * scale);
  const double c = u < -kFourierHalf - 1 ? (double)(-kFourierHalf - 1) : (u > kFourierHalf ? (double)kFourierHalf : u);
  return (uint32_t)(int)(c + kFourierHalf + 1);
}

// Pass 2: the 1024-point transforms of rows k1 and 512 - k1 (rows 0 and 256
// pair with themselves), which give F_k for k = k1 + 512 k2 and the partner
// N - k of each; then the real-input split
//   E = (F_k + conj F_{N-k}) / 2,  O = (F_k - conj F_{N-k}) / (2i),
//   X_k = E + w_M^k O,  X_{N-k} = conj(E - w_M^k O),
// scaled by 1/sqrt(M), and the categories of their real and imaginary parts.
__global__ __launch_bounds__(256) void fft_pass2_kernel(const double2 *__restrict__ y, unsigned long long *hist,
                                                        double *__restrict__ coef, Twiddles tw, double scale) {
  constexpr int L = kFftN2;
  __shared__ double re[2 * L], im[2 * L];
  __shared__ uint32_t h[kFourierCats];
  const uint64_t blk = blockIdx.x / kFftPass2Groups;
  const uint32_t ra = blockIdx.x % kFftPass2Groups;  // 0 .. 256
  const uint32_t rb = (ra == 0 || ra == kFftN1 / 2) ? ra : kFftN1 - ra;
  const double2 *src = y + blk * (uint64_t)kFftN;
  if (threadIdx.x < kFourierCats) h[threadIdx.x] = 0;
  for (uint32_t e = threadIdx.x; e < 2 * L; e += 256) {
    const uint32_t row = e < (uint32_t)L ? ra : rb;
    const double2 v = src[(uint64_t)row * L + (e % L)];
    re[e] = v.x;
    im[e] = v.y;
  }
  __syncthreads();
  lds_fft<L, 2, L, 256>(re, im, tw.w1024);
  const double fs = 1.0 / 1024.0;  // 1 / sqrt(M), exact
  double *cb = coef ? coef + blk * (uint64_t)kBlock : nullptr;
  // Work items: all 1024 k2 of a row pair, k2 = 0..512 for row 0, k2 = 0..511
  // for row 256.  For the rows other than 0 the items walk LDS positions in
  // order (k2 = out_freq(p)); the partner 1023 - k2 then sits at position
  // 1023 - p (complementing every base-4 digit commutes with reversing them),
  // so neither read strides across the banks.  Row 256 takes the positions
  // whose lowest digit is 0 or 1, i.e. k2 < 512.
  const uint32_t nk2 = ra == 0 ? 513u : (ra == kFftN1 / 2 ? 512u : 1024u);
  for (uint32_t j = threadIdx.x; j < nk2; j += 256) {
    uint32_t k, kp, pa, pb;
    if (ra == 0) {
      const uint32_t k2 = j, k2p = (1024 - k2) & 1023;
      k = kFftN1 * k2;
      kp = (kFftN - k) % kFftN;
      pa = pos_of<L>(k2);
      pb = pos_of<L>(k2p);
    } else {
      const uint32_t p = ra == kFftN1 / 2 ? ((j >> 1) << 2) | (j & 1) : j;
      const uint32_t k2 = out_freq<L>(p);
      k = ra + kFftN1 * k2;
      kp = kFftN - k;
      pa = p;
      pb = L + (L - 1 - p);  // row rb sits in the second column (for row 256 it is the same row)
    }
    const double ar = re[pa], ai = im[pa], br = re[pb], bi = im[pb];
    const double er = (ar + br) * 0.5, ei = (ai - bi) * 0.5;
    const double orr = (ai + bi) * 0.5, oi = (br - ar) * 0.5;
    const double2 w = cmul(tw.fineM[k & 1023], tw.w1024[k >> 10]);
    const double tr = orr * w.x - oi * w.y, ti = orr * w.y + oi * w.x;
    const double xr = (er + tr) * fs, xi = (ei + ti) * fs;
    atomicAdd(&h[fourier_cat(xr, scale)], 1u);
    atomicAdd(&h[fourier_cat(xi, scale)], 1u);
    if (cb) {
      cb[2 * k] = xr;
      cb[2 * k + 1] = xi;
    }
    if (kp != k) {  // the partner coefficient, unless it is the same one (k = 0 or N/2)
      const double pr = (er - tr) * fs, pi = -(ei - ti) * fs;
      atomicAdd(&h[fourier_cat(pr, scale)], 1u);
      atomicAdd(&h[fourier_cat(pi, scale)], 1u);
      if (cb) {
        cb[2 * kp] = pr;
        cb[2 * kp + 1] = pi;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kFourierCats && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// One workgroup per test: the total count, then sum (O - E)^2 / E with
// E = total * probability, in a fixed reduction order.
__global__ __launch_bounds__(1024) void chi2_kernel(const Chi2Job *jobs, double *chi2, unsigned long long *total) {
  __shared__ unsigned long long su[1024];
  __shared__ double sd[1024];
  const Chi2Job J = jobs[blockIdx.x];
  unsigned long long s = 0;
  for (uint32_t i = threadIdx.x; i < J.ncat; i += 1024) s += J.counts[i];
  su[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) su[threadIdx.x] += su[threadIdx.x + w];
    __syncthreads();
  }
  const double tot = (double)su[0];
  const double eq = 1.0 / (double)J.ncat;
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < J.ncat; i += 1024) {
    const double ex = tot * (J.probs ? J.probs[i] : eq);
    const double d = (double)J.counts[i] - ex;
    acc += d * d / ex;
  }
  sd[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sd[threadIdx.x] += sd[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    chi2[blockIdx.x] = sd[0];
    total[blockIdx.x] = su[0];
  }
}

// out[t * S + a] = in[a * L + t] through a 64 x 64 LDS tile.
__global__ __launch_bounds__(256) void interleave_kernel(const double *__restrict__ in, double *__restrict__ out,
                                                         uint64_t S, uint64_t L) {
  __shared__ double tile[64][65];
  const uint64_t t0 = (uint64_t)blockIdx.x * 64, a0 = (uint64_t)blockIdx.y * 64;
  for (uint32_t j = threadIdx.y; j < 64; j += 4) {
    const uint64_t a = a0 + j, t = t0 + threadIdx.x;
    if (a < S && t < L) tile[j][threadIdx.x] = in[a * L + t];
  }
  __syncthreads();
  for (uint32_t j = threadIdx.y; j < 64; j += 4) {
    const uint64_t t = t0 + j, a = a0 + threadIdx.x;
    if (a < S && t < L) out[t * S + a] = tile[threadIdx.x][j];
  }
}

}  // namespace

hipError_t launch_hist(const double *r, uint64_t nblocks, const ph::PartSet &P, const BatteryParts &bp,
                       unsigned long long *poker, uint64_t *bits, hipStream_t st) {
  hist_kernel<<<dim3((unsigned)(nblocks * kHistTilesPerBlock)), dim3(256), 0, st>>>(r, P, bp, poker, bits);
  return hipGetLastError();
}

hipError_t launch_collision(const double *r, uint64_t nblocks, unsigned long long *coll, hipStream_t st) {
  collision_kernel<<<dim3((unsigned)(nblocks * (kBlock / kCollBalls))), dim3(1024), 0, st>>>(r, coll);
  return hipGetLastError();
}

hipError_t launch_runs(const uint64_t *bits, uint64_t nblocks, unsigned long long *runs, hipStream_t st) {
  const uint64_t nwords = nblocks * kWordsPerBlock;
  runs_kernel<<<dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, st>>>(bits, nwords, runs);
  return hipGetLastError();
}

hipError_t launch_fft_pass1(const double *r, uint64_t nblocks, double2 *y, Twiddles tw, hipStream_t st) {
  fft_pass1_kernel<<<dim3((unsigned)(nblocks * kFftPass1Groups)), dim3(256), 0, st>>>(r, y, tw);
  return hipGetLastError();
}

hipError_t launch_fft_pass2(const double2 *y, uint64_t nblocks, unsigned long long *fourier, double *coef,
                            Twiddles tw, double scale, hipStream_t st) {
  fft_pass2_kernel<<<dim3((unsigned)(nblocks * kFftPass2Groups)), dim3(256), 0, st>>>(y, fourier, coef, tw, scale);
  return hipGetLastError();
}

hipError_t launch_chi2(const Chi2Job *jobs, int njobs, double *chi2, unsigned long long *total, hipStream_t st) {
  chi2_kernel<<<dim3(njobs), dim3(1024), 0, st>>>(jobs, chi2, total);
  return hipGetLastError();
}

hipError_t launch_interleave(const double *in, double *out, uint64_t nstreams, uint64_t length, hipStream_t st) {
  interleave_kernel<<<dim3((unsigned)((length + 63) / 64), (unsigned)((nstreams + 63) / 64)), dim3(64, 4), 0, st>>>(
      in, out, nstreams, length);
  return hipGetLastError();
}

}  // namespace bat
}  // namespace phprng
