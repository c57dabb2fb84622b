// gfx950 kernels of the statistical battery (the chi-square tests of the
// paper's Tests section): histograms of the frequency, serial, poker,
// collision, runs and Fourier tests over blocks of 2^20 uniforms, the
// chi-square reduction, and the interstream interleave.
#include "battery.hpp"

#include "arith.hpp"
#include "wavefft.hpp"

namespace phprng {
namespace bat {

namespace {

// Bin of a uniform among B equal bins, clamped so that R = 1.0 (possible for
// 64-bit moduli) falls in the last one.
__device__ __forceinline__ uint32_t bin_of(double x, uint32_t b) {
  const uint32_t u = (uint32_t)floor(x * (double)b);
  return u < b ? u : b - 1;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  const uint32_t lo = __shfl_xor((int)(uint32_t)v, mask, 64);
  const uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
  return ((uint64_t)hi << 32) | lo;
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
// histogram: item j = threadIdx.x + it * kHistThreads is the j-th D-tuple of
// the tile (D = 1: the j-th uniform), its key the partition-space offset of
// the test plus its cell (first element most significant).  The cells come
// from each uniform's bins, found once per uniform: b20 among 2^20 bins, whose
// top 10, 5 and 4 bits are the bins among 1024, 32 and 16 (x 2^k is exact, so
// floor(x 2^k) = floor(x 2^20) >> (20 - k)), and b100 among 100.
template <int D, int K>
__device__ __forceinline__ void tuple_keys(const uint32_t *b20, const uint8_t *b100, uint32_t len, uint32_t key0,
                                           uint32_t *key) {
  static_assert(kFreqBins == 1u << 20 && kAxis2 == 1024 && kAxis3 == 100 && kAxis4 == 32 && kAxis5 == 16,
                "bins derived from the 2^20 bin");
  const uint32_t ntup = len / D;
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const uint32_t j = threadIdx.x + it * kHistThreads;
    uint32_t cell = 0;
    if (j < ntup) {
      if constexpr (D == 1) {
        cell = b20[j];
      } else if constexpr (D == 3) {
        cell = (b100[3 * j] * 100u + b100[3 * j + 1]) * 100u + b100[3 * j + 2];
      } else {
        constexpr int kShift = D == 2 ? 10 : (D == 4 ? 15 : 16), kBits = 20 - kShift;
#pragma unroll
        for (int i = 0; i < D; ++i) cell = (cell << kBits) | (b20[j * D + i] >> kShift);
      }
    }
    key[it] = j < ntup ? key0 + cell : ph::kNoKey;
  }
}

// Registers per thread for the keys of one tile: 8 + 4 + 3 + 2 + 2.
constexpr int kT = (int)kHistThreads;
constexpr int kK1 = (kHistTile + kT - 1) / kT, kK2 = (kHistTile / 2 + kT - 1) / kT, kK3 = (kHistTile / 3 + kT - 1) / kT;
constexpr int kK4 = (kHistTile / 4 + kT - 1) / kT, kK5 = (kHistTile / 5 + kT - 1) / kT;
constexpr int kKeys = kK1 + kK2 + kK3 + kK4 + kK5;

// One tile of one block: frequency and serial D = 2..5 keys into the
// partitioned histograms, the poker histogram, and the bits R > 1/2 packed
// one 64-bit word per 64 uniforms (for the runs test).
__global__ __launch_bounds__(kHistThreads, 8) void hist_kernel(const double *__restrict__ r, ph::PartSet P, BatteryParts bp,
                                                   unsigned long long *poker_hist, uint64_t *__restrict__ bits) {
  // the tile's bins (b20 among 2^20, b100 among 100, b10 among 10 for the
  // poker digits), later reused as the key staging area of the scatter
  __shared__ __align__(16) uint32_t buf[kKeys * kHistThreads];
  static_assert(kKeys * kHistThreads * 4 >= kHistTile * 6, "staging area must hold the tile's bins");
  __shared__ uint32_t poker[kPokerCats];
  __shared__ uint32_t cnt[kMaxParts], poff[kMaxParts], base[kMaxParts];
  uint32_t *b20 = buf;
  uint8_t *b100 = reinterpret_cast<uint8_t *>(buf + kHistTile), *b10 = b100 + kHistTile;
  const uint32_t tile = blockIdx.x % kHistTilesPerBlock;
  const uint64_t blk = blockIdx.x / kHistTilesPerBlock;
  const uint32_t off = tile * kHistTile;
  const uint32_t len = (kBlock - off) < kHistTile ? (kBlock - off) : kHistTile;  // 7680 or 4096
  const uint64_t base_i = blk * kBlock + off;
  if (threadIdx.x < kPokerCats) poker[threadIdx.x] = 0;
  // all of the thread's loads in flight at once (a loop that waits for each
  // load before the next pays the memory latency every step), then the LDS
  // copy and the run bits; len is a multiple of 64, so the bounds test is
  // uniform over a wave and every wave covers 64 consecutive uniforms per step
  constexpr uint32_t kPer = (kHistTile + kHistThreads - 1) / kHistThreads;
  static_assert(kHistTile % 64 == 0 && (kBlock % kHistTile) % 64 == 0, "whole wave steps");
  double x[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = threadIdx.x + kHistThreads * k;
    x[k] = i < len ? r[base_i + i] : 0.0;
  }
  // the wave's k-th run-bit word is kept by lane k and all are stored at the
  // end with one instruction: a store inside the loop would make every later
  // step wait for it
  const uint32_t lane = threadIdx.x & 63, wbase = threadIdx.x - lane;
  uint64_t mine = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = threadIdx.x + kHistThreads * k;
    if (i < len) {
      b20[i] = bin_of(x[k], kFreqBins);
      b100[i] = (uint8_t)bin_of(x[k], kAxis3);
      b10[i] = (uint8_t)bin_of(x[k], 10);
      const uint64_t word = __ballot(x[k] > 0.5);
      if (lane == k) mine = word;
    }
  }
  if (lane < kPer && wbase + kHistThreads * lane < len) bits[(base_i + wbase + kHistThreads * lane) >> 6] = mine;
  __syncthreads();
  // poker: a wave counts its hands per category with ballots and adds each
  // count once (an LDS atomic per hand queued on the seven addresses)
  const uint32_t nhand = len / 5;
  uint32_t wcount[kPokerCats];
#pragma unroll
  for (uint32_t c = 0; c < kPokerCats; ++c) wcount[c] = 0;
  for (uint32_t j0 = wbase; j0 < nhand; j0 += kHistThreads) {  // wave-uniform bound
    const uint32_t j = j0 + lane;
    uint32_t cat = kPokerCats;  // lanes past the last hand count nowhere
    if (j < nhand) {
      uint32_t d[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) d[i] = b10[j * 5 + i];
      cat = poker_cat(d);
    }
#pragma unroll
    for (uint32_t c = 0; c < kPokerCats; ++c) wcount[c] += (uint32_t)__popcll(__ballot(cat == c));
  }
  if (lane < kPokerCats) {
    uint32_t v = 0;
#pragma unroll
    for (uint32_t c = 0; c < kPokerCats; ++c) v = lane == c ? wcount[c] : v;
    if (v) atomicAdd(&poker[lane], v);
  }
  // all five tests' keys of the tile in registers, then one scatter over the
  // partition space (its first barrier orders the last reads of the tile
  // before the staging area is overwritten)
  uint32_t key[kKeys];
  tuple_keys<1, kK1>(b20, b100, len, bp.p0[0] << ph::kPartBits, key);
  tuple_keys<2, kK2>(b20, b100, len, bp.p0[1] << ph::kPartBits, key + kK1);
  tuple_keys<3, kK3>(b20, b100, len, bp.p0[2] << ph::kPartBits, key + kK1 + kK2);
  tuple_keys<4, kK4>(b20, b100, len, bp.p0[3] << ph::kPartBits, key + kK1 + kK2 + kK3);
  tuple_keys<5, kK5>(b20, b100, len, bp.p0[4] << ph::kPartBits, key + kK1 + kK2 + kK3 + kK4);
  ph::scatter_staged<kHistThreads, kKeys>(key, P, 0, P.npart, cnt, poff, base, buf);
  if (threadIdx.x < kPokerCats && poker[threadIdx.x])
    atomicAdd(&poker_hist[(blockIdx.x % kRep) * kPokerCats + threadIdx.x], (unsigned long long)poker[threadIdx.x]);
}

// One collision trial per workgroup: 2^14 uniforms into 2^20 urns held as a
// 128 KB bitmap in LDS; a ball that finds its bit already set is a collision.
__global__ __launch_bounds__(1024) void collision_kernel(const double *__restrict__ r, unsigned long long *hist) {
  __shared__ uint32_t bm[kCollUrns / 32];
  __shared__ uint32_t total;
  const double *src = r + (uint64_t)blockIdx.x * kCollBalls;
  // the balls' loads go out before the bitmap is cleared, all at once
  constexpr uint32_t kPer = kCollBalls / 1024;
  double x[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) x[k] = src[threadIdx.x + 1024 * k];
  for (uint32_t i = threadIdx.x; i < kCollUrns / 32; i += 1024) bm[i] = 0;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  uint32_t coll = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t u = bin_of(x[k], kCollUrns);
    const uint32_t bit = 1u << (u & 31);
    const uint32_t old = atomicOr(&bm[u >> 5], bit);
    coll += (old & bit) ? 1u : 0u;
  }
  for (int s = 32; s > 0; s >>= 1) coll += __shfl_xor(coll, s);
  if ((threadIdx.x & 63) == 0) atomicAdd(&total, coll);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t c = total < kCollLo ? kCollLo : (total > kCollHi ? kCollHi : total);
    atomicAdd(&hist[(blockIdx.x % kRep) * kCollCats + (c - kCollLo)], 1ull);
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
  // Runs of length 1..8 (all but 0.4% of them) are counted in registers, four
  // 16-bit fields per word (lengths 1-4 in lo4, 5-8 in hi4; at most 64 runs
  // start in a word, and a wave's sums stay below 2^16); longer runs go to the
  // LDS histogram.  An LDS atomic per run queued on the few short-run bins.
  uint64_t lo4 = 0, hi4 = 0;
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
      if (len <= 4)
        lo4 += 1ull << (16 * (len - 1));
      else if (len <= 8)
        hi4 += 1ull << (16 * (len - 5));
      else
        atomicAdd(&h[(len < kRunsCats ? len : kRunsCats) - 1], 1u);
    }
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    lo4 += shfl_xor_u64(lo4, d);
    hi4 += shfl_xor_u64(hi4, d);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t a = (uint32_t)(lo4 >> (16 * b)) & 0xffffu, c = (uint32_t)(hi4 >> (16 * b)) & 0xffffu;
      if (a) atomicAdd(&h[b], a);
      if (c) atomicAdd(&h[4 + b], c);
    }
  }
  __syncthreads();
  if (threadIdx.x < kRunsCats && h[threadIdx.x])
    atomicAdd(&hist[(blockIdx.x % kRep) * kRunsCats + threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Pass-1 LDS layout: column c of a workgroup's 8 columns at c * kP1Stride
// (double2); 529 = 16 * 33 + 1 holds the column and then, in place, the
// wave transform's transpose, and spreads the columns over the banks.
constexpr int kP1Stride = 529;

// Pass 1 of the four-step transform of z_n = (x_2n - 1/2) + i (x_2n+1 - 1/2),
// n = 1024 j1 + j2: the 512-point transforms over j1 of kFftCols columns j2
// (two per wave, one per half-wave), times exp(2 pi i j2 k1 / 2^19), written
// as rows Y[k1][j2].
__global__ __launch_bounds__(256) void fft_pass1_kernel(const double *__restrict__ r, double2 *__restrict__ y,
                                                        Twiddles tw) {
  __shared__ double2 st[kFftCols * kP1Stride];
  const uint64_t blk = blockIdx.x / kFftPass1Groups;
  const uint32_t c0 = (blockIdx.x % kFftPass1Groups) * kFftCols;
  const double2 *src = reinterpret_cast<const double2 *>(r + blk * kBlock);
  // the thread's 16 loads in flight at once, then into the columns
  constexpr uint32_t kPer = kFftCols * kFftN1 / 256;
  double2 in[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t e = threadIdx.x + 256 * k, j1 = e / kFftCols, col = e % kFftCols;
    in[k] = src[(uint64_t)j1 * kFftN2 + c0 + col];
  }
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t e = threadIdx.x + 256 * k, j1 = e / kFftCols, col = e % kFftCols;
    st[col * kP1Stride + j1] = make_double2(in[k].x - 0.5, in[k].y - 0.5);
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, l = lane & 31;
  const uint32_t col = 2 * (threadIdx.x >> 6) + (lane >> 5);
  double2 *cs = st + col * kP1Stride;
  double2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = cs[l + 32 * m];
  wf::wave_fft<32>(v, cs, tw.w1024, l);
  // v[kb] = F[k1], k1 = k_a + 16 kb + 256 q; times the twiddle, back to the
  // column in frequency order
  const uint32_t ka = l >> 1, q = wf::wave_fft_q<32>(l);
  const uint32_t j2 = c0 + col;
  dev::wave_lds_sync();
  // w_N^{j2 k1} = w_N^{j2 (ka + 256 q)} (w_N^{16 j2})^kb: two roots loaded, then products
  const uint32_t t0 = j2 * (ka + 256 * q), t1 = 16 * j2;  // < 2^19
  double2 wt = cmul(tw.fineN[t0 & 1023], tw.w1024[2 * (t0 >> 10)]);
  const double2 ws = cmul(tw.fineN[t1 & 1023], tw.w1024[2 * (t1 >> 10)]);
#pragma unroll
  for (int kb = 0; kb < 16; ++kb) {
    cs[ka + 16 * kb + 256 * q] = cmul(v[kb], wt);
    wt = cmul(wt, ws);
  }
  __syncthreads();
  double2 *dst = y + blk * (uint64_t)kFftN;
  for (uint32_t e = threadIdx.x; e < kFftCols * kFftN1; e += 256) {
    const uint32_t k1 = e / kFftCols, c = e % kFftCols;
    dst[(uint64_t)k1 * kFftN2 + c0 + c] = st[c * kP1Stride + k1];
  }
}

__device__ __forceinline__ uint32_t fourier_cat(double v, double scale) {
  const double u = floor(v * scale);
  const double c = u < -kFourierHalf - 1 ? (double)(-kFourierHalf - 1) : (u > kFourierHalf ? (double)kFourierHalf : u);
  return (uint32_t)(int)(c + kFourierHalf + 1);
}

// Pass 2: the 1024-point transforms of rows k1 and 512 - k1 (rows 0 and 256
// pair with themselves), one wave per row, which give F_k for
// k = k1 + 512 k2 and the partner N - k of each; then the real-input split
//   E = (F_k + conj F_{N-k}) / 2,  O = (F_k - conj F_{N-k}) / (2i),
//   X_k = E + w_M^k O,  X_{N-k} = conj(E - w_M^k O),
// scaled by 1/sqrt(M), and the categories of their real and imaginary parts.
// split_and_bin takes A = F_k, B = F_{N-k} and wk = w_M^k.
__device__ __forceinline__ void split_and_bin(double2 A, double2 B, double2 wk, uint32_t k, double scale,
                                              uint32_t *h, double *cb) {
  const double fs = 1.0 / 1024.0;  // 1 / sqrt(M), exact
  const double ar = A.x, ai = A.y, br = B.x, bi = B.y;
  const double er = (ar + br) * 0.5, ei = (ai - bi) * 0.5;
  const double orr = (ai + bi) * 0.5, oi = (br - ar) * 0.5;
  const double tr = orr * wk.x - oi * wk.y, ti = orr * wk.y + oi * wk.x;
  const double xr = (er + tr) * fs, xi = (ei + ti) * fs;
  atomicAdd(&h[fourier_cat(xr, scale)], 1u);
  atomicAdd(&h[fourier_cat(xi, scale)], 1u);
  if (cb) {
    cb[2 * k] = xr;
    cb[2 * k + 1] = xi;
  }
  const uint32_t kp = (kFftN - k) % kFftN;
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

// Row pairs (k1, 512 - k1) with 1 <= k1 <= 255.  Each wave transforms its row
// with the split transpose (half the LDS of a complex one, so more
// workgroups fit on a CU), then the two waves swap half of their
// coefficients through the same areas.  Lane t holds F[c], c = ka + 16 kb +
// 256 q (ka = t / 4, q its output index); the mirror index 1023 - c of the
// other row sits in lane 63 - t of the other wave, register 15 - kb.  Wave 0
// (row k1) takes the pairs whose row-k1 index has kb < 8, wave 1 the pairs
// whose row-(512 - k1) index has kb < 8: every pair once.
constexpr int kP2Half = 16 * 65;  // doubles per wave
constexpr uint32_t kP2PairRows = kFftN1 / 2 - 1;
__global__ __launch_bounds__(128) void fft_pass2_pairs_kernel(const double2 *__restrict__ y, unsigned long long *hist,
                                                              double *__restrict__ coef, Twiddles tw, double scale) {
  constexpr int L = kFftN2;
  __shared__ __align__(16) double buf[2 * kP2Half];
  static_assert(8 * 64 * 2 <= kP2Half && (kP2Half * 8) % 16 == 0, "swap slots fit the area");
  __shared__ uint32_t h[kFourierCats];
  const uint64_t blk = blockIdx.x / kP2PairRows;
  const uint32_t ra = 1 + blockIdx.x % kP2PairRows, rb = kFftN1 - ra;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < kFourierCats) h[threadIdx.x] = 0;
  const double2 *row = y + blk * (uint64_t)kFftN + (uint64_t)(w ? rb : ra) * L;
  double *area = buf + w * kP2Half;
  double2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = row[lane + 64 * m];
  wf::wave_fft_split<64>(v, area, tw.w1024, lane);
  // registers 8..15 to the other wave: slot j * 64 + t holds v[8 + j] of lane t
  double2 *mine = reinterpret_cast<double2 *>(area);
  wf::wave_lds_fence();
#pragma unroll
  for (int j = 0; j < 8; ++j) mine[j * 64 + lane] = v[8 + j];
  __syncthreads();
  const double2 *other = reinterpret_cast<const double2 *>(buf + (1 - w) * kP2Half);
  double *cb = coef ? coef + blk * (uint64_t)kBlock : nullptr;
  // k = ra + 512 k2: w_M^k = fineM[ra + 512 (k2 & 1)] w_1024^{k2 >> 1}, with
  // k2 >> 1 = c0 + 8 kb (wave 0) or 511 - c0 - 8 kb (wave 1): one loaded root
  // and its products with w_1024^{+-8}
  const uint32_t ka = lane >> 2, q = wf::wave_fft_q<64>(lane);
  const uint32_t c0 = (ka >> 1) + 128 * q;
  const double2 fine = tw.fineM[ra + 512 * ((ka & 1) ^ w)];
  const double2 s8 = tw.w1024[8];
  const double2 step = w ? make_double2(s8.x, -s8.y) : s8;
  double2 wc = tw.w1024[w ? 511 - c0 : c0];
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    const uint32_t cown = ka + 16 * kb + 256 * q;
    const uint32_t k2 = w ? 1023 - cown : cown;
    const double2 pv = other[(7 - kb) * 64 + (63 - lane)];
    // A = row ra at k2, B = row rb at 1023 - k2
    split_and_bin(w ? pv : v[kb], w ? v[kb] : pv, cmul(fine, wc), ra + kFftN1 * k2, scale, h, cb);
    wc = cmul(wc, step);
  }
  __syncthreads();
  if (threadIdx.x < kFourierCats && h[threadIdx.x])
    atomicAdd(&hist[(blockIdx.x % kRep) * kFourierCats + threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// Rows 0 and 256, each paired with itself: one wave per copy of the row,
// the coefficients in frequency order in LDS (one pad slot every 256).
constexpr int kP2Area = 16 * 65;
__device__ __forceinline__ uint32_t p2_slot(uint32_t k2) { return k2 + (k2 >> 8); }

__global__ __launch_bounds__(128) void fft_pass2_self_kernel(const double2 *__restrict__ y, unsigned long long *hist,
                                                             double *__restrict__ coef, Twiddles tw, double scale) {
  constexpr int L = kFftN2;
  __shared__ double2 buf[2 * kP2Area];
  __shared__ uint32_t h[kFourierCats];
  const uint64_t blk = blockIdx.x >> 1;
  const uint32_t ra = (blockIdx.x & 1) ? kFftN1 / 2 : 0u;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < kFourierCats) h[threadIdx.x] = 0;
  const double2 *row = y + blk * (uint64_t)kFftN + (uint64_t)ra * L;
  double2 *area = buf + w * kP2Area;
  double2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = row[lane + 64 * m];
  wf::wave_fft<64>(v, area, tw.w1024, lane);
  const uint32_t ka = lane >> 2, q = wf::wave_fft_q<64>(lane);
  dev::wave_lds_sync();
#pragma unroll
  for (int kb = 0; kb < 16; ++kb) area[p2_slot(ka + 16 * kb + 256 * q)] = v[kb];
  __syncthreads();
  double *cb = coef ? coef + blk * (uint64_t)kBlock : nullptr;
  // row 0: k2 = 0..512 with partner 1024 - k2; row 256: k2 = 0..511 with
  // partner 1023 - k2 (in the second wave's copy of the row)
  const uint32_t nk2 = ra == 0 ? 513u : 512u;
  const double2 fine0 = tw.fineM[ra], fine1 = tw.fineM[ra + 512];
  for (uint32_t k2 = threadIdx.x; k2 < nk2; k2 += 128) {
    const uint32_t pa = p2_slot(k2);
    const uint32_t pb = ra == 0 ? p2_slot((1024 - k2) & 1023) : kP2Area + p2_slot(1023 - k2);
    const double2 wk = cmul((k2 & 1) ? fine1 : fine0, tw.w1024[k2 >> 1]);
    split_and_bin(buf[pa], buf[pb], wk, ra + kFftN1 * k2, scale, h, cb);
  }
  __syncthreads();
  if (threadIdx.x < kFourierCats && h[threadIdx.x])
    atomicAdd(&hist[(blockIdx.x % kRep) * kFourierCats + threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// dst[c] += sum of the kRep replicas of bin c, which are cleared.
__global__ __launch_bounds__(256) void fold_kernel(unsigned long long *rep, unsigned long long *dst, uint32_t ncat) {
  const uint32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= ncat) return;
  unsigned long long s = 0;
  for (uint32_t r = 0; r < kRep; ++r) {
    s += rep[(uint64_t)r * ncat + c];
    rep[(uint64_t)r * ncat + c] = 0;
  }
  if (s) dst[c] += s;
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
  clear_launch_error();
  hist_kernel<<<dim3((unsigned)(nblocks * kHistTilesPerBlock)), dim3(kHistThreads), 0, st>>>(r, P, bp, poker, bits);
  return hipGetLastError();
}

hipError_t launch_collision(const double *r, uint64_t nblocks, unsigned long long *coll, hipStream_t st) {
  clear_launch_error();
  collision_kernel<<<dim3((unsigned)(nblocks * (kBlock / kCollBalls))), dim3(1024), 0, st>>>(r, coll);
  return hipGetLastError();
}

hipError_t launch_runs(const uint64_t *bits, uint64_t nblocks, unsigned long long *runs, hipStream_t st) {
  clear_launch_error();
  const uint64_t nwords = nblocks * kWordsPerBlock;
  runs_kernel<<<dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, st>>>(bits, nwords, runs);
  return hipGetLastError();
}

hipError_t launch_fft_pass1(const double *r, uint64_t nblocks, double2 *y, Twiddles tw, hipStream_t st) {
  clear_launch_error();
  fft_pass1_kernel<<<dim3((unsigned)(nblocks * kFftPass1Groups)), dim3(256), 0, st>>>(r, y, tw);
  return hipGetLastError();
}

hipError_t launch_fft_pass2(const double2 *y, uint64_t nblocks, unsigned long long *fourier, double *coef,
                            Twiddles tw, double scale, hipStream_t st) {
  clear_launch_error();
  fft_pass2_pairs_kernel<<<dim3((unsigned)(nblocks * kP2PairRows)), dim3(128), 0, st>>>(y, fourier, coef, tw, scale);
  fft_pass2_self_kernel<<<dim3((unsigned)(nblocks * 2)), dim3(128), 0, st>>>(y, fourier, coef, tw, scale);
  return hipGetLastError();
}

hipError_t launch_fold(unsigned long long *rep, unsigned long long *dst, uint32_t ncat, hipStream_t st) {
  clear_launch_error();
  fold_kernel<<<dim3((ncat + 255) / 256), dim3(256), 0, st>>>(rep, dst, ncat);
  return hipGetLastError();
}

hipError_t launch_chi2(const Chi2Job *jobs, int njobs, double *chi2, unsigned long long *total, hipStream_t st) {
  clear_launch_error();
  chi2_kernel<<<dim3(njobs), dim3(1024), 0, st>>>(jobs, chi2, total);
  return hipGetLastError();
}

hipError_t launch_interleave(const double *in, double *out, uint64_t nstreams, uint64_t length, hipStream_t st) {
  clear_launch_error();
  interleave_kernel<<<dim3((unsigned)((length + 63) / 64), (unsigned)((nstreams + 63) / 64)), dim3(64, 4), 0, st>>>(
      in, out, nstreams, length);
  return hipGetLastError();
}

}  // namespace bat
}  // namespace phprng
