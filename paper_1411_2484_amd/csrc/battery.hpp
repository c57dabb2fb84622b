// Statistical battery of the paper's Tests section on gfx950: shapes and the
// host-side launchers of battery.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "phist.hpp"

namespace phprng {
namespace bat {

// The tested sequence is consumed in blocks of 2^20 uniforms (the Fourier
// length); every test works inside a block.
constexpr uint32_t kBlock = 1u << 20;
constexpr uint32_t kFreqBins = 1u << 20;
constexpr uint32_t kAxis2 = 1024, kAxis3 = 100, kAxis4 = 32, kAxis5 = 16;
constexpr uint32_t kCells2 = kAxis2 * kAxis2, kCells3 = kAxis3 * kAxis3 * kAxis3;
constexpr uint32_t kCells4 = kAxis4 * kAxis4 * kAxis4 * kAxis4;
constexpr uint32_t kCells5 = kAxis5 * kAxis5 * kAxis5 * kAxis5 * kAxis5;
constexpr uint32_t kPokerCats = 7;
constexpr uint32_t kCollBalls = 1u << 14, kCollUrns = 1u << 20;
constexpr uint32_t kCollLo = 100, kCollHi = 155, kCollCats = kCollHi - kCollLo + 1;
constexpr uint32_t kRunsMax = 20, kRunsCats = kRunsMax + 1;
constexpr int kFourierHalf = 32;
constexpr uint32_t kFourierCats = 2 * kFourierHalf + 2;
constexpr uint32_t kWordsPerBlock = kBlock / 64;

// Histogram tile: 7680 = 120 * 64 uniforms for a workgroup of 1024 threads,
// a multiple of every tuple length (2..5) and of the wave width; a block is
// 136 full tiles and a 4096-uniform tail.  Every tile reserves bucket room
// once per partition with a global atomic, so a larger tile means fewer of
// them; 1024 threads keep the registers per thread low enough for two
// workgroups per CU.
constexpr uint32_t kHistThreads = 1024;
constexpr uint32_t kHistTile = 7680;
constexpr uint32_t kHistTilesPerBlock = (kBlock + kHistTile - 1) / kHistTile;

// Real transform of M = 2^20 points through one complex transform of
// N = 2^19 = N1 * N2 points (N1 = 512 rows, N2 = 1024 columns).
constexpr uint32_t kFftN = kBlock / 2, kFftN1 = 512, kFftN2 = 1024;
constexpr uint32_t kFftCols = 8;                           // pass-1 columns per workgroup
constexpr uint32_t kFftPass1Groups = kFftN2 / kFftCols;   // workgroups per block, pass 1

// The frequency and serial tests go through partitioned histograms: test t
// owns the partitions from p0[t] on in one partition space.
constexpr int kPartTests = 5;
constexpr uint32_t kMaxParts = 160;  // 32 + 32 + 31 + 32 + 32 partitions of 2^15 cells
struct BatteryParts {
  uint32_t p0[kPartTests];
};

// Roots of unity with the positive exponent of the paper's Fourier sum:
// w1024[t] = exp(2 pi i t / 1024), fineN[t] = exp(2 pi i t / 2^19),
// fineM[t] = exp(2 pi i t / 2^20), t = 0 .. 1023.
struct Twiddles {
  const double2 *w1024, *fineN, *fineM;
};

struct Chi2Job {
  const unsigned long long *counts;
  const double *probs;  // null: equal probabilities 1 / ncat
  uint32_t ncat;
  uint32_t pad;
};

// The small histograms (poker, collision, runs, Fourier categories) take a
// count from every workgroup.  Global atomics on the same address serialise
// (about 5e7 per second per address, measured), so a workgroup adds into
// replica blockIdx.x % kRep of the histogram, an array [kRep][categories]
// that launch_fold sums into the histogram (and clears).
constexpr uint32_t kRep = 256;

hipError_t launch_hist(const double *r, uint64_t nblocks, const ph::PartSet &P, const BatteryParts &bp,
                       unsigned long long *poker_rep, uint64_t *bits, hipStream_t st);
hipError_t launch_collision(const double *r, uint64_t nblocks, unsigned long long *coll_rep, hipStream_t st);
hipError_t launch_runs(const uint64_t *bits, uint64_t nblocks, unsigned long long *runs_rep, hipStream_t st);
hipError_t launch_fft_pass1(const double *r, uint64_t nblocks, double2 *y, Twiddles tw, hipStream_t st);
// coef (may be null): per block, M doubles = (Re, Im) of coefficients 0 .. M/2 - 1.
hipError_t launch_fft_pass2(const double2 *y, uint64_t nblocks, unsigned long long *fourier_rep, double *coef,
                            Twiddles tw, double scale, hipStream_t st);
hipError_t launch_fold(unsigned long long *rep, unsigned long long *dst, uint32_t ncat, hipStream_t st);
hipError_t launch_chi2(const Chi2Job *jobs, int njobs, double *chi2, unsigned long long *total, hipStream_t st);
hipError_t launch_interleave(const double *in, double *out, uint64_t nstreams, uint64_t length, hipStream_t st);

}  // namespace bat
}  // namespace phprng
