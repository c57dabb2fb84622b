// Host-side launchers of the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace phprng {

// Fixed device scratch of the allocation-free entry point (one per device):
// the work counter, the batch header, the planned requests and the width-64
// tile state, at these byte offsets.
constexpr int kMaxDevices = 64;
constexpr uint64_t kNoAllocMaxRequests = 16384;
constexpr uint64_t kNoAllocMaxTiles64 = 1ull << 18;
constexpr uint64_t kScratchCtrOff = 0;
constexpr uint64_t kScratchReqOff = 256;
constexpr uint64_t kScratchHdrOff = kScratchReqOff - sizeof(BatchHdr);  // header right before the requests
constexpr uint64_t kScratchTileOff = kScratchReqOff + kNoAllocMaxRequests * sizeof(ReqRec);
constexpr uint64_t kScratchBytes = kScratchTileOff + 3 * kNoAllocMaxTiles64 * sizeof(uint64_t);
constexpr uint64_t kScratchClearBytes = sizeof(WorkCtr);
static_assert(kScratchTileOff % 256 == 0, "tile arrays aligned");

// Device address of this device's scratch (the current device must be
// `device`).  The first call on a device looks the address up and clears the
// work counter; later calls return the kept address.
hipError_t scratch_address(int device, void **ptr);

hipError_t launch_table_segments32(uint64_t nseg, uint64_t *seg_sum, uint32_t *seg_start, hipStream_t st);
hipError_t launch_table_segments64(uint64_t nseg, uint64_t *seg_lo, uint64_t *seg_hi, uint64_t *seg_start,
                                   hipStream_t st);
hipError_t launch_seed_prime_flags(uint64_t seed, uint64_t j0, uint64_t count, int width, uint8_t *flags,
                                   hipStream_t st);
hipError_t launch_build_records(const uint64_t *n, const uint64_t *e, uint64_t count, int width, InstRec *out,
                                hipStream_t st);
// m64[ids[i]] = m0[i] + U(ta[i]) - U(tb[i]) mod n[ids[i]] from the width-64
// positioning table (ta, tb < kTab64Range; U(t) = sum_{j<=t} (a^j mod p));
// m0, ta, tb may be NULL (zeros).  All arrays are device arrays of `count`
// entries.
hipError_t launch_position64(const InstRec *inst, const uint32_t *ids, const uint64_t *m0, const uint64_t *ta,
                             const uint64_t *tb, uint64_t count, const uint64_t *u_lo, const uint64_t *u_hi,
                             const uint64_t *u_s, uint64_t *m64, hipStream_t st);
// Width-64 tile starts of a batch: the reduce writes each tile's start skip
// and skip sum (hdr->units64 units of hdr->reduce_tiles tiles, grid-stride
// with at most max_blocks blocks); the scan turns the sums into tile-start
// messages per instance and commits the instances' messages (one workgroup
// per width-64 request).
hipError_t launch_tiles64_reduce(const GenArgs &A, uint64_t units64, unsigned max_blocks, hipStream_t st);
hipError_t launch_tiles64_scan(const GenArgs &A, uint64_t nreq64, hipStream_t st);
// Width-64 tile starts from the table for the instances whose draws in the
// batch all lie below kTab64Range (kSegTable in their requests' seg): one
// wave per width-64 request; also commits those instances' messages.  The
// scan serves the other instances.
hipError_t launch_tiles64_table(const GenArgs &A, uint64_t nreq64, hipStream_t st);
// *m = *m + sign * (sum_{i=1}^{count} (a^{t+i} mod p) + extra) mod n, with
// `blocks` 256-thread blocks writing blocks * 4 partial sums to `partial`.
hipError_t launch_skip_total64(uint64_t t, uint64_t count, uint64_t n, const LaneMul *lm, uint64_t *partial,
                               unsigned blocks, uint64_t extra, int sign, uint64_t *m, hipStream_t st);
// grid: number of blocks; block: 64/128/256/512 threads; unroll: 1/2/4.
hipError_t launch_persistent(const GenArgs &A, unsigned grid, int block, int unroll, bool has64, hipStream_t st);
// One plain grid of `grid` one-wave blocks for request r.
hipError_t launch_plain(const GenArgs &A, uint64_t r, unsigned grid, int unroll, bool has64, hipStream_t st);

}  // namespace phprng
