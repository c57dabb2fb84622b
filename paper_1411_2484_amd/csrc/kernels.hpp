// Host-side launchers of the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace phprng {

hipError_t launch_table_segments32(uint64_t nseg, uint64_t *seg_sum, uint32_t *seg_start, hipStream_t st);
hipError_t launch_table_segments64(uint64_t nseg, uint64_t *seg_lo, uint64_t *seg_hi, uint64_t *seg_start,
                                   hipStream_t st);
hipError_t launch_seed_prime_flags(uint64_t seed, uint64_t j0, uint64_t count, int width, uint8_t *flags,
                                   hipStream_t st);
hipError_t launch_build_records(const uint64_t *n, const uint64_t *e, uint64_t count, int width, InstRec *out,
                                hipStream_t st);
// src: nreq host-written requests, device-accessible (pinned host memory or
// device memory); req: nreq device records; gbase: ceil(nreq / kPlanGroup)
// words; hdr->done must be 0 (every plan leaves it so).
hipError_t launch_plan(const InstRec *inst, const HostReq *src, ReqRec *req, uint64_t nreq, uint64_t *gbase,
                       PlanHdr *hdr, uint32_t tiles_per_chunk, hipStream_t st);
hipError_t launch_advance(HostReq *req, uint64_t nreq, hipStream_t st);
// grid: number of blocks; block: 64/128/256/512 threads; unroll: 1/2/4.
hipError_t launch_persistent(const GenArgs &A, unsigned grid, int block, int unroll, bool has64, hipStream_t st);
// One plain grid of `grid` one-wave blocks for request r.
hipError_t launch_plain(const GenArgs &A, uint64_t r, unsigned grid, int unroll, bool has64, hipStream_t st);

}  // namespace phprng
