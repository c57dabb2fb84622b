// Records shared by the host runtime and the gfx950 kernels.
#pragma once

#include <cstdint>

namespace phprng {

// Skip generators of eq. (5) (see include/phprng.h for the 64-bit choice).
constexpr uint32_t kP32 = 2147483647u;             // 2^31 - 1
constexpr uint32_t kA32 = 784588716u;
constexpr uint64_t kP64 = 2305843009213693951ull;  // 2^61 - 1
constexpr uint64_t kA64 = 1633150009242682173ull;

// Tiles: one wave produces TILE = 64 * RUN consecutive draws of one instance;
// lane l owns the run [l * RUN, (l + 1) * RUN) of the tile for the message
// prefix, and the tile starts are aligned to the skip-prefix table stride.
constexpr int kRun = 32;
constexpr int kTile = 64 * kRun;        // 2048 draws
constexpr uint64_t kTableStride = kTile;
// Tiles per skip period for width 32: ceil((p - 1) / kTile).
constexpr uint64_t kTilesPerPeriod32 = ((uint64_t)kP32 - 1 + kTile - 1) / kTile;
// Width-64 positions (internal index) stay below this bound.
constexpr uint64_t kMaxPos64 = 1ull << 34;

// Device instance record (one 128-byte line).  All modular constants are
// precomputed on the host so that the kernels only multiply.
struct alignas(128) InstRec {
  uint64_t n;      // prime modulus
  uint64_t ninv;   // n^{-1} mod 2^W (W = 32 or 64)
  uint64_t kcorr;  // R^e mod n, R = 2^W
  uint64_t r2;     // R^2 mod n
  uint64_t br2;    // (p(p-1)/2 mod n) * R^2 mod n (width 32)
  uint64_t mbase;  // message offset: m at internal index x is mbase + q b + U(r) mod n
  uint64_t e;      // exponent
  double den;      // binary64(n + 1)
  double rcp;      // RN(1 / den)
  uint32_t width;  // 32 or 64
  uint32_t ekind;  // 3, 5, 9, 17, or 0 for the generic chain
  uint32_t ebits;  // bit length of e
  uint32_t sched;  // kSchedSkipLcg or kSchedConstant
  uint64_t bskip;  // constant skip b mod n
  uint64_t bR2;    // b R^2 mod n
  uint64_t b64;    // 64 b mod n (one lane-interleaved step)
  uint64_t pad1;
};

// Message schedules (Sec. II): the pseudorandom skip of eq. (5)-(7), or a
// constant skip b (the unit skip is b = 1) with m_k = m_0 + k b mod n.
constexpr uint32_t kSchedSkipLcg = 0;
constexpr uint32_t kSchedConstant = 1;
static_assert(sizeof(InstRec) == 128, "InstRec must be one 128-byte line");

// Request as the host writes it (32 bytes).  The plan kernel reads the list
// straight from pinned host memory, so no copy precedes it.
struct alignas(32) HostReq {
  uint64_t k;        // internal index of the state before the first draw
  uint64_t count;    // number of draws
  uint64_t out_off;  // output element offset
  uint32_t inst;     // instance id
  uint32_t pad;
};
static_assert(sizeof(HostReq) == 32, "HostReq must be 32 bytes");

// Requests per plan workgroup.  chunk_base below counts from the first chunk
// of the request's plan group; gbase[r / kPlanGroup] holds that group's first
// chunk in the whole batch.
constexpr uint32_t kPlanGroup = 256;

// Device request record: the host's request plus the plan kernel's tile and
// chunk bookkeeping.
struct alignas(64) ReqRec {
  uint64_t k;           // internal index of the state before the first draw
  uint64_t count;       // number of draws
  uint64_t out_off;     // output element offset
  uint64_t g1;          // first tile (global tile index q * tiles_per_period + j)
  uint64_t ntiles;      // tiles touched
  uint64_t chunk_base;  // exclusive prefix of chunks inside the plan group
  uint32_t inst;        // instance id
  uint32_t nchunks;     // chunks of this request
  uint64_t pad;
};
static_assert(sizeof(ReqRec) == 64, "ReqRec must be 64 bytes");

struct alignas(64) PlanHdr {
  uint64_t total_chunks;
  uint32_t counter;  // work-stealing counter
  uint32_t done;     // plan workgroups finished (back to 0 when the plan ends)
  uint32_t pad[12];
};

// Pointers to the universal skip-prefix tables: entry i holds U(i * stride)
// = sum_{j=1}^{i*stride} (a^j mod p) and S(i * stride) = a^{i*stride} mod p.
struct SkipTables {
  const uint64_t *u32;     // width 32: U (< 2^62)
  const uint32_t *s32;     // width 32: S
  const uint64_t *u64_lo;  // width 64: U low word
  const uint64_t *u64_hi;  // width 64: U high word
  const uint64_t *s64;     // width 64: S
  uint64_t n32, n64;       // entry counts
};

// Lane start multipliers a^{l * RUN} mod p for l = 0..63.
struct LaneMul {
  uint32_t m32[64];
  uint64_t m64[64];
};

struct GenArgs {
  const InstRec *inst;
  ReqRec *req;
  const uint64_t *gbase;  // first chunk of each plan group
  PlanHdr *hdr;
  uint64_t nreq;
  SkipTables tab;
  const LaneMul *lanemul;
  uint32_t *out_c32;
  uint64_t *out_c64;
  double *out_r;
  uint32_t tiles_per_chunk;
};

}  // namespace phprng
