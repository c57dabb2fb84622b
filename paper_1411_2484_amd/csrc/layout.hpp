// Records shared by the host runtime and the gfx950 kernels.
#pragma once

#include <cstdint>

namespace phprng {

// Skip generators of eq. (5) (see include/phprng.h for the 64-bit choice).
constexpr uint32_t kP32 = 2147483647u;             // 2^31 - 1
constexpr uint32_t kA32 = 784588716u;
constexpr uint64_t kP64 = 2305843009213693951ull;  // 2^61 - 1
constexpr uint64_t kA64 = 1633150009242682173ull;

// Width-32 tiles: one wave produces kTile32 = 64 * kRun32 consecutive draws of
// one instance; lane l owns the run [l * kRun32, (l + 1) * kRun32) of the
// tile for the message prefix, and tile starts are aligned to the stride of
// the universal skip-prefix table, so that every tile start is one table
// entry (eq. (7)).
constexpr int kRun32 = 32;
constexpr int kTile32 = 64 * kRun32;  // 2048 draws
constexpr uint64_t kTableStride = kTile32;
// Tiles per skip period for width 32: ceil((p - 1) / kTile32).
constexpr uint64_t kTilesPerPeriod32 = ((uint64_t)kP32 - 1 + kTile32 - 1) / kTile32;

// Width-64 tiles: 64 runs of kRun64 draws, counted from the first draw of
// their request (tile starts come from the request's own skip sums, not from
// a table), so a width-64 tile needs the same LDS as a width-32 one.
constexpr int kRun64 = 16;
constexpr int kTile64 = 64 * kRun64;  // 1024 draws
// The width-64 reduce takes up to this many consecutive tiles of a request
// per wave (fewer when the batch is too small to keep every wave busy).
constexpr int kReduceTiles = 16;
// Constant-skip tiles (both widths): 2048 draws aligned to multiples of 2048.
constexpr int kTileCS = 2048;
// The width-64 skip-prefix table covers skip logarithms below kTab64Range
// with an entry every kTab64Stride: it positions instances, serves jumps,
// and gives the tile starts of batches whose width-64 draws all lie in its
// range (tiles then start at entries, like width-32 tiles).
constexpr uint64_t kTab64Stride = kTile64;
constexpr uint64_t kTab64Range = 1ull << 34;

// Device instance record (one 128-byte line).  All modular constants are
// precomputed on the host so that the kernels only multiply.
struct alignas(128) InstRec {
  uint64_t n;      // prime modulus
  uint64_t ninv;   // n^{-1} mod 2^W (W = 32 or 64)
  uint64_t kcorr;  // R^e mod n, R = 2^W
  uint64_t r2;     // R^2 mod n
  uint64_t br2;    // (p(p-1)/2 mod n) * R^2 mod n (width 32)
  uint64_t mbase;  // width 32: m at internal index x is mbase + q b + U(r) mod n; constant skip: m_0
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

// A planned request (written by the host, copied to the device once per
// call).  A batch lists its width-64 pseudorandom-skip requests first,
// grouped by instance in call order, then the other width-64 requests, then
// the width-32 ones.
struct alignas(64) ReqRec {
  uint64_t x;           // width 32 / constant skip: internal index of the state before the first draw;
                        // width 64 pseudorandom skip: skip logarithm t of that state (s = a^t mod p)
  uint64_t count;       // number of draws
  uint64_t out_off;     // output element offset
  uint64_t g1;          // width 32: global tile of the first draw (q * tiles per period + j);
                        // constant skip: x / kTileCS; width 64: first entry in the batch's tile-state arrays
                        // (its tiles start at x + 1024 j, or at table entries when seg has kSegTable)
  uint64_t chunk_base;  // first chunk of this request in the batch
  uint32_t inst;        // instance id
  uint32_t ntiles;      // tiles touched
  uint32_t nchunks;     // chunks of this request
  uint32_t seg;         // width 64 pseudorandom skip: number of consecutive requests of this instance
                        // starting here (0 for a request that is not the first of its instance), plus
                        // kSegTable when the instance's tiles start at table entries
  uint64_t rbase;       // width 64 pseudorandom skip: first reduce unit of this request
};
static_assert(sizeof(ReqRec) == 64, "ReqRec must be 64 bytes");
// ReqRec::seg: the table flag and the request count of an instance segment.
constexpr uint32_t kSegTable = 1u << 31;
constexpr uint32_t kSegCount = kSegTable - 1;

// Per-call totals, copied with the requests (kernels read them from device
// memory, so that captured graphs take new values at every launch).
struct alignas(64) BatchHdr {
  uint64_t total_chunks;  // chunks of the whole batch
  uint64_t nreq;          // requests
  uint64_t nreq64;        // width-64 pseudorandom-skip requests (the first nreq64)
  uint64_t tiles64;       // their tiles (entries of the tile-state arrays)
  uint64_t units64;       // their reduce units
  uint64_t reduce_tiles;  // tiles per reduce unit (1 .. kReduceTiles)
  uint64_t pad[2];
};
static_assert(sizeof(BatchHdr) == 64, "BatchHdr must be 64 bytes");

// Work-stealing counter of the generation kernel: zero when a launch starts;
// the wave that makes the launch's last grab sets it back to zero.
struct alignas(64) WorkCtr {
  uint32_t counter;
  uint32_t pad[15];
};

// Width-64 tile state of a batch: skip and message before each tile, and
// the sum of the tile's skips mod n.
struct Tile64 {
  uint64_t *s;
  uint64_t *sum;
  uint64_t *m;
};

// Universal width-32 skip-prefix table: entry i holds U(i * stride) =
// sum_{j=1}^{i*stride} (a^j mod p) and S(i * stride) = a^{i*stride} mod p.
// The width-64 table holds the same below kTab64Range (U as 128 bits).
struct SkipTables {
  const uint64_t *u32;  // U (< 2^62)
  const uint32_t *s32;  // S
  uint64_t n32;         // entries
  const uint64_t *u64lo, *u64hi;  // width 64: U, low and high words
  const uint64_t *s64;            // width 64: S
};

// Per-lane and per-tile skip multipliers.
struct LaneMul {
  uint32_t m32[64];     // a^{l * kRun32} mod (2^31 - 1)
  uint64_t m64[64];     // a^{l * kRun64} mod (2^61 - 1)
  uint64_t pow64[64];   // a^{2^b} mod (2^61 - 1), b = 0..60
};

struct GenArgs {
  const InstRec *inst;
  const ReqRec *req;
  const BatchHdr *hdr;
  uint64_t nreq;
  WorkCtr *ctr;
  SkipTables tab;
  const LaneMul *lanemul;
  Tile64 t64;
  uint64_t *m64;  // per-instance width-64 message at the committed position
  uint32_t *out_c32;
  uint64_t *out_c64;
  double *out_r;
  uint32_t tiles_per_chunk;
};

}  // namespace phprng
