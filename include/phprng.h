/*
 * phprng.h -- C interface of the MI355X (gfx950) library for the Pohlig-Hellman
 * parameter-split pseudorandom number generator of P. D. Beale ("A new class
 * of scalable parallel pseudorandom number generators based on Pohlig-Hellman
 * exponentiation ciphers").
 *
 * Each generator instance owns a prime modulus n and an exponent e coprime to
 * n - 1 (Sec. I, eq. (1)).  Its messages follow the pseudorandom-skip
 * schedule of eqs. (5)-(7): s_k = a s_{k-1} mod p, m_k = (m_{k-1} + s_k) mod n,
 * and each draw follows algorithm (9) of Sec. IV:
 *     s := a s mod p;  m := (m + s) mod n;  c := m^e mod n;  R := (c+1)/(n+1).
 *
 * Conventions fixed by this interface (readings of the paper):
 *   - Position.  An instance at position k holds the state (m_k, s_k) of
 *     eq. (7).  A draw advances to k+1 and returns c_{k+1} (and R_{k+1}), so
 *     the t-th draw (t = 0, 1, ...) from position k returns c_{k+1+t}, and N
 *     draws leave the instance at k + N.
 *   - Base state.  Position 0 is (m_0, s_0) = (0, 1) (Sec. IV, seeding by
 *     skipping from a base state) unless m_0 / s_0 are supplied.
 *   - Widths.  Width 32: n prime in [2^31, 2^32), skip p = 2^31 - 1,
 *     a = 784588716 (the L'Ecuyer skip generator tested in Sec. II); c is a
 *     uint32.  Width 64: n prime in [2^62, 2^63), skip p = 2^61 - 1 with the
 *     fixed primitive root a = 1633150009242682173 (the paper names no 64-bit
 *     skip parameters); c is a uint64.  p < n always holds.
 *   - Uniform.  R is the IEEE binary64 round-to-nearest-even quotient of
 *     binary64(c+1) by binary64(n+1).  For width 32 both conversions are
 *     exact and R lies in (0, 1); for width 64 the conversions round and R
 *     lies in (0, 1] (R = 1.0 occurs for the largest ciphertexts).
 *   - Positions.  Positions of both widths use the whole uint64 range.  A
 *     width-64 instance carries its message on the device (the state
 *     (m, s) of Sec. II): each batch continues it from the instance's own
 *     skip sums, so generation from any state and any position needs no
 *     table.  Width-32 tile starts come from eq. (7) and one universal table
 *     of skip sums over the whole skip period.
 *
 * Threading: a context may be used from one host thread at a time.  Every
 * call validates all of its arguments before it changes any state or
 * launches any kernel, so an error return leaves the context unchanged.
 * Nothing throws across this interface.
 */
#ifndef PHPRNG_H
#define PHPRNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PHPRNG_OK = 0,
  PHPRNG_E_INVALID = -1,   /* null pointer, bad width/mode/id, bad size      */
  PHPRNG_E_NOT_PRIME = -2, /* modulus n is not prime                          */
  PHPRNG_E_EXPONENT = -3,  /* e < 3, gcd(e, n-1) != 1, or e = 1 mod (n-1)     */
  PHPRNG_E_RANGE = -4,     /* n outside its width range, output range beyond
                              the stated capacity, position beyond range      */
  PHPRNG_E_NOMEM = -5,     /* host or device allocation failed                */
  PHPRNG_E_DEVICE = -6     /* a HIP call failed; the message is kept in the
                              context (phprng_last_error)                     */
} phprng_status;

typedef struct phprng_ctx phprng_ctx;

/* The mutable state of an instance (Sec. II: m, s and c change; n, e, p, a
 * are fixed) plus its position k.  c is c_k = m_k^e mod n. */
typedef struct {
  uint64_t m, s, c, k;
} phprng_state;

/* One generation request: `count` draws from instance `instance`, written to
 * element offsets [out_offset, out_offset + count) of the output arrays. */
typedef struct {
  uint32_t instance;
  uint32_t reserved; /* must be 0 */
  uint64_t count;
  uint64_t out_offset;
} phprng_request;

/* Launch shape of the batched kernel.  Zero fields mean "library default". */
typedef struct {
  int32_t block_threads;   /* 64, 128, 256 or 512 */
  int32_t blocks_per_cu;   /* resident blocks per compute unit for the persistent grid */
  int32_t tiles_per_chunk; /* consecutive tiles a wave takes per work grab (1..64; a tile is
                              2048 draws at width 32 and for constant skips, 1024 draws at
                              width 64); halved for batches too small to give every wave 4 grabs */
  int32_t unroll;          /* encryption-loop unroll: 1, 2 or 4 */
} phprng_tuning;

enum { PHPRNG_MODE_PERSISTENT = 0, PHPRNG_MODE_PLAIN = 1 };

/* ---- host-only helpers (no device needed) --------------------------------*/

/* Skip generator of eq. (5) for a width: p and a (see the conventions). */
phprng_status phprng_skip_params(int width, uint64_t *p, uint64_t *a);

/* Admissibility of (n, e) for a width (Sec. I, II, IV): PHPRNG_OK, or the
 * reason it is rejected.  Primality is decided by trial division followed by
 * deterministic Rabin-Miller (five prime bases below 2^32, twelve above). */
phprng_status phprng_check_instance(int width, uint64_t n, uint64_t e);

/* Seeded draw of `count` instance parameters (host arrays n, e, k of length
 * count).  One SplitMix64 stream (Steele, Lea and Flood, 2014) started at
 * `seed` is consumed in this order, per instance:
 *   repeat { x = next(); n = (lo + x mod span) | 1 over the width's range
 *            [lo, lo + span); reject n unless prime and not drawn before in
 *            this call; y = next(); take the first admissible e among
 *            e_set[(y mod e_len + t) mod e_len], t = 0, 1, ...; reject n if
 *            none is }
 *   then k = k_lo + next() mod (k_hi - k_lo) if k_hi > k_lo, else k = k_lo.
 * e_set: host array of e_len candidate exponents. */
phprng_status phprng_draw_instances(int width, uint64_t seed, uint64_t count, const uint64_t *e_set, int e_len,
                                    uint64_t k_lo, uint64_t k_hi, uint64_t *n, uint64_t *e, uint64_t *k);

const char *phprng_status_string(phprng_status st);

/* ---- contexts --------------------------------------------------------------*/

/* Create a context on HIP device `device` with room for max_instances
 * instances (device records of 128 bytes each).  Builds the universal
 * 32-bit skip-prefix table of eq. (7b) on the device (12 MB); the 64-bit
 * table (400 MB) is built when the first width-64 instance is added.  Also
 * sets up the context's eight staging slots for batches of up to 8192
 * requests and 2^16 width-64 tiles (about 4 MB of pinned host memory and
 * 17 MB of device memory); a larger batch grows a slot, and that growth
 * waits for the device.  *ctx receives the context; the caller owns it and
 * frees it with phprng_destroy. */
phprng_status phprng_create(phprng_ctx **ctx, int device, uint64_t max_instances);
phprng_status phprng_destroy(phprng_ctx *ctx);

/* Message of the last PHPRNG_E_DEVICE (or other) error on this context;
 * owned by the context, valid until the next call. */
const char *phprng_last_error(const phprng_ctx *ctx);

/* Add `count` instances of one width (host arrays of length count).
 * m0, s0, k0 may each be NULL (then 0, 1, 0): instance i starts from
 * (m_0, s_0) = (m0[i], s0[i]) and is positioned at k0[i] by eq. (7).
 * s0[i] must lie in [1, p-1] and m0[i] in [0, n-1].  All instances are
 * validated before any is added; ids receives the new instance ids. */
phprng_status phprng_add_instances(phprng_ctx *ctx, uint64_t count, int width, const uint64_t *n, const uint64_t *e,
                                   const uint64_t *m0, const uint64_t *s0, const uint64_t *k0, uint32_t *ids);

/* Add `count` instances that use the constant-skip schedule of Sec. II
 * instead of the pseudorandom skip: m_k = (m_0 + k b) mod n, so the t-th draw
 * from position k encrypts m_0 + (k + 1 + t) b (b = 1 is the unit skip, the
 * counter mode of the cipher).  b[i] must lie in [1, n[i] - 1]; m0, k0 may be
 * NULL (then 0).  Positions of these instances use the whole uint64 range
 * for both widths; their skip s is b at every position. */
phprng_status phprng_add_instances_skip(phprng_ctx *ctx, uint64_t count, int width, const uint64_t *n,
                                        const uint64_t *e, const uint64_t *b, const uint64_t *m0, const uint64_t *k0,
                                        uint32_t *ids);

/* Schedule of instance `id`: *sched = 0 (pseudorandom skip) or 1 (constant
 * skip), *b = its constant skip (0 for the pseudorandom skip). */
phprng_status phprng_get_schedule(phprng_ctx *ctx, uint32_t id, int *sched, uint64_t *b);

/* Seeding of Sec. IV (each process draws its own modulus from a seeded
 * stream and skips forward from the base state (m_0, s_0) = (0, 1) of
 * eq. (7)): the same result as phprng_draw_instances followed by
 * phprng_add_instances with m0 = 0, s0 = 1.  For count >= 1024 the primality
 * of the stream outputs is decided on the device (one deterministic
 * Rabin-Miller per output) and the instance records are built there; the
 * draw order is unchanged.  In that bulk form width-64 starts must lie below
 * 2^34 (k_hi <= 2^34; the start messages come from the positioning table),
 * else PHPRNG_E_RANGE; smaller counts accept any start that
 * phprng_add_instances accepts.  ids: host array of count entries that
 * receives the new instance ids. */
phprng_status phprng_seed_instances(phprng_ctx *ctx, uint64_t count, int width, uint64_t seed,
                                    const uint64_t *e_set, int e_len, uint64_t k_lo, uint64_t k_hi, uint32_t *ids);

uint64_t phprng_instance_count(const phprng_ctx *ctx);

/* The hot path: algorithm (9) of Sec. IV, s := a s mod p; m := (m + s) mod n;
 * c := m^e mod n (eq. (1)); R := (c + 1)/(n + 1), run `count` times per
 * request from the instance's current state.  Generate draws for `nreq`
 * requests (host array) into caller-owned device arrays: out_c32 receives the ciphertexts of width-32 requests, out_c64 those
 * of width-64 requests, out_r the uniforms of both; any of them may be NULL
 * (that output is not written).  `capacity` is the element count of every
 * non-NULL output array; each request must satisfy out_offset + count <=
 * capacity.  Requests must not overlap in the outputs they write.  Several
 * requests may name the same instance: they are served in request order, so
 * each continues where the previous one ends.  Positions advance on the host
 * at call time; the kernels run asynchronously on `stream` (a hipStream_t, or
 * NULL for the null stream) and the outputs are valid once it completes.
 * Successive calls may use different streams without synchronizing: the
 * device-side message a call commits for its width-64 instances is waited
 * for by the next call's kernels that read it (one event), so streams
 * continue correctly in any stream order of the calls.
 * mode: PHPRNG_MODE_PERSISTENT (one work-stealing launch for the whole batch)
 * or PHPRNG_MODE_PLAIN (one launch per request).  A request with count 0 is
 * allowed and does nothing.  The requests are planned on the host during
 * the call, so the caller may reuse the array on return. */
phprng_status phprng_generate(phprng_ctx *ctx, const phprng_request *reqs, uint64_t nreq, uint32_t *out_c32,
                              uint64_t *out_c64, double *out_r, uint64_t capacity, void *stream, int mode);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): phprng_generate in
 * persistent mode that calls no hipMalloc, hipFree or other allocating
 * routine.  Its device scratch (the planned requests, the work counter and
 * the width-64 tile state) is one fixed array per device, about 7.3 MB, held
 * until the process ends; its host staging buffer is allocated when the
 * context is created.  Limits: at most 16384 requests and 2^18 width-64
 * tiles (2^28 width-64 draws) per call, else PHPRNG_E_RANGE with nothing
 * changed.  Every call on a device shares that device's scratch: calls that
 * overlap on one device (different streams, or different contexts) race;
 * calls ordered on one stream do not.  Arguments and results as for
 * phprng_generate; no kernel timing is recorded. */
phprng_status phprng_generate_noalloc(phprng_ctx *ctx, const phprng_request *reqs, uint64_t nreq, uint32_t *out_c32,
                                      uint64_t *out_c64, double *out_r, uint64_t capacity, void *stream);

/* Move instance `id` by delta positions (eq. (7); delta < 0 moves backward as
 * in Sec. II).  PHPRNG_E_RANGE if the position would leave its range.  A
 * width-64 move of d = q (p - 1) + r draws adds q whole skip periods
 * (p(p-1)/2 each, Sec. II) and the skip sum of the remaining r draws, taken
 * from the positioning table when both ends lie below 2^34 and otherwise
 * summed on the device (time proportional to min(r, p - 1 - r); either must
 * stay below 2^42, else PHPRNG_E_RANGE). */
phprng_status phprng_jump(phprng_ctx *ctx, uint32_t id, int64_t delta);

/* Current state (m_k, s_k, c_k, k) of instance `id`: the mutable integers m,
 * s and c of Sec. II (c_k = m_k^e mod n, eq. (1)) and the position k of
 * eq. (7).  Waits for queued width-64 work, whose message is on the device.
 * out: host struct owned by the caller. */
phprng_status phprng_get_state(phprng_ctx *ctx, uint32_t id, phprng_state *out);

/* Current position k of instance `id` (cheap: no state is computed). */
phprng_status phprng_get_position(phprng_ctx *ctx, uint32_t id, uint64_t *k);

/* Restore instance `id` to the state (st->m, st->s) reported at position
 * st->k (st->c is ignored; for a constant-skip instance st->s must equal
 * its b).  Any m in [0, n-1] and any s in [1, p-1] are accepted, for both
 * widths: the library finds t with a^t = s mod p by a Pohlig-Hellman
 * discrete logarithm (p - 1 is smooth for both skip moduli), so that the
 * stream continues by eq. (5)-(6) from exactly that state. */
phprng_status phprng_set_state(phprng_ctx *ctx, uint32_t id, const phprng_state *st);

/* Fixed parameters of instance `id`: the modulus n and exponent e of
 * eq. (1) and the skip generator's p and a of eq. (5) (the four constant
 * integers of the state in Sec. II), and its width.  Any pointer may be
 * NULL. */
phprng_status phprng_get_params(phprng_ctx *ctx, uint32_t id, uint64_t *n, uint64_t *e, uint64_t *p, uint64_t *a,
                                int *width);

/* Launch shapes used by phprng_generate (persistent mode) and graphs, one
 * per class of batch: width-32 requests only, width-64 only, or both.
 * phprng_set_tuning sets all three classes; phprng_get_tuning reads the
 * width-32 class. */
enum { PHPRNG_CLASS_W32 = 0, PHPRNG_CLASS_W64 = 1, PHPRNG_CLASS_MIXED = 2 };
phprng_status phprng_set_tuning(phprng_ctx *ctx, const phprng_tuning *t);
phprng_status phprng_get_tuning(phprng_ctx *ctx, phprng_tuning *t);
phprng_status phprng_set_tuning_class(phprng_ctx *ctx, int cls, const phprng_tuning *t);
phprng_status phprng_get_tuning_class(phprng_ctx *ctx, int cls, phprng_tuning *t);

/* Time candidate launch shapes (block size, blocks per CU, tiles per chunk,
 * unroll) on a synthetic batch of about `draws` draws spread over the
 * context's first (up to 4096) instances, writing FP64 uniforms only, into a
 * temporary device buffer of 8 bytes per draw.  Each shape is timed by the
 * median of three kernel times after a 300 ms warm-up; the fastest is kept
 * (if it beats the current shape on a re-run) for the class of that batch
 * (the widths among those instances), returned in *best (may be NULL), and
 * remembered for the process: later contexts on a device of the same
 * architecture and compute-unit count start from it.  Instance positions
 * and width-64 messages are restored afterwards. */
phprng_status phprng_autotune(phprng_ctx *ctx, uint64_t draws, phprng_tuning *best);

/* ---- captured repeat draws -------------------------------------------------*/

typedef struct phprng_graph phprng_graph;

/* Capture one persistent generation of `reqs` into a HIP graph.  Each
 * phprng_graph_launch draws every request's count from its instance's
 * current position (whatever moved it since the last launch: generate,
 * jump, set_state), advances the positions and overwrites the same output
 * ranges; the planned requests are copied to the device before each
 * replay.  Requests must name distinct instances. */
phprng_status phprng_graph_create(phprng_ctx *ctx, const phprng_request *reqs, uint64_t nreq, uint32_t *out_c32,
                                  uint64_t *out_c64, double *out_r, uint64_t capacity, void *stream,
                                  phprng_graph **graph);
phprng_status phprng_graph_launch(phprng_graph *graph, void *stream);
phprng_status phprng_graph_destroy(phprng_graph *graph);

/* Kernel time of the last phprng_generate / phprng_graph_launch call on the
 * context, in milliseconds, measured with HIP events recorded on its stream
 * right before and after the call's kernels (for width-64 requests the
 * tile-start reduce and scan, then the generation kernel or kernels); waits
 * for that stream.  PLAIN mode reports the span of all its launches. */
phprng_status phprng_last_kernel_ms(phprng_ctx *ctx, double *ms);

/* Cumulative generation-kernel time (same events as above) and number of
 * timed calls since the last phprng_timing_reset, without stalling the host
 * between calls: each call's events are read when its staging slot is
 * recycled, and this function waits for the calls still in flight. */
phprng_status phprng_timing_reset(phprng_ctx *ctx);
phprng_status phprng_timing_read(phprng_ctx *ctx, double *total_ms, uint64_t *calls);

/* Per-call kernel timing on (on != 0, the default) or off.  Off, a call
 * records only the event that ends its kernels (the staging slot's
 * completion), not the one before them: one HIP event record fewer per
 * call, about 5 microseconds of host time on MI355X with ROCm 7, for
 * latency-bound callers such as a serving loop.  Calls made with timing off
 * are not counted by phprng_timing_read, and phprng_last_kernel_ms fails
 * after one.  phprng_autotune times its candidates either way. */
phprng_status phprng_set_timing(phprng_ctx *ctx, int on);

/* ---- serving: continuous batching over resident instances -------------------*/

/* A server owns a device output arena and a scheduler thread that runs
 * generation for queued requests on the instances of `ctx` (the instance
 * table stays resident on the device; positions are reserved on the host at
 * admission).  Requests are admitted in FIFO order while the arena has room
 * for their FP64 uniforms and the batch limits allow; each admitted group is
 * one batched launch on the next of `streams` HIP streams, so batches
 * submitted while others run overlap on the device.  A request's output
 * depends only on its instance and the position range reserved for it, not
 * on what else is in its batch.  While a server exists, only the server may
 * use `ctx`.  Zero fields take defaults (arena 2^28 uniforms, 2 streams,
 * max_inflight = streams + 1 but at most 6, 8192 requests / 2^28 draws per
 * batch).  More batches in flight than streams queue a formed batch behind a
 * running one, so that the device does not idle while the host forms the
 * next batch. */
typedef struct phprng_server phprng_server;

typedef struct {
  uint64_t arena_doubles;      /* device arena capacity in FP64 uniforms */
  int32_t streams;             /* 1..8 */
  int32_t max_inflight;        /* batches on the device at once, 1..6 */
  uint32_t max_batch_requests; /* requests per batched launch */
  uint32_t reserved;           /* must be 0 */
  uint64_t max_batch_draws;    /* draws per batched launch (a single larger request still runs) */
} phprng_server_config;

/* A finished request.  data points to `count` FP64 uniforms inside the arena
 * (device memory), valid until phprng_server_release(ticket).  k is the
 * instance position before the request's first draw.  Times are host
 * steady-clock nanoseconds: submission, admission (launch), and completion
 * as observed by the scheduler. */
typedef struct {
  uint64_t ticket, tag;
  uint32_t instance;
  int32_t status;
  uint64_t count, k;
  double *data;
  int64_t t_submit_ns, t_admit_ns, t_done_ns;
} phprng_completion;

phprng_status phprng_server_create(phprng_ctx *ctx, const phprng_server_config *cfg, phprng_server **server);
/* Queue `count` uniforms from `instance`; thread-safe.  *ticket identifies it. */
phprng_status phprng_server_submit(phprng_server *server, uint32_t instance, uint64_t count, uint64_t tag,
                                   uint64_t *ticket);
/* Move up to `max` completions into out (host array); waits up to timeout_us
 * microseconds when none is ready.  *n receives the number returned. */
phprng_status phprng_server_poll(phprng_server *server, phprng_completion *out, uint64_t max, uint64_t *n,
                                 int64_t timeout_us);
/* Return a completed request's arena range. */
phprng_status phprng_server_release(phprng_server *server, uint64_t ticket);
/* Return the ranges of n completed requests under one lock; an unknown
 * ticket gives PHPRNG_E_INVALID after the others are released. */
phprng_status phprng_server_release_many(phprng_server *server, const uint64_t *tickets, uint64_t n);
phprng_status phprng_server_stats(phprng_server *server, uint64_t *pending, uint64_t *arena_used);
/* Launch counters since creation or the last reset: batched launches, the
 * requests and uniforms they held, and the host time spent issuing them
 * (position reservation, planning inputs, kernel launches), summed and the
 * longest single launch; how often a batch was cut short because the arena
 * had no room for the next request, and the most arena elements in use at
 * a launch; the scheduler's host time spent forming batches before the
 * launch (taking requests off the queue, arena admission, reading start
 * positions) and moving finished batches into the completion queue.
 * reset != 0 clears them after the read. */
typedef struct {
  uint64_t batches;
  uint64_t requests;
  uint64_t draws;
  int64_t launch_ns;
  int64_t launch_ns_max;
  uint64_t arena_stalls;
  uint64_t arena_peak;
  int64_t form_ns;
  int64_t retire_ns;
} phprng_server_counters;
phprng_status phprng_server_read_counters(phprng_server *server, phprng_server_counters *out, int reset);
/* Drains the batches on the device, stops the scheduler, frees the arena. */
phprng_status phprng_server_destroy(phprng_server *server);

/* Open-loop load: a native thread submits arrival i at t_ns nanoseconds after
 * the start (non-decreasing), each completed result is released at once, and
 * latency_ns[i] receives completion minus scheduled arrival (-1 on error).
 * admit_ns (may be NULL) receives, per arrival, the time from its scheduled
 * arrival to its admission (t_admit_ns: its batch is formed and about to be
 * launched), i.e. queueing and the scheduler's reaction; the launch and the
 * device work make up the rest of the latency.  *wall_s receives the time
 * from the start to the last completion. */
typedef struct {
  int64_t t_ns;
  uint32_t instance;
  uint32_t reserved;
  uint64_t count;
} phprng_arrival;

phprng_status phprng_server_replay(phprng_server *server, const phprng_arrival *arrivals, uint64_t n,
                                   int64_t *latency_ns, int64_t *admit_ns, double *wall_s);


/* ---- statistical battery: the chi-square tests of the Tests section ---------*/

/* The battery histograms a sequence of uniforms on the device and reports
 * chi^2 and P for nine of the paper's tests.  The sequence is consumed in
 * blocks of PHPRNG_BATTERY_BLOCK = 2^20 uniforms (the Fourier length); every
 * test works inside a block, so the result does not depend on how the blocks
 * are split over calls.  A uniform R falls in bin min(floor(R B), B - 1) of B
 * equal bins (the clamp only acts on R = 1.0).  Per block:
 *   FREQUENCY  all uniforms, 2^20 bins;
 *   SERIAL2..5 non-overlapping D-tuples (the last 2^20 mod D uniforms are
 *              unused), first element most significant, 1024 / 100 / 32 / 16
 *              bins per axis (2^20, 10^6, 2^20, 2^20 cells);
 *   POKER      non-overlapping hands of five digits min(floor(10 R), 9):
 *              all different, one pair, two pairs, three of a kind, full
 *              house, four of a kind, five of a kind;
 *   COLLISION  64 trials of 2^14 consecutive uniforms into 2^20 urns,
 *              collisions = 2^14 - occupied urns, categories <= 100, 101 ..
 *              154, >= 155;
 *   RUNS       bits R > 1/2, maximal runs with a differing bit on both sides
 *              inside the block, lengths 1 .. 20 and >= 21, expected counts
 *              = observed runs x the exact length law;
 *   FOURIER    x_j = R_j - 1/2, coefficients M^-1/2 sum_j x_j exp(+2 pi i j k / M)
 *              for k < M/2; real and imaginary parts in 64 bins of width
 *              sigma / 8 over [-4 sigma, 4 sigma) and two tails, sigma^2 =
 *              1/24, the bin of v being floor(v RN(8 sqrt 24)).
 * chi^2 = sum (O - E)^2 / E over the categories, dof = categories - 1, and P
 * is the one-sided probability about the median of the chi^2 law:
 * min(Q, 1 - Q) with Q its upper tail.  The paper's pass criterion is no
 * P < 1e-8. */
#define PHPRNG_BATTERY_BLOCK 1048576u

enum {
  PHPRNG_TEST_FREQUENCY = 0,
  PHPRNG_TEST_SERIAL2,
  PHPRNG_TEST_SERIAL3,
  PHPRNG_TEST_SERIAL4,
  PHPRNG_TEST_SERIAL5,
  PHPRNG_TEST_POKER,
  PHPRNG_TEST_COLLISION,
  PHPRNG_TEST_RUNS,
  PHPRNG_TEST_FOURIER,
  PHPRNG_TEST_COUNT
};

typedef struct {
  double chi2;
  double p_value;
  uint64_t dof;
  uint64_t samples; /* histogram entries: uniforms, tuples, hands, trials, runs or coefficient parts */
} phprng_test_result;

typedef struct phprng_battery phprng_battery;

/* Create a battery on HIP device `device`: 42 MB of histograms and about
 * 2.8 GB of transform and histogram scratch (128 blocks of 2^20 per pass).  The caller owns it (phprng_battery_destroy). */
phprng_status phprng_battery_create(phprng_battery **battery, int device);
phprng_status phprng_battery_destroy(phprng_battery *battery);
const char *phprng_battery_last_error(const phprng_battery *battery);

/* Zero the histograms and the kernel timing (asynchronous on `stream`). */
phprng_status phprng_battery_reset(phprng_battery *battery, void *stream);

/* Add `count` uniforms (a multiple of 2^20; device array, 16-byte aligned)
 * to the histograms; asynchronous on `stream`.  `r` must stay valid until the
 * stream completes.  Calls on one battery must be ordered on one stream. */
phprng_status phprng_battery_accumulate(phprng_battery *battery, const double *r, uint64_t count, void *stream);

/* Reduce the histograms to chi^2 on the device and fill out[PHPRNG_TEST_COUNT]
 * (host array); waits for `stream`. */
phprng_status phprng_battery_report(phprng_battery *battery, phprng_test_result *out, void *stream);

/* Copy the histogram of `test` (host array of `capacity` counts) and/or its
 * number of categories (*ncat; either pointer may be NULL); waits for `stream`. */
phprng_status phprng_battery_counts(phprng_battery *battery, int test, uint64_t *out, uint64_t capacity,
                                    uint64_t *ncat, void *stream);

/* The category probabilities of `test` used for the expected counts (host;
 * equal for the frequency and serial tests). */
phprng_status phprng_battery_probabilities(int test, double *out, uint64_t capacity, uint64_t *ncat);

/* The Fourier coefficients alone: for each block of `count` uniforms (device),
 * coef receives 2^20 doubles (device), the real and imaginary parts of
 * coefficients k = 0 .. 2^19 - 1 interleaved.  The histograms are unchanged. */
phprng_status phprng_battery_fourier(phprng_battery *battery, const double *r, uint64_t count, double *coef,
                                     void *stream);

/* Kernel time (ms) and launches since the last reset for the six kernel
 * classes (ms and launches are host arrays of 6): histogram keys, collision,
 * runs, transform pass 1, transform pass 2, histogram counting (HIP events
 * on the launch stream; waits for them). */
phprng_status phprng_battery_timing(phprng_battery *battery, double *ms, uint64_t *launches);

/* One-sided P-value min(Q, 1 - Q) of chi^2 with `dof` degrees of freedom (host). */
phprng_status phprng_chi2_pvalue(double chi2, double dof, double *p);

/* Interstream order of the Tests section (device arrays, asynchronous on
 * `stream`): out[t * nstreams + i] = in[i * length + t], i.e. the t-th
 * uniform of every stream, then the (t+1)-th.  in and out must not overlap;
 * nstreams <= 4,194,240. */
phprng_status phprng_interleave(const double *in, double *out, uint64_t nstreams, uint64_t length, void *stream);


/* ---- full-period local pattern (Sec. II, Figs. 3-4) --------------------------*/

/* Over one period n(p-1) of a width-32 instance every state (m_k, s_k)
 * occurs once, so the windows (c_k, c_{k+1}, ..., c_{k+D-1}) whose first
 * point lies in [x0, x0 + l0) are enumerated by that first point c and the
 * skip s = s_{k+1} of the next step, in O(p l0) steps:
 *   m = c^d mod n (d = e^{-1} mod (n-1)),
 *   c_{k+1} = (m + s)^e,  c_{k+2} = (m + s + (a s mod p))^e,  ...  (mod n).
 * The D-1 following points are binned by floor(c_j bins / n) per axis (the
 * first following point is the most significant digit of the cell index).
 * The full period takes s over [1, p); any sub-range [s_lo, s_hi) may be
 * given, and histograms of disjoint ranges add up.  The Tests section uses
 * l0 = 2^7 and 2^24 cells (bins = 2^(24/(D-1))) for D = 3, 4, 5. */
typedef struct {
  uint64_t n, e;       /* a width-32 instance (phprng_check_instance rules) */
  uint64_t x0, l0;     /* first points c in [x0, x0 + l0), x0 + l0 <= n */
  uint64_t s_lo, s_hi; /* skips in [s_lo, s_hi), 1 <= s_lo < s_hi <= p = 2^31 - 1 */
  uint32_t dim;        /* D, 2..5 */
  uint32_t bins;       /* cells per following axis; bins^(D-1) <= 2^24 */
} phprng_pattern;

/* Add the counts of `pat` to hist, a caller-owned device array of
 * bins^(D-1) uint64 counts (not cleared).  Runs on `stream` and waits for
 * it; uses stream-ordered scratch of about 2.5 bytes per key of a round of
 * up to 2^30 keys (at most about 2.8 GB). */
phprng_status phprng_pattern_histogram(const phprng_pattern *pat, uint64_t *hist, void *stream);

/* chi^2 of a histogram of `pat` (device) against the uniform model: each
 * following point uniform over [0, n), so a cell expects
 * T prod_j (w_{b_j} / n) with T = l0 (s_hi - s_lo) and w_b the number of
 * c in [0, n) with bin b; dof = cells - 1; P one-sided about the median as
 * for the battery.  *total receives the histogram's sum.  Any output pointer
 * may be NULL; waits for `stream` (uses 16 KB of stream-ordered scratch). */
phprng_status phprng_pattern_chi2(const phprng_pattern *pat, const uint64_t *hist, double *chi2, double *p_value,
                                  uint64_t *total, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PHPRNG_H */
