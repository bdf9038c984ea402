/*
 * rngx -- many independent per-thread random-number streams and their use in
 * a checkerboard Metropolis update of the 2D Ising ferromagnet, on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow Manssen, Weigel & Hartmann, "Random number
 * generators for massively parallel simulations on GPU" (arXiv:1204.6193):
 * thousands to millions of generator instances, one per updating unit, each
 * delivering its own stream (Introduction), with generator state kept in
 * fast on-chip storage during a launch and moved to and from device memory
 * once (Introduction; LCG section on state loads per Ising tile visit).
 *
 * General conventions
 *   - Plain C ABI.  Device pointers ("d_" prefix) are addresses in the
 *     memory of the device the handle was created on; host pointers are
 *     ordinary process memory.  `stream` is a hipStream_t passed as void*
 *     (NULL = the default stream).
 *   - Every call validates all arguments before it touches the device.  On
 *     any error nothing is modified and the call returns a negative status;
 *     rngx_last_error() gives a description (per calling thread).
 *   - Calls that take a stream only enqueue work on it and return; results
 *     are ready when the stream reaches that point.  Calls without a stream
 *     argument are synchronous.  A handle must not be used from two host
 *     threads at once, nor by two streams whose work overlaps.
 *   - Output buffers belong to the caller, must be 16-byte aligned and hold
 *     the stated number of elements; the library owns generator state and
 *     lattices (allocated by *_create, released by *_destroy).
 *
 * Streams and outputs
 *   - Stream s of a generator created with (kind, n_streams = S, seed)
 *     produces outputs u_0, u_1, ... (32-bit).  Every recursive generator
 *     steps first and then outputs.
 *   - Uniform fills write output k of stream s to out[k*S + s] (the paper's
 *     "warp order" for one XORShift-1024 instance; the interleaved sub-stream
 *     order for LCGs), k < count_per_stream.
 *   - FP32 uniforms are f = (u >> 8) * 2^-24, exact, in [0, 1).
 *   - XS1024W: a stream is one 32-bit lane of a 1024-bit instance; stream s
 *     is lane s % 32 of instance s / 32, so S must be a multiple of 32.
 *   - LFG521 / LFG1279: the values u_n = x_n / 2^32 follow the section's
 *     u_n = u_{n-r} + u_{n-s} mod 1 exactly.  One sequence (instance) is
 *     shared by 1024 streams, as by the threads of a block: stream s is lane
 *     s % 1024 of instance s / 1024, and output k of lane i is the instance's
 *     value 1024 k + i (warp order), so S must be a multiple of 1024.  Fills,
 *     consume, skip, state images and Ising sweeps (L a multiple of 64) take
 *     these kinds; ragged fills, batches and the server do not.
 *
 * Seeding (the paper seeds instances "with another RNG"; the exact indices
 * are this library's definition), with SM(k) = splitmix64 output k of
 * `seed`, i.e. mix64(seed + k * 0x9E3779B97F4A7C15):
 *   LCG32    x = low32(SM(1+s))            LCG64  x = SM(1+s)
 *   MWC      x = low32(SM(1+s)), carry = high32(SM(1+s)) mod (a-1), x = 1 if both 0
 *   XORWOW   (x,y) (z,w) (v,d) = low/high words of SM(1+3s), SM(2+3s), SM(3+3s);
 *            x = 1 if x..v are all 0
 *   PHILOX   key = (low32, high32) of SM(1+s), position 0
 *   XS1024W  word i of instance g = low32 (i even) / high32 (i odd) of
 *            SM(1 + 16 g + i/2); Weyl seed y0 = high32(SM(0)) shared by all
 *            instances; step counter 0
 *   LFG521 / LFG1279 (lags (r, s) = (521, 353) / (1279, 861)): instance g
 *            holds the last r values of its sequence; word j of instance g =
 *            low32 (j even) / high32 (j odd) of SM(1 + H g + j/2), H = (r+1)/2,
 *            and if all r words are even, word 0 gets its low bit set
 *   MWC_DIFF stream s uses multiplier a_s, the (s+1)-th largest a < 2^32
 *            for which a*2^32 - 1 and (a*2^32 - 2)/2 are both prime (the MWC
 *            section's downward search from 4294967118; a_0 = 4294967118);
 *            x = low32(SM(1+s)), carry = high32(SM(1+s)) mod (a_s - 1),
 *            x = 1 if both 0.  At most 2^21 streams (every a_s > 2^31).
 *   LCG32_SUB / LCG64_SUB: one global sequence g_0 = the LCG32 / LCG64
 *            stream-0 value above, g_{n+1} = a g_n + c; stream s starts at
 *            g_s and steps S positions with the S-step map (A_S, C_S), so
 *            output k of stream s is g_{s + (k+1) S} and an interleaved fill
 *            is the global sequence from position S on
 *
 * Checkpoint image (rng_get_state / rng_set_state), little-endian,
 * structure of arrays:
 *   LCG32    u32 x[S]                    LCG64   u64 x[S]
 *   MWC      u64 y[S], y = carry << 32 | x
 *   XORWOW   u32 x[S] y[S] z[S] w[S] v[S] d[S]
 *   PHILOX   u32 k0[S] k1[S] u64 pos[S]  (pos = outputs consumed)
 *   XS1024W  u32 W[S] (W[32g+i] = word i of instance g, word 0 most
 *            significant) u64 n[S/32] (steps taken) u32 y0
 *   LFG521 / LFG1279  u32 X[S/1024][r]: X[g][j] = x_{n-r+j} of instance g,
 *            oldest first (an instance whose r words are all even is refused)
 *   MWC_DIFF u64 y[S] (as MWC), then u32 a[S] (the multipliers; an image
 *            whose multipliers differ from the handle's is refused with
 *            RNGX_E_STATE)
 *   LCG32_SUB u32 x[S], u32 A_S, u32 C_S   LCG64_SUB u64 x[S], u64 A_S, C_S
 *            (rng_set_state refuses an image whose (A_S, C_S) is not the
 *            handle's, with RNGX_E_STATE)
 */
#ifndef RNGX_H
#define RNGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RNGX_LCG32 = 1,         /* x <- 1664525 x + 1013904223 mod 2^32; out x          (LCG section)  */
    RNGX_LCG64 = 2,         /* x <- a x + c mod 2^64 (a, c of the LCG section); out x >> 32        */
    RNGX_MWC = 3,           /* lag-1 multiply-with-carry, base 2^32, a = 4294967118; out x (MWC sec.) */
    RNGX_XORWOW = 4,        /* 160-bit xorshift (2,1,4) + Weyl d += 362437; out d + v (XORShift sec.) */
    RNGX_PHILOX4X32_10 = 5, /* counter-based Philox4x32, 10 rounds (counter-based section)         */
    RNGX_XS1024W = 6,       /* the paper's XORShift-1024 (329,347,344) + Weyl (XORShift section)    */
    RNGX_PHILOX4X32_7 = 7,  /* Philox4x32 with 7 rounds (counter-based section); otherwise as 5     */
    RNGX_LCG32_SUB = 8,     /* LCG32 sub-streams of one sequence (eq. lcg_skipping, t = S), below   */
    RNGX_LCG64_SUB = 9,     /* LCG64 sub-streams of one sequence, as 8                              */
    RNGX_LFG521 = 10,       /* additive lagged Fibonacci x_n = x_{n-521} + x_{n-353} mod 2^32, an   */
                            /* instance shared by 1024 streams (Lagged Fibonacci section), below     */
    RNGX_LFG1279 = 11,      /* as 10 with lags (1279, 861)                                          */
    RNGX_MWC_DIFF = 12      /* MWC as 3 with a different safe-prime multiplier per stream (MWC sec.) */
} rngx_kind;

typedef enum {
    RNGX_OK = 0,
    RNGX_E_INVALID = -1,  /* bad kind, null pointer, zero size, bad beta, unknown handle        */
    RNGX_E_ALIGN = -2,    /* S % 32 != 0 for XS1024W; L % 16 != 0 or L < 16; unaligned buffer  */
    RNGX_E_NOMEM = -3,    /* device allocation failed                                          */
    RNGX_E_HIP = -4,      /* a HIP runtime call failed                                         */
    RNGX_E_OVERFLOW = -5, /* element or byte counts overflow 64 bits                           */
    RNGX_E_STATE = -6,    /* a state image holds a fixed point of the generator or bad size    */
    RNGX_E_BUSY = -7      /* resource temporarily unavailable                                  */
} rngx_status;

typedef struct rngx_gen_s *rngx_gen;     /* opaque; owns the device state of S streams      */
typedef struct rngx_ising_s *rngx_ising; /* opaque; owns L*L int8 spins and L*L/4 streams    */
typedef struct rngx_ising_batch_s *rngx_ising_batch; /* opaque; lattices swept together   */
typedef struct rngx_ragged_s *rngx_ragged;           /* opaque; uneven per-stream requests */
typedef struct rngx_server_s *rngx_server;           /* opaque; request server             */

typedef struct {
    uint32_t slots;          /* HIP streams the requests are spread over (>= 1)                 */
    uint32_t max_inflight;   /* requests on the device at once (>= 1); 1 with 1 slot = plain FIFO */
    uint64_t memory_budget;  /* bytes of device memory: request outputs, Ising jobs, jump tables  */
    uint64_t seed;           /* master seed of every client generator and Ising job              */
} rngx_server_config;

/* A fill configuration (see rng_fill_configs): paced (1) or free-running (0)
 * workgroups, streams per thread (XS1024W: 2, one lane pair of an instance),
 * threads per workgroup.  All configurations of a kind produce the same
 * values; they differ only in speed. */
typedef struct rngx_fill_config {
    int32_t paced;
    int32_t streams_per_thread;
    int32_t block;
} rngx_fill_config;

typedef struct {
    int32_t status;    /* RNGX_OK once done                                                       */
    void *d_output;    /* device memory owned by the server until srv_release (see srv_submit_*) */
    uint64_t n_values; /* fill: count; Ising: L*L                                                 */
    double latency_s;  /* from submission to completion on the device                             */
} rngx_request_result;

/* Create S = n_streams streams of `kind` seeded from `seed` as above, on the
 * current device.  Seeding runs on the device; the call returns when it is
 * done.  *out receives the handle.  Errors: RNGX_E_INVALID (kind, S = 0,
 * out NULL), RNGX_E_ALIGN (XS1024W with S % 32 != 0, LFG with S % 1024 != 0), RNGX_E_OVERFLOW
 * (S > 2^36; MWC_DIFF: S > 2^21), RNGX_E_NOMEM.  MWC_DIFF's multipliers are
 * found on the device (a Rabin-Miller test of every candidate) once per
 * process and kept for later handles.  (No XS1024W instance can be seeded all-zero:
 * at most one of its 16 distinct splitmix64 words is 0.) */
rngx_status rng_create(rngx_kind kind, uint64_t n_streams, uint64_t seed, rngx_gen *out);

/* XS1024W only: sub-stream seeding (XORShift section: the sequence is cut
 * into blocks of 2^137 numbers, assigned to the instances in turn).  Every
 * instance g starts from the state rng_create gives instance 0 and skips
 * g * 2^137 steps; step counters are 0 (g * 2^137 mod 2^64) and the Weyl
 * seed is rng_create's.  Synchronous.  Errors as rng_create, and
 * RNGX_E_INVALID for any other kind. */
rngx_status rng_create_substreams(rngx_kind kind, uint64_t n_streams, uint64_t seed, rngx_gen *out);

/* Release the handle and its device memory (waits for the device first). */
rngx_status rng_destroy(rngx_gen g);

/* Kind and stream count of a handle; either output pointer may be NULL. */
rngx_status rng_info(rngx_gen g, rngx_kind *kind, uint64_t *n_streams);

/* Write the next count_per_stream outputs of every stream to the device
 * buffer d_out (S * count_per_stream u32 elements, out[k*S + s]) and advance
 * every stream by count_per_stream.  count 0 is a no-op.  Errors:
 * RNGX_E_INVALID, RNGX_E_ALIGN (d_out not 16-byte aligned),
 * RNGX_E_OVERFLOW (S * count * 4 bytes overflows). */
rngx_status rng_fill_u32(rngx_gen g, uint32_t *d_out, uint64_t count_per_stream, void *stream);

/* As rng_fill_u32, writing f = (u >> 8) * 2^-24 as float. */
rngx_status rng_fill_f32(rngx_gen g, float *d_out, uint64_t count_per_stream, void *stream);

/* Generate count_per_stream outputs of every stream without storing them:
 * d_xor[s] (S u32 elements) receives the XOR of stream s's outputs.  The
 * numbers are produced exactly as by rng_fill_u32 and the streams advance
 * the same way; this isolates generation from output bandwidth (the paper's
 * Table 3 peak rates are measured without storing the numbers). */
rngx_status rng_consume(rngx_gen g, uint32_t *d_xor, uint64_t count_per_stream, void *stream);

/* Advance every stream by n outputs without producing them (jump-ahead):
 * LCGs by the n-step affine map (eq. lcg_skipping), MWC by y <- a^n y mod
 * (a 2^32 - 1) (MWC_DIFF: each stream with its own a and modulus), XORWOW
 * and XS1024W by the n-th power of the GF(2)
 * transition matrix of their xorshift part (the XORShift section's
 * sub-stream seeding multiplies by such a power) plus n steps of the Weyl
 * term, Philox by its counter, LFG instances (1024 n values each) by
 * J(x) = x^(1024 n) mod (x^r - x^(r-s) - 1) over Z/2^32 applied to the
 * window.  The result equals producing and discarding
 * n outputs. */
rngx_status rng_skip(rngx_gen g, uint64_t n, void *stream);

/* Fill configurations and their autotuner.  The block size, streams per
 * thread and pacing of rng_fill_u32/_f32 are chosen per handle from a fixed
 * list per kind (the defaults were measured at 2^20 streams x 4096; other
 * sizes or devices may prefer others).  Pacing keeps the workgroups of a
 * large fill within a few bands of rows of each other, which HBM rewards for
 * the interleaved layout; it needs every workgroup resident and is skipped
 * otherwise.  rng_consume and rng_fill_ragged_u32 do not use these.
 *
 * rng_fill_configs: the list for `kind` in index order; out (n entries) may
 * be NULL to ask for *n only.
 * rng_set_fill_config: use entry `index` for this handle (-1: the kind's
 * default); rng_get_fill_config: the entry in use (the default resolved).
 * rng_autotune_fill: times every entry on this handle's fills of `count`
 * outputs per stream into d_out (S*count u32 elements, overwritten), one
 * warm-up and `reps` (>= 1) timed launches each, selects the fastest and
 * leaves the stream state as it was (it is saved to device memory that the
 * call allocates and frees).  ms_out (may be NULL) receives the mean launch
 * time of each entry in index order.  Synchronizes the stream. */
rngx_status rng_fill_configs(rngx_kind kind, rngx_fill_config *out, int32_t *n);
rngx_status rng_set_fill_config(rngx_gen g, int32_t index);
rngx_status rng_get_fill_config(rngx_gen g, int32_t *index);
rngx_status rng_autotune_fill(rngx_gen g, uint32_t *d_out, uint64_t count_per_stream, int32_t reps, float *ms_out,
                              void *stream);

/* Ising plans and their autotuner.  A lattice runs either as strips held on
 * chip by cooperating workgroups (one per strip; the strip count is the
 * sub-lattice tiling) or, if no strip plan fits, one launch per colour pass.
 * Every plan gives the same spins, energies and stream states.
 * ising_plans: the strip counts that fit this lattice, most strips first,
 * then 0 (the per-pass path); strips_out (n entries) may be NULL to ask for
 * *n only.  ising_set_plan: use `strips` strips (0: per pass); synchronizes
 * the device.  ising_autotune: times every plan on `reps` (>= 1) calls of
 * n_sweeps sweeps at beta after one warm-up call, keeps the fastest and
 * restores the spins and stream states it started from (saved to device
 * memory the call allocates and frees); ms_out (may be NULL) receives the
 * mean call time of each plan in ising_plans order.  Synchronizes the device. */
rngx_status ising_plans(rngx_ising lat, uint32_t *strips_out, int32_t *n);
rngx_status ising_set_plan(rngx_ising lat, uint32_t strips);
rngx_status ising_autotune(rngx_ising lat, double beta, uint64_t n_sweeps, int32_t reps, float *ms_out, void *stream);

/* Uneven per-stream requests (streams of very different length served in one
 * pass, the batched form of rng_fill_u32).  `offsets` (host memory, copied)
 * holds n_units + 1 non-decreasing element indices, n_units = S, or S/32
 * instances for XS1024W.  Each rng_fill_ragged_u32 call writes
 *   small-state kinds: the next offsets[s+1]-offsets[s] outputs of stream s
 *                      to d_out[offsets[s] ...], in order;
 *   XS1024W:           len = offsets[g+1]-offsets[g] values of instance g in
 *                      warp order (step k, lane i at d_out[offsets[g] + 32k+i]);
 *                      the instance takes ceil(len/32) steps and the lanes
 *                      of a last partial step are dropped;
 * and advances the streams accordingly.  Long requests are cut into chunks
 * whose start states come from jump-ahead, so a call costs two launches on
 * `stream` whatever the lengths; it may be captured in a HIP graph.  d_out
 * must be 4-byte aligned and hold offsets[n_units] elements.  The generator
 * must outlive the plan (rng_destroy returns RNGX_E_BUSY meanwhile).
 * Errors: RNGX_E_INVALID (wrong count, decreasing offsets, NULL),
 * RNGX_E_OVERFLOW (output size, or 2^32 or more chunks), RNGX_E_NOMEM. */
rngx_status rng_ragged_create(rngx_gen g, const uint64_t *offsets, uint64_t n_offsets, rngx_ragged *out);
rngx_status rng_fill_ragged_u32(rngx_ragged r, uint32_t *d_out, void *stream);
rngx_status rng_ragged_destroy(rngx_ragged r);

/* Shapes of a ragged plan and their autotuner.  The value of a shape is, for
 * XS1024W, the generating rows per compute unit (fewer rows: fewer jumps at
 * row starts, less parallelism), else the outputs per chunk (a lane's or a
 * wave's; smaller chunks: more jumps, better balance).  Every shape writes
 * the same values and leaves the same stream states.
 * rng_ragged_shapes: the values for `kind` in index order (shape 0, the
 * default, first); values (n entries) may be NULL to ask for *n only.
 * rng_ragged_set_shape: re-plan with shape `index`; synchronizes the device.
 * rng_ragged_autotune: times every shape on `reps` (>= 1) fills into d_out
 * (overwritten; as for rng_fill_ragged_u32) after one warm-up fill, keeps the
 * fastest and restores the streams to their state before the call (saved to
 * device memory the call allocates and frees); ms_out (may be NULL, else one
 * entry per shape) receives the mean fill time of each shape; synchronizes
 * the device.  Re-planning frees the device buffers a fill reads: a graph
 * captured before either call must not be replayed after it.  Errors:
 * RNGX_E_INVALID (kind without ragged fills, bad index, reps < 1, NULL),
 * RNGX_E_NOMEM, RNGX_E_HIP (if re-planning fails, fills return RNGX_E_HIP
 * until a shape is set again). */
rngx_status rng_ragged_shapes(rngx_kind kind, uint64_t *values, int32_t *n);
rngx_status rng_ragged_set_shape(rngx_ragged r, int32_t index);
rngx_status rng_ragged_get_shape(rngx_ragged r, int32_t *index);
rngx_status rng_ragged_autotune(rngx_ragged r, uint32_t *d_out, int32_t reps, float *ms_out, void *stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid it): the same fill
 * as rng_ragged_create(g, offsets, n_offsets) followed by
 * rng_fill_ragged_u32 -- same values, same final stream states -- made in
 * one call that allocates nothing.  The plan is made on the host for every
 * call and staged, with the chunk states, in a fixed 64 MiB device array
 * that each device running the library holds until the process ends.
 * Synchronous: returns when the fill is done.  Calls are serialised within
 * the process (they share the array); calls from other processes use their
 * own.  Not for graph capture.  Errors: those of rng_ragged_create, and
 * RNGX_E_OVERFLOW when the plan needs more than the 64 MiB (about a million
 * chunks of 4096 values for the small-state kinds, far more values for the
 * LCGs and XS1024W), before anything is modified. */
rngx_status rng_fill_ragged_u32_noalloc(rngx_gen g, const uint64_t *offsets, uint64_t n_offsets, uint32_t *d_out,
                                        void *stream);

/* Copy the handle's state image (layout above) to host memory.  If host_buf
 * is NULL only *bytes is set to the image size.  Otherwise *bytes must be at
 * least that size; the call waits for `stream` and then copies. */
rngx_status rng_get_state(rngx_gen g, void *host_buf, size_t *bytes, void *stream);

/* Replace the handle's state by an image (layout above) of exactly the
 * image size.  Images holding a fixed point (XS1024W all-zero instance,
 * XORWOW all-zero xorshift words, MWC y = 0 or y >= a 2^32 - 1) are refused
 * with RNGX_E_STATE.  The copy is ordered on `stream` and the host buffer
 * may be reused when the call returns. */
rngx_status rng_set_state(rngx_gen g, const void *host_buf, size_t bytes, void *stream);

/* Create an L x L periodic Ising lattice (J = 1, h = 0; Sec. 2 application
 * test) with int8 spins +-1 at y*L + x, hot-started: spin i = +1 iff bit 63
 * of splitmix64 output i+1 of (seed ^ 0xD1B54A32D192ED03) is set.  It owns
 * S = L*L/4 streams of `kind` seeded from `seed` as rng_create would; stream
 * s = y*(L/4) + x/4 drives the four sites x0..x0+3 (x0 = 4*(x/4)) of row y.
 * Synchronous.  Errors: RNGX_E_ALIGN unless L % 16 == 0 and L >= 16 (LFG
 * kinds: L % 64 == 0, whole 1024-stream instances), RNGX_E_OVERFLOW when
 * the kind cannot hold L*L/4 streams (MWC_DIFF: L > 2896).  LFG lattices
 * run on chip when strips of whole instances fit (every strip keeps its
 * instances' windows in LDS for the call and makes each pass's values there
 * row by row; e.g. r = 521 up to L = 4096, r = 1279 up to L = 2048), else
 * one launch per colour pass with a workgroup per instance; multi-hit
 * sweeps of LFG lattices always take the per-pass form.  Either gives the
 * same spins, energies and windows. */
rngx_status ising_create(uint32_t L, rngx_kind kind, uint64_t seed, rngx_ising *out);

/* Run n_sweeps checkerboard Metropolis sweeps at inverse temperature beta
 * (finite, >= 0).  A sweep updates colour 0 (x+y even), then colour 1; in
 * pass c stream s updates site x0 + ((c+y)&1) with its next output r and
 * then site x0 + 2 + ((c+y)&1) with the following one.  A flip with energy
 * change dE is accepted iff dE <= 0 or r < floor(exp(-beta dE) 2^32), the
 * two thresholds (dE = 4, 8) being computed on the host in IEEE double.
 * If d_energy_trace is not NULL, entry t (n_sweeps int32 elements) receives
 * E = -sum s(x,y)[s(x+1,y) + s(x,y+1)] after sweep t. */
rngx_status ising_sweep(rngx_ising lat, double beta, uint64_t n_sweeps, int32_t *d_energy_trace,
                        void *stream);

/* Multi-hit sweeps (Sec. 2 and the Philox discussion: k updates per load of
 * the generator states, here read as k Metropolis updates of each visited
 * site in a row, its neighbours fixed).  In pass c stream s gives site
 * x0 + ((c+y)&1) its next `hits` outputs, one per update, and site
 * x0 + 2 + ((c+y)&1) the `hits` after those; each update flips the site
 * under the rule above, so a sweep draws 4*hits outputs per stream.
 * hits = 1 is ising_sweep.  Errors as ising_sweep, and RNGX_E_INVALID
 * unless 1 <= hits <= 2^20. */
rngx_status ising_sweep_hits(rngx_ising lat, double beta, uint64_t n_sweeps, uint32_t hits,
                             int32_t *d_energy_trace, void *stream);

/* How the lattice is swept: *strips receives the number of workgroups that
 * hold the lattice on chip as horizontal strips for a whole ising_sweep call
 * (1 = a single workgroup), or 0 when every colour pass is a separate launch
 * that streams spins and state through memory (large L).  Results do not
 * depend on it.  Any output pointer may be NULL. */
rngx_status ising_info(rngx_ising lat, uint32_t *L, rngx_kind *kind, uint32_t *strips);

/* Borrow the device pointer of the spins (L*L int8, row-major).  The
 * pointer stays valid until ising_destroy; writes through it are allowed
 * (values must stay +-1) and are ordered by the caller's streams. */
rngx_status ising_spins(rngx_ising lat, int8_t **d_spins);

/* Copy the L*L spins to host memory (waits for `stream`), or replace them
 * from host memory (every value must be +1 or -1, else RNGX_E_STATE; the
 * copy is ordered on `stream` and done when the call returns).  With the
 * generator image these form the lattice checkpoint. */
rngx_status ising_get_spins(rngx_ising lat, int8_t *host_spins, void *stream);
rngx_status ising_set_spins(rngx_ising lat, const int8_t *host_spins, void *stream);

/* Borrow the generator handle that drives the lattice (for checkpoints via
 * rng_get_state / rng_set_state).  It must not be destroyed by the caller. */
rngx_status ising_rng(rngx_ising lat, rngx_gen *g);

/* Whether the lattice is valid (waits for `stream`): *invalid receives 0,
 * or 1 if a strip of a multi-workgroup sweep gave up waiting for a
 * neighbour's boundary spins (a bounded wait, reached only when the strips
 * could not run at the same time), after which spins and state are
 * meaningless until replaced by ising_set_spins and rng_set_state. */
rngx_status ising_status(rngx_ising lat, uint32_t *invalid, void *stream);

/* Release the lattice, its spins and its streams. */
rngx_status ising_destroy(rngx_ising lat);

/* Batched replicas: group n lattices of one kind (distinct handles, one
 * device) so that one launch sweeps them all -- many independent Ising
 * replicas of uneven size and temperature, as in the paper's use of one
 * generator instance per updating thread.  Each ising_batch_run gives
 * replica i n_sweeps[i] sweeps at betas[i] (finite, >= 0) and, when d_traces
 * and d_traces[i] are not NULL, its energies in d_traces[i] (n_sweeps[i]
 * int32, as ising_sweep writes them).  Results equal ising_sweep on each
 * lattice.  A run is a one-word reset plus one kernel launch on `stream`
 * and may be captured in a HIP graph.  The lattices must outlive the batch:
 * ising_destroy returns RNGX_E_BUSY for a lattice that a batch holds.
 * Errors: RNGX_E_INVALID (n = 0, NULL arrays, unknown or repeated handles,
 * mixed kinds or devices, bad beta).
 *
 * Large replicas run as gangs of strip workgroups that wait on each other
 * every pass, so all strips of a gang must run at the same time.  Outside
 * graph capture a run is a cooperative launch, which guarantees that.  A
 * captured run relies on the grid being no larger than what fits on the
 * device at once: other kernels running beside it only delay it, unless
 * they hold the device for longer than a gang member waits for the others
 * to start (60 s); then that replica is marked invalid (ising_status,
 * ising_batch_status) rather than left with wrong spins unreported.
 * ising_batch_status waits for `stream` and counts the invalid replicas. */
rngx_status ising_batch_create(const rngx_ising *lats, uint32_t n, const double *betas, const uint64_t *n_sweeps,
                               int32_t *const *d_traces, rngx_ising_batch *out);
rngx_status ising_batch_run(rngx_ising_batch b, void *stream);
rngx_status ising_batch_status(rngx_ising_batch b, uint32_t *n_invalid, void *stream);
/* The launch shape of a run: work items (one per single-workgroup replica,
 * one per strip of a gang), workgroups that fit on the device at once, and
 * workgroups of the persistent grid (the smaller of the two).  Any pointer
 * may be NULL. */
rngx_status ising_batch_info(rngx_ising_batch b, uint32_t *n_items, uint32_t *resident, uint32_t *grid);

/* Launch shapes of the batch kernel and their autotuner.  A shape gives the
 * threads per workgroup, the most lattice sites one workgroup holds per
 * thread (one random number per site and sweep: the numbers per thread) and
 * the LDS a strip may take; together they fix how each replica is tiled into
 * strips (one workgroup if it fits, else a gang of strips, else streamed
 * through memory).  Every shape gives the same spins, energies and stream
 * states.  ising_batch_shapes: the list in index order; out (n entries) may
 * be NULL to ask for *n only.  ising_batch_set_shape: re-plan the batch with
 * shape `index` (a new batch uses shape 0); synchronizes the device.
 * ising_batch_autotune: times every shape on `reps` (>= 1) runs after one
 * warm-up run, each replica's sweep count scaled by one factor so that the
 * longest runs max_sweeps (at least one sweep each; the real counts when
 * they are all <= max_sweeps), with no energy traces; keeps the fastest and
 * restores every replica's spins, stream states and status as they were
 * (saved to device memory the call allocates and frees); ms_out (may be
 * NULL, else one entry per shape of ising_batch_shapes) receives the mean
 * run time of each shape; synchronizes the device.  Re-planning frees the
 * device buffers a run reads: a graph captured before ising_batch_set_shape
 * or ising_batch_autotune must not be replayed after it.  Errors:
 * RNGX_E_INVALID (bad index, max_sweeps or reps = 0), RNGX_E_NOMEM,
 * RNGX_E_HIP (if re-planning fails the batch's runs return RNGX_E_HIP
 * until a shape is set again). */
typedef struct {
    uint32_t threads;          /* per workgroup: 256, 512 or 1024              */
    uint32_t sites_per_thread; /* most lattice sites per thread in a workgroup */
    uint32_t lds_cap;          /* most LDS bytes of one strip                  */
} rngx_batch_shape;
rngx_status ising_batch_shapes(rngx_batch_shape *out, int32_t *n);
rngx_status ising_batch_set_shape(rngx_ising_batch b, int32_t index);
rngx_status ising_batch_get_shape(rngx_ising_batch b, int32_t *index);
rngx_status ising_batch_autotune(rngx_ising_batch b, uint64_t max_sweeps, int32_t reps, float *ms_out, void *stream);
rngx_status ising_batch_destroy(rngx_ising_batch b);

/* Served form.  A server admits requests in arrival order as soon as its
 * device-memory budget and in-flight limit allow (continuous batching:
 * requests that arrive while others run are started without waiting for
 * them), spreads them over `slots` streams so that their work overlaps, and
 * keeps one generator stream per (client, kind) resident on the device:
 * stream 0 (XS1024W: instance 0) of rng_create(kind, 1 (XS1024W: 32),
 * splitmix64 output 16*client + kind of cfg->seed).  A client's requests of
 * one kind run in submission order; results depend only on the client's own
 * requests, not on what else is served.  The server allocates its budget
 * once; no request allocates device memory.
 *   (kinds: every kind but the sub-stream LCGs, whose streams only exist as
 *   parts of one S-stream sequence, MWC_DIFF, whose multiplier is a
 *   property of a stream index, and the LFG kinds, whose instances are
 *   1024 streams: RNGX_E_INVALID)
 *   srv_submit_fill:  the next `count` (<= 2^28) outputs of the (client, kind)
 *     stream, contiguous (XS1024W: the instance's values in warp order), as
 *     uint32 or as FP32 (u >> 8) * 2^-24 if as_f32.  Long requests are cut
 *     into chunks that start from jump-ahead, so one request uses the whole
 *     device.
 *   srv_submit_ising: a hot-started L x L lattice (L % 16 == 0, L >= 16) of
 *     the client's Ising job number j (counting that client's jobs from 0),
 *     seeded with splitmix64 output 2^62 + 2^24 client + j of cfg->seed as
 *     ising_create would seed it, swept n_sweeps times at beta; the output
 *     holds the L*L int8 spins, then (at offset L*L rounded up to 16) the
 *     n_sweeps int32 energies.
 * Both return a ticket at once; a request larger than the whole budget is
 * refused with RNGX_E_NOMEM.  srv_wait blocks up to timeout_s seconds (< 0:
 * no limit) and returns RNGX_E_BUSY if the request is not done;
 * srv_wait_any blocks likewise until some request finishes that no
 * srv_wait_any call has returned yet (completion order) and reports it;
 * srv_release returns the output memory to the budget.  srv_destroy waits
 * for the device and frees everything.
 *
 * Admission: a request that does not fit in the free budget yet is passed
 * by later requests of other (client, kind) pairs that do fit -- never by a
 * later request of its own pair, whose stream order it fixes -- until 64
 * later requests have passed it; from then on nothing is admitted before
 * it, so a large request cannot be starved.
 *
 * srv_cancel withdraws a request that has not been admitted yet (the
 * ticket becomes unknown, its (client, kind) stream does not advance, an
 * Ising job's number stays used); RNGX_E_BUSY once it is on the device.
 *
 * srv_get_client_state / srv_set_client_state export and import the state
 * of one (client, kind) stream in the checkpoint image of rng_get_state for
 * 1 stream (XS1024W: 32), so that a new server (same or other seed) can
 * continue a client exactly where an old one stopped.  Both are synchronous
 * and return RNGX_E_BUSY while requests of that (client, kind) are queued or
 * running; get with host_buf NULL reports the size in *bytes; set refuses an
 * image of the wrong size or a fixed point (RNGX_E_STATE).  A pair that has
 * not served yet is seeded first. */
rngx_status srv_create(const rngx_server_config *cfg, rngx_server *out);
rngx_status srv_submit_fill(rngx_server s, uint32_t client, rngx_kind kind, uint64_t count, int as_f32,
                            uint64_t *ticket);
rngx_status srv_submit_ising(rngx_server s, uint32_t client, rngx_kind kind, uint32_t L, double beta,
                             uint32_t n_sweeps, uint64_t *ticket);
rngx_status srv_wait(rngx_server s, uint64_t ticket, double timeout_s, rngx_request_result *res);
rngx_status srv_wait_any(rngx_server s, double timeout_s, uint64_t *ticket, rngx_request_result *res);
rngx_status srv_release(rngx_server s, uint64_t ticket);
rngx_status srv_cancel(rngx_server s, uint64_t ticket);
rngx_status srv_get_client_state(rngx_server s, uint32_t client, rngx_kind kind, void *host_buf, size_t *bytes);
rngx_status srv_set_client_state(rngx_server s, uint32_t client, rngx_kind kind, const void *host_buf, size_t bytes);
rngx_status srv_destroy(rngx_server s);

/* Description of the calling thread's most recent error ("" if none). */
const char *rngx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RNGX_H */
