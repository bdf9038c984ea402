// Internal declarations of the rngx library: handles, launchers and status
// helpers shared by the HIP translation units.  The generators themselves are
// in rngx_device.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "rngx.h"
#include "rngx_device.h"

namespace rngx {

// ---------------------------------------------------------------------------
// Handles.  The device state is one allocation laid out exactly as the
// checkpoint image documented in rngx.h (structure of arrays).
struct Gen {
    uint64_t magic;
    rngx_kind kind;
    uint64_t S;
    int device;
    uint8_t *d_state;
    size_t state_bytes;
    const void *owner;  // the lattice that owns this generator, if any
    uint32_t plans;     // ragged plans that hold this generator
    uint32_t *d_ring;   // fill pacing counters (kRing x kPaceSlots)
    int n_cu;           // compute units of the device
    int fill_cfg;       // fill configuration (index into the kind's list), -1: default
    int resident[8];    // per configuration: workgroups that fit at once, -1: not known yet
    uint64_t sub_a, sub_c;  // sub-stream LCG kinds: the S-step map (A_S, C_S) of the image header
    uint32_t *d_aux;        // LFG kinds: r words staging a jump polynomial
};
inline bool is_sub_lcg(rngx_kind k) { return k == RNGX_LCG32_SUB || k == RNGX_LCG64_SUB; }
inline bool is_lfg(rngx_kind k) { return k == RNGX_LFG521 || k == RNGX_LFG1279; }
constexpr uint64_t kLfgLanes = 1024;  // streams of one lagged Fibonacci instance
constexpr int kMaxFillConfigs = 8;

// One chunk of one stream's (XS1024W: one instance's) ragged request.
struct RaggedItem {
    uint64_t unit;   // stream, or XS1024W instance
    uint64_t out;    // output index of the chunk's first value
    uint64_t j;      // chunk index: the chunk starts j*C outputs (steps) in
    uint64_t nvals;  // values the chunk writes
    uint32_t len;    // outputs (XS1024W: instance steps) the chunk takes
    uint32_t last;   // the chunk ends the request: it writes the state back
};

struct Ragged {
    uint64_t magic;
    Gen *gen;
    uint64_t n_items, total;
    RaggedItem *d_items;
    uint8_t *d_scratch;  // chunk start states
    uint64_t *d_t64;     // jump tables (see jump_table)
    uint32_t *d_t32;
    uint64_t step;       // jump table step: chunk j starts j*step outputs (steps) in
    uint32_t n_slots;    // XS1024W: rows of the generation kernel
    uint32_t *d_slots;   // XS1024W: first item of each row, n_slots + 1 entries
    uint64_t *d_lane;    // affine kinds: (i+1)-step maps for lanes i = 0..63, then the 64-step map
    int shape;                       // index into the kind's ragged shapes (ragged_shape_value)
    std::vector<uint64_t> offsets;   // the request list, kept to re-plan under another shape
};

// How a lattice is swept: as strips held on chip by co-resident
// workgroups (strips = true) or by one launch per colour pass.
struct IsingPlan {
    bool strips;
    uint32_t R;        // rows per strip
    uint32_t nwg;      // strips = workgroups
    uint32_t units;    // update units per strip
    uint32_t spt;      // units per thread
    uint32_t threads;  // threads per workgroup
    uint32_t lds;      // dynamic LDS bytes per workgroup
    bool early;        // top and bottom rows in the first and last unit slots
};

struct Ising {
    uint64_t magic;
    uint32_t L;
    int device;
    int8_t *d_spins;
    Gen *gen;
    IsingPlan plan;
    uint64_t *d_halo;    // strips: 2 slots x nwg x 2 rows x L/4 tagged words (4 spins | pass tag << 32)
    uint32_t halo_nwg;   // strips the halo allocation is sized for
    uint32_t *d_err;     // strips: set if a neighbour wait gave up
    int32_t *d_partial;  // per-pass path: per-block energy partials
    uint64_t epoch;      // passes run since the halo tags were last cleared
    uint32_t batches;    // batches that hold this lattice
};

// A launch shape of the batch kernel: threads per workgroup, most lattice
// sites per workgroup and thread (one random draw per site and sweep, so the
// numbers per thread), and the LDS a strip may take (which bounds the strip
// height, i.e. the sub-lattice tiling).  The autotuner picks one of a fixed
// list.
struct BatchShape {
    uint32_t threads, sites_per_thread, lds_cap;
};
constexpr int kBatchShapes = 5;
extern const BatchShape kBatchShape[kBatchShapes];

// A fixed list of lattices swept together in one launch.
struct IsingBatch {
    uint64_t magic;
    int device;
    rngx_kind kind;
    uint32_t n;
    void *d_reps;        // replica descriptors (device)
    void *d_items;       // (replica, strip) work items, gangs consecutive, decreasing work
    uint32_t n_items;
    uint32_t *d_next;    // work counter
    void *d_halo;        // tagged halo words of the gang replicas
    uint32_t lds, grid;  // launch shape
    uint32_t resident;   // workgroups of the batch kernel that fit at once
    bool gangs;          // some replica runs as a gang of strips
    int shape;           // index into kBatchShape
    int n_cu;
    Ising **lats;        // host copy of the members
    std::vector<double> betas;        // the run's arguments, kept to re-plan
    std::vector<uint64_t> sweeps;     //   under another shape
    std::vector<int32_t *> traces;
};

struct Server;  // request server (server.hip)
constexpr uint64_t kMaxServedValues = 1ull << 28;  // largest served fill
rngx_status server_create(const rngx_server_config *cfg, Server **out);
rngx_status server_submit_fill(Server *s, uint32_t client, rngx_kind kind, uint64_t count, int f32, uint64_t *ticket);
rngx_status server_submit_ising(Server *s, uint32_t client, rngx_kind kind, uint32_t L, double beta, uint32_t sweeps,
                                uint64_t *ticket);
rngx_status server_wait(Server *s, uint64_t ticket, double timeout_s, rngx_request_result *res);
rngx_status server_wait_any(Server *s, double timeout_s, uint64_t *ticket, rngx_request_result *res);
rngx_status server_release(Server *s, uint64_t ticket);
rngx_status server_cancel(Server *s, uint64_t ticket);
int server_device(const Server *s);
size_t server_client_state_bytes(rngx_kind kind);
rngx_status server_get_client_state(Server *s, uint32_t client, rngx_kind kind, void *host_buf);
rngx_status server_set_client_state(Server *s, uint32_t client, rngx_kind kind, const void *host_buf);
void server_destroy(Server *s);

size_t state_bytes(rngx_kind kind, uint64_t S);
bool kind_valid(int kind);

// Thread-local error text; returns `st` for `return fail(...)`.
rngx_status fail(rngx_status st, const std::string &msg);
rngx_status hip_fail(hipError_t e, const char *what);
void clear_error();

// Launchers (stream-ordered, no host synchronisation).
hipError_t launch_seed(Gen *g, uint64_t seed, hipStream_t st);
hipError_t fill_setup(Gen *g, int n_cu);  // pacing counters, default configuration
int fill_configs(rngx_kind kind, const rngx_fill_config **list);  // autotuner candidates of a kind
int fill_default(rngx_kind kind);
hipError_t launch_fill(Gen *g, void *d_out, uint64_t count, int mode, hipStream_t st);
hipError_t launch_clear_ring(Gen *g, hipStream_t st);  // zero the pacing counters before a paced launch
hipError_t launch_skip(Gen *g, uint64_t n, hipStream_t st);
hipError_t launch_substreams(Gen *g, hipStream_t st);  // XS1024W: instance g skips g 2^137 steps (synchronous)
// MWC_DIFF: the first n multipliers (found on the device once per process)
// copied to device memory d_dst (may be NULL to only extend the list);
// synchronous on st.
hipError_t mwc_diff_multipliers(uint64_t n, uint32_t *d_dst, hipStream_t st);
bool mwc_diff_multipliers_match(const uint32_t *a, uint64_t n);  // a[0..n) = the first n multipliers
hipError_t launch_skip_mwc_diff(Gen *g, uint64_t n, hipStream_t st);
constexpr uint64_t kMwcDiffMaxStreams = 1ull << 21;
// Lagged Fibonacci kinds (lfg.hip): lags, seeding, fills, jump-ahead.
int lfg_lag_r(rngx_kind kind);
int lfg_lag_s(rngx_kind kind);
hipError_t launch_seed_lfg(Gen *g, uint64_t seed, hipStream_t st);
hipError_t launch_fill_lfg(Gen *g, void *out, uint64_t count, int mode, hipStream_t st);
hipError_t launch_skip_lfg(Gen *g, uint64_t n, hipStream_t st);  // synchronous

// Host-side jump tables for j = 0 .. count-1 steps of size `step`:
//  LCG32/LCG64: (A, C) pairs of the affine map f^(j step), 2 u64 each;
//  MWC: a^(j step) mod p, 1 u64 each;
//  XORWOW / XS1024W: x^(j step) mod P packed in 5 / 32 u32 each;
//  PHILOX: empty (the counter jumps by j step).
void jump_table(rngx_kind kind, uint64_t step, uint64_t count, std::vector<uint64_t> *u64s,
                std::vector<uint32_t> *u32s);
// As jump_table, for a handle (sub-stream LCG kinds use the handle's S-step map).
void jump_table_gen(const Gen *g, uint64_t step, uint64_t count, std::vector<uint64_t> *u64s,
                    std::vector<uint32_t> *u32s);
hipError_t launch_hot_start(Ising *lat, uint64_t seed, hipStream_t st);
hipError_t launch_ising(Ising *lat, double beta, uint64_t n_sweeps, int32_t *d_trace, hipStream_t st,
                        uint32_t hits = 1);  // hits: Metropolis updates per visited site
hipError_t launch_zero(uint32_t *p, uint64_t n, hipStream_t st);
bool ising_plan(uint32_t L, rngx_kind kind, int n_cu, IsingPlan *out);
int ising_plan_list(uint32_t L, rngx_kind kind, int n_cu, IsingPlan *out, int max);  // strip candidates
// Plans b (shape b->shape) from b->lats, b->betas, b->traces and `sweeps`
// (b->sweeps for real runs; scaled-down counts and no traces while tuning),
// replacing any earlier plan's device buffers.
hipError_t batch_prepare(IsingBatch *b, const uint64_t *sweeps, bool with_traces);
void batch_release(IsingBatch *b);  // the plan's device buffers
hipError_t launch_batch(IsingBatch *b, hipStream_t st);
// Work items of a ragged fill.  Small-state kinds: chunks of ragged_chunk
// outputs, one per lane.  XS1024W: the steps of all instances, concatenated,
// are cut into about equal slots, one per generating row (up to
// kXsRowsPerCu per compute unit); cuts inside an instance fall on multiples
// of *step.  *max_j is the largest chunk index (jump table size - 1).
struct RaggedPlan {
    std::vector<RaggedItem> items;
    std::vector<uint32_t> slots;  // XS1024W only
    uint64_t step = 1, max_j = 0;
};
constexpr uint32_t kXsRowsPerCu = 128;      // most rows per CU of any shape: 8 waves per SIMD x 4 SIMDs x 4 rows
constexpr uint64_t kXsMinSlotSteps = 2048;  // slots are not cut finer than this
// Shapes of a ragged plan, tuned per plan: XS1024W generating rows per CU,
// other kinds outputs per chunk.  Shape 0 is the default.
constexpr int kRaggedShapes = 3;
uint64_t ragged_shape_value(rngx_kind kind, int shape);
uint64_t ragged_chunk(rngx_kind kind, int shape = 0);
bool ragged_affine(rngx_kind kind);  // LCG32/LCG64 and sub-stream forms: one wave per chunk
bool ragged_wave(rngx_kind kind);    // affine kinds, MWC, MWC_DIFF, Philox: one wave per chunk, 1 KiB spans
bool ragged_lane_table(rngx_kind kind);  // kinds whose wave kernel takes lane_maps (ragged_lane_maps)
void ragged_plan(rngx_kind kind, const uint64_t *off, uint64_t n_units, int n_cu, RaggedPlan *plan, int shape = 0);
size_t ragged_scratch_bytes(rngx_kind kind, uint64_t n_items);
void ragged_lane_maps(const Gen *g, std::vector<uint64_t> *lane);  // affine kinds: lane start and advance maps
// The one-call ragged fill of rng_fill_ragged_u32_noalloc (noalloc.hip):
// plans on the host and stages the plan in the device's static scratch.
rngx_status ragged_fill_noalloc(Gen *g, const uint64_t *offsets, uint64_t units, uint32_t *d_out, hipStream_t st);
hipError_t launch_ragged(Ragged *r, uint32_t *d_out, hipStream_t st);
uint64_t stream_fill_chunk(rngx_kind kind);
hipError_t launch_stream_fill(rngx_kind kind, const uint8_t *st_in, uint8_t *st_out, uint64_t N, int f32,
                              const uint64_t *t64, const uint32_t *t32, void *out, hipStream_t st);
uint64_t ising_partials(uint32_t L);


}  // namespace rngx
