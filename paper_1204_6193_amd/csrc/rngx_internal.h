// Internal declarations of the rngx library: handles, status helpers and the
// device-side generator definitions shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "rngx.h"

namespace rngx {

// ---------------------------------------------------------------------------
// Constants of the generators (paper sections cited in rngx.h).
constexpr uint32_t kLcg32A = 1664525u;
constexpr uint32_t kLcg32C = 1013904223u;
constexpr uint64_t kLcg64A = 2862933555777941757ull;
constexpr uint64_t kLcg64C = 1442695040888963407ull;
constexpr uint64_t kMwcA = 4294967118ull;
constexpr uint64_t kMwcP = (kMwcA << 32) - 1;  // safe prime a*2^32 - 1
constexpr uint32_t kWeylC = 362437u;
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint64_t kSmGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSpinSeedXor = 0xD1B54A32D192ED03ull;

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
};
constexpr int kMaxFillConfigs = 8;

// Fill pacing (see k_fill_xs).
constexpr uint32_t kBand = 8;         // rows per band
constexpr uint32_t kSlack = 3;        // bands a workgroup may run ahead of the slowest
constexpr uint32_t kRing = 32;        // band entries in the counter ring
constexpr uint32_t kPaceSlots = 256;  // counters per entry (a multiple of 64)
constexpr uint32_t kPollLimit = 4096; // polls before a workgroup stops waiting

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
    Ising **lats;        // host copy of the members
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
hipError_t launch_skip(Gen *g, uint64_t n, hipStream_t st);

// Host-side jump tables for j = 0 .. count-1 steps of size `step`:
//  LCG32/LCG64: (A, C) pairs of the affine map f^(j step), 2 u64 each;
//  MWC: a^(j step) mod p, 1 u64 each;
//  XORWOW / XS1024W: x^(j step) mod P packed in 5 / 32 u32 each;
//  PHILOX: empty (the counter jumps by j step).
void jump_table(rngx_kind kind, uint64_t step, uint64_t count, std::vector<uint64_t> *u64s,
                std::vector<uint32_t> *u32s);
hipError_t launch_hot_start(Ising *lat, uint64_t seed, hipStream_t st);
hipError_t launch_ising(Ising *lat, double beta, uint64_t n_sweeps, int32_t *d_trace, hipStream_t st);
hipError_t launch_zero(uint32_t *p, uint64_t n, hipStream_t st);
bool ising_plan(uint32_t L, rngx_kind kind, int n_cu, IsingPlan *out);
int ising_plan_list(uint32_t L, rngx_kind kind, int n_cu, IsingPlan *out, int max);  // strip candidates
hipError_t batch_prepare(IsingBatch *b, Ising *const *lats, const double *betas, const uint64_t *n_sweeps,
                         int32_t *const *traces, int n_cu);
hipError_t launch_batch(IsingBatch *b, hipStream_t st);
uint64_t ragged_chunk(rngx_kind kind);
void ragged_plan(rngx_kind kind, const uint64_t *off, uint64_t n_units, std::vector<RaggedItem> *items,
                 uint64_t *max_chunks);
size_t ragged_scratch_bytes(rngx_kind kind, uint64_t n_items);
hipError_t launch_ragged(Ragged *r, uint32_t *d_out, hipStream_t st);
uint64_t stream_fill_chunk(rngx_kind kind);
hipError_t launch_stream_fill(rngx_kind kind, const uint8_t *st_in, uint8_t *st_out, uint64_t N, int f32,
                              const uint64_t *t64, const uint32_t *t32, void *out, hipStream_t st);
uint64_t ising_partials(uint32_t L);

enum { kOutU32 = 0, kOutF32 = 1, kOutXor = 2 };

// ---------------------------------------------------------------------------
// Device-side helpers.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t splitmix(uint64_t seed, uint64_t k) { return mix64(seed + k * kSmGamma); }

// One generator per stream, held in registers between load() and store().
// Each reads and writes its own arrays of the structure-of-arrays image.
struct Lcg32 {
    uint32_t x;
    __device__ void load(const uint8_t *st, uint64_t, uint64_t s) { x = reinterpret_cast<const uint32_t *>(st)[s]; }
    __device__ void store(uint8_t *st, uint64_t, uint64_t s) const { reinterpret_cast<uint32_t *>(st)[s] = x; }
    __device__ uint32_t next() { x = kLcg32A * x + kLcg32C; return x; }
};

struct Lcg64 {
    uint64_t x;
    __device__ void load(const uint8_t *st, uint64_t, uint64_t s) { x = reinterpret_cast<const uint64_t *>(st)[s]; }
    __device__ void store(uint8_t *st, uint64_t, uint64_t s) const { reinterpret_cast<uint64_t *>(st)[s] = x; }
    __device__ uint32_t next() { x = kLcg64A * x + kLcg64C; return static_cast<uint32_t>(x >> 32); }
};

struct Mwc {
    uint64_t y;  // carry << 32 | x
    __device__ void load(const uint8_t *st, uint64_t, uint64_t s) { y = reinterpret_cast<const uint64_t *>(st)[s]; }
    __device__ void store(uint8_t *st, uint64_t, uint64_t s) const { reinterpret_cast<uint64_t *>(st)[s] = y; }
    __device__ uint32_t next() {
        y = kMwcA * static_cast<uint32_t>(y) + (y >> 32);  // one 32x32+32 -> 64 multiply-add
        return static_cast<uint32_t>(y);
    }
};

struct Xorwow {
    uint32_t x, y, z, w, v, d;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t s) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        x = p[s]; y = p[S + s]; z = p[2 * S + s]; w = p[3 * S + s]; v = p[4 * S + s]; d = p[5 * S + s];
    }
    __device__ void store(uint8_t *st, uint64_t S, uint64_t s) const {
        uint32_t *p = reinterpret_cast<uint32_t *>(st);
        p[s] = x; p[S + s] = y; p[2 * S + s] = z; p[3 * S + s] = w; p[4 * S + s] = v; p[5 * S + s] = d;
    }
    __device__ uint32_t next() {
        uint32_t t = x ^ (x >> 2);
        x = y; y = z; z = w; w = v;
        v = (v ^ (v << 4)) ^ (t ^ (t << 1));
        d += kWeylC;
        return d + v;
    }
};

// Philox4x32-10 block function on counter (lo, hi, 0, 0) with key (k0, k1).
__device__ inline void philox_block(uint32_t k0, uint32_t k1, uint64_t blk, uint32_t &o0, uint32_t &o1,
                                    uint32_t &o2, uint32_t &o3) {
    uint32_t x0 = static_cast<uint32_t>(blk), x1 = static_cast<uint32_t>(blk >> 32), x2 = 0, x3 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * x0;
        const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * x2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ x1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ x3 ^ k1;
        x1 = static_cast<uint32_t>(p1);
        x3 = static_cast<uint32_t>(p0);
        x0 = n0; x2 = n2;
        k0 += kPhiloxW0; k1 += kPhiloxW1;
    }
    o0 = x0; o1 = x1; o2 = x2; o3 = x3;
}

struct Philox {
    uint32_t k0, k1, b0, b1, b2, b3;
    uint64_t pos;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t s) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        k0 = p[s]; k1 = p[S + s];
        pos = reinterpret_cast<const uint64_t *>(st + 8 * S)[s];
        if (pos & 3) philox_block(k0, k1, pos >> 2, b0, b1, b2, b3);  // resume mid-block
    }
    __device__ void store(uint8_t *st, uint64_t S, uint64_t s) const {
        reinterpret_cast<uint64_t *>(st + 8 * S)[s] = pos;
    }
    __device__ uint32_t next() {
        const uint32_t j = static_cast<uint32_t>(pos) & 3;
        if (j == 0) philox_block(k0, k1, pos >> 2, b0, b1, b2, b3);
        ++pos;
        return j == 0 ? b0 : j == 1 ? b1 : j == 2 ? b2 : b3;
    }
};

// ---------------------------------------------------------------------------
// XORShift-1024 on wave64: one 1024-bit instance per 16-lane DPP row, two
// 32-bit words per lane (lane j holds words 2j and 2j+1, word 0 most
// significant).  A word shift by 10 is then a lane shift by 5 inside the row,
// and DPP row shifts read zero from outside the row, which is exactly the
// zero fill of a shift of a 1024-bit number (bound_ctrl set: a source lane
// outside the row reads as 0).
template <int N>
__device__ __forceinline__ uint32_t from_lane_plus(uint32_t v) {  // lane j <- lane j+N of its row
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x100 + N, 0xF, 0xF, true));
}
template <int N>
__device__ __forceinline__ uint32_t from_lane_minus(uint32_t v) {  // lane j <- lane j-N of its row
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x110 + N, 0xF, 0xF, true));
}
// (hi << (32 - s)) | (lo >> s)
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// X ^= X << 329; X ^= X >> 347; X ^= X << 344  on the row-distributed state.
__device__ __forceinline__ void xs1024_step(uint32_t &a, uint32_t &b) {
    // << 329 = 10 words + 9 bits: W[i] ^= W[i+10] << 9 | W[i+11] >> 23
    uint32_t p5a = from_lane_plus<5>(a), p5b = from_lane_plus<5>(b), p6a = from_lane_plus<6>(a);
    a ^= funnel(p5a, p5b, 23);
    b ^= funnel(p5b, p6a, 23);
    // >> 347 = 10 words + 27 bits: W[i] ^= W[i-11] << 5 | W[i-10] >> 27
    uint32_t m6b = from_lane_minus<6>(b), m5a = from_lane_minus<5>(a), m5b = from_lane_minus<5>(b);
    a ^= funnel(m6b, m5a, 27);
    b ^= funnel(m5a, m5b, 27);
    // << 344 = 10 words + 24 bits: W[i] ^= W[i+10] << 24 | W[i+11] >> 8
    p5a = from_lane_plus<5>(a); p5b = from_lane_plus<5>(b); p6a = from_lane_plus<6>(a);
    a ^= funnel(p5a, p5b, 8);
    b ^= funnel(p5b, p6a, 8);
}

// Weyl output term y (I + R^16) with y = y0 + n c.
__device__ __forceinline__ uint32_t weyl_mix(uint32_t y) { return y ^ (y >> 16); }

// J(M) v for the XS1024W transition matrix M and J(x) = sum c_i x^i
// (coefficient i at bit i%32 of c[i/32], degree < 1024), by Horner's rule:
// 1024 generator steps.  (a, b) is the calling lane's word pair of v.
__device__ __forceinline__ void xs1024_apply_poly(const uint32_t *c, uint32_t &a, uint32_t &b) {
    const uint32_t va = a, vb = b;
    a = 0;
    b = 0;
    for (int i = 1023; i >= 0; --i) {
        xs1024_step(a, b);
        if ((c[i >> 5] >> (i & 31)) & 1u) { a ^= va; b ^= vb; }
    }
}

// Same for XORWOW's 160-bit xorshift part (x, y, z, w, v) = s[0..4].
__device__ __forceinline__ void xorwow_apply_poly(const uint32_t *c, uint32_t (&s)[5]) {
    uint32_t acc[5] = {0, 0, 0, 0, 0};
    for (int i = 159; i >= 0; --i) {
        const uint32_t t = acc[0] ^ (acc[0] >> 2);
        acc[0] = acc[1]; acc[1] = acc[2]; acc[2] = acc[3]; acc[3] = acc[4];
        acc[4] = (acc[4] ^ (acc[4] << 4)) ^ (t ^ (t << 1));
        if ((c[i >> 5] >> (i & 31)) & 1u)
            for (int q = 0; q < 5; ++q) acc[q] ^= s[q];
    }
    for (int q = 0; q < 5; ++q) s[q] = acc[q];
}

// Jumps by j*C outputs with tables made by jump_table(kind, C, ...):
// t64 = affine pairs (LCG) or a^(jC) mod p (MWC), t32 = x^(jC) mod P
// polynomials (XORWOW).  Philox needs none.
__device__ __forceinline__ uint64_t mwc_mulmod(uint64_t y, uint64_t A);
__device__ __forceinline__ void jump(Lcg32 &g, const uint64_t *t64, const uint32_t *, uint64_t j, uint64_t) {
    g.x = static_cast<uint32_t>(t64[2 * j]) * g.x + static_cast<uint32_t>(t64[2 * j + 1]);
}
__device__ __forceinline__ void jump(Lcg64 &g, const uint64_t *t64, const uint32_t *, uint64_t j, uint64_t) {
    g.x = t64[2 * j] * g.x + t64[2 * j + 1];
}
__device__ __forceinline__ void jump(Mwc &g, const uint64_t *t64, const uint32_t *, uint64_t j, uint64_t) {
    g.y = mwc_mulmod(g.y, t64[j]);
}
__device__ __forceinline__ void jump(Xorwow &g, const uint64_t *, const uint32_t *t32, uint64_t j, uint64_t C) {
    if (!j) return;
    uint32_t s[5] = {g.x, g.y, g.z, g.w, g.v};
    xorwow_apply_poly(t32 + 5 * j, s);
    g.x = s[0]; g.y = s[1]; g.z = s[2]; g.w = s[3]; g.v = s[4];
    g.d += static_cast<uint32_t>(j * C) * kWeylC;
}
__device__ __forceinline__ void jump(Philox &g, const uint64_t *, const uint32_t *, uint64_t j, uint64_t C) {
    g.pos += j * C;
    if (g.pos & 3) philox_block(g.k0, g.k1, g.pos >> 2, g.b0, g.b1, g.b2, g.b3);  // resume mid-block
}

// y * A mod p for the MWC modulus p = a 2^32 - 1, using 2^64 = R (mod p)
// with R = 2^64 - p < 2^41.
__device__ __forceinline__ uint64_t mwc_mulmod(uint64_t y, uint64_t A) {
    constexpr uint64_t R = 0ull - kMwcP;
    uint64_t lo = y * A, hi = __umul64hi(y, A);
    while (hi) {  // (hi, lo) <- hi * R + lo; hi shrinks by >= 23 bits a round
        const uint64_t plo = hi * R, phi = __umul64hi(hi, R);
        const uint64_t sum = plo + lo;
        hi = phi + (sum < plo ? 1 : 0);
        lo = sum;
    }
    return lo >= kMwcP ? lo - kMwcP : lo;
}

}  // namespace rngx
