// Uneven ("ragged") fills: every stream receives a request of its own length
// in one launch pair, however long or short the requests are.
//
// Stream s (small-state kinds) writes its next len_s outputs to
// out[off_s .. off_s + len_s); XS1024W instance g writes len_g values in warp
// order (step k, lane i -> out[off_g + 32 k + i]), taking ceil(len_g / 32)
// steps and dropping the lanes of a last partial step.
//
// A request is cut into chunks so that long requests spread over many
// threads.  The first kernel puts the start state of every chunk j into
// scratch by jumping the stream's state by j*C (precomputed powers of the
// C-step map: affine pairs, a^(jC) mod p, or GF(2) polynomials x^(jC) mod P
// applied by Horner's rule); the second kernel generates every chunk from its
// start state, and the last chunk of a stream writes the stream's final state
// back.  Small-state kinds take one chunk of C outputs per lane.  XS1024W
// balances rows instead: the instances' steps, concatenated, are cut into
// about equal slots (cuts inside an instance on multiples of C), and one
// 16-lane row generates all chunks of its slot in turn, so no row waits on a
// longer one and the only jumps are those at the cuts.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kBlock = 256;

// Each lane owns one chunk.  Rounds of 32 outputs go through a per-wave LDS
// tile so that the wave writes two lanes' segments with one store.  Rounds
// are aligned to 32-word (128-byte) lines of the output: round r of a chunk
// covers the line-aligned window [base + 32 r, base + 32 r + 32) and only the
// chunk's first and last windows are partial, so every cache line but those
// at chunk ends is written whole by one store.  Each lane puts the window's
// address and its column range [lo, hi) in LDS for the store loop.
constexpr int kSeg = 32;

template <class G>
__global__ __launch_bounds__(kBlock) void k_ragged_gen_small(const RaggedItem *items, uint64_t n_items,
                                                              const uint8_t *scratch, uint8_t *st, uint64_t S,
                                                              uint32_t *out) {
    __shared__ uint32_t tile[kBlock / 64][64][kSeg + 1];
    __shared__ uint64_t desc[kBlock / 64][64][2];  // window address; lo | hi << 32
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    const bool mine = i < n_items;
    RaggedItem it{};
    G g;
    if (mine) {
        it = items[i];
        g.load(scratch, n_items, i);
    }
    const uint32_t len = mine ? it.len : 0;
    const uint32_t mis = static_cast<uint32_t>(it.out) & (kSeg - 1);
    const uint64_t base = it.out - mis;
    uint32_t rounds = len ? (mis + len + kSeg - 1) / kSeg : 0;  // rounds needed by the longest chunk of the wave
    for (int off = 32; off > 0; off >>= 1) rounds = max(rounds, static_cast<uint32_t>(__shfl_xor(static_cast<int>(rounds), off)));
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const int64_t rem = static_cast<int64_t>(mis) + len - static_cast<int64_t>(rd) * kSeg;
        const uint32_t lo = rd == 0 ? mis : 0;
        const uint32_t hi = rem <= 0 ? 0 : static_cast<uint32_t>(min(rem, static_cast<int64_t>(kSeg)));
        if (lo == 0 && hi == kSeg) {
#pragma unroll
            for (int c = 0; c < kSeg; ++c) tile[w][lane][c] = g.next();
        } else {
            for (uint32_t c = lo; c < hi; ++c) tile[w][lane][c] = g.next();
        }
        const uint64_t a = base + static_cast<uint64_t>(rd) * kSeg;
        desc[w][lane][0] = a;
        desc[w][lane][1] = lo | static_cast<uint64_t>(hi) << 32;
        __builtin_amdgcn_wave_barrier();
        // lanes 0-31 write lane j's window, lanes 32-63 lane j+1's.  When
        // every window of the wave is whole (all rounds but a chunk's first
        // and last) the stores need no test.
        if (__all((lo == 0) & (hi == kSeg))) {
#pragma unroll 8
            for (uint32_t j = 0; j < 64; j += 2) {
                const uint32_t src = j + half;
                out[desc[w][src][0] + col] = tile[w][src][col];
            }
        } else {
#pragma unroll 4
            for (uint32_t j = 0; j < 64; j += 2) {
                const uint32_t src = j + half;
                const uint64_t dr = desc[w][src][1];
                if ((col >= static_cast<uint32_t>(dr)) & (col < static_cast<uint32_t>(dr >> 32)))
                    out[desc[w][src][0] + col] = tile[w][src][col];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (mine && it.last) g.store(st, S, it.unit);
}

// Affine kinds (LCG32, LCG64 and their sub-stream forms): one wave per
// chunk, leapfrogging four values per lane.  The wave's stores are aligned
// to 256-word (1 KiB) spans of the output: in step k lane i writes words
// A + 256 k + 4 i + j (j = 0..3), A being the chunk's first word rounded down
// to a multiple of 256, i.e. chunk positions b + j with b = 256 k + 4 i - mis
// (mis = first word - A).  A lane keeps the state of position b (the
// (b+1)-step map from the chunk's start state, lane_maps[b] for its first
// step with b >= 0), derives b+1..b+3 by single steps and advances 256 steps
// per store (lane_maps[256]).  Whole spans before the chunk's last one are
// written as one 16-byte non-temporal store per lane with no checks; the
// first and last spans word by word.  The streams' states are only read
// here; the lane that writes a stream's last value puts the final state in
// scratch[item] for k_ragged_commit_affine.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kAffSpan = 256;  // words per wave store (64 lanes x 4)
template <bool L64>
__global__ __launch_bounds__(kBlock) void k_ragged_affine(const RaggedItem *items, uint64_t n_items,
                                                           const uint64_t *t64, const uint64_t *lane_maps,
                                                           const uint8_t *st, uint64_t *scratch, uint32_t *out) {
    const uint64_t q = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    if (q >= n_items) return;  // whole waves
    const RaggedItem it = items[q];
    const uint64_t x0 = L64 ? reinterpret_cast<const uint64_t *>(st)[it.unit]
                            : reinterpret_cast<const uint32_t *>(st)[it.unit];
    const uint64_t xc = t64[2 * it.j] * x0 + t64[2 * it.j + 1];  // state at the chunk's start
    const uint32_t mis = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(out) >> 2) + it.out) & (kAffSpan - 1);
    using T = std::conditional_t<L64, uint64_t, uint32_t>;  // 32-bit kinds: arithmetic mod 2^32
    // first position of the lane in a step with b >= 0 (step 0 if 4 lane >= mis, else step 1)
    const uint32_t pf = 4 * lane >= mis ? 4 * lane - mis : kAffSpan + 4 * lane - mis;
    T x = static_cast<T>(lane_maps[2 * pf] * xc + lane_maps[2 * pf + 1]);
    const T s0 = static_cast<T>(lane_maps[0] * xc + lane_maps[1]);  // state of position 0
    const T a1 = static_cast<T>(lane_maps[0]), c1 = static_cast<T>(lane_maps[1]);  // the one-step map
    const T Am = static_cast<T>(lane_maps[2 * kAffSpan]), Cm = static_cast<T>(lane_maps[2 * kAffSpan + 1]);
    const int64_t len = it.len;
    const uint32_t kend = static_cast<uint32_t>((len + mis + kAffSpan - 1) / kAffSpan);
    // Spans k in [kb, kw) are whole (256 k >= mis and 256 k + 256 - mis <= len);
    // the body loop takes them up to, not including, the last span, which
    // holds the stream's last value and goes through the checked loop.
    const uint32_t kb = mis ? 1u : 0u;
    const uint32_t kw = static_cast<uint32_t>((len + mis) / kAffSpan);
    const uint32_t kl = kend ? (kw < kend - 1 ? kw : kend - 1) : 0u;
    const uint32_t body_end = kl > kb ? kl : kb;
    auto word = [](T v) { return L64 ? static_cast<uint32_t>(v >> 32) : static_cast<uint32_t>(v); };
    uint32_t *o = out + (it.out - mis) + 4 * lane;
    auto checked = [&](uint32_t k) {
        const int64_t b = static_cast<int64_t>(kAffSpan) * k + 4 * lane - mis;
        T y = b >= 0 ? x : s0;  // state of the lane's first position >= 0
        for (int j = 0; j < 4; ++j) {
            const int64_t p = b + j;
            if (p < 0) continue;
            if (p < len) o[j] = word(y);
            if (it.last && p == len - 1) scratch[q] = y;
            y = a1 * y + c1;
        }
        if (b >= 0) x = Am * x + Cm;
        o += kAffSpan;
    };
    uint32_t k = 0;
    for (; k < kb && k < kend; ++k) checked(k);
    for (; k < body_end; ++k) {
        const T y1 = a1 * x + c1, y2 = a1 * y1 + c1, y3 = a1 * y2 + c1;
        const u32x4 v = {word(x), word(y1), word(y2), word(y3)};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(o));
        x = Am * x + Cm;
        o += kAffSpan;
    }
    for (; k < kend; ++k) checked(k);
}

// MWC and MWC_DIFF the same way: the MWC is y -> a y mod p (y = carry 2^32 +
// x, p = a 2^32 - 1), so a lane's first state is a^(pf+1) times the chunk's
// start state, the next three come by plain MWC steps and a store advances
// the lane by a^256.  MWC: the powers of its one a are in lane_maps (a^(i+1)
// mod p, i < 256, then a^256) and the chunk starts in t64 (a^(j C));
// MWC_DIFF: each chunk computes its stream's powers with Montgomery
// arithmetic (a product by a power kept in Montgomery form returns a plain
// residue).
template <bool DIFF>
__global__ __launch_bounds__(kBlock) void k_ragged_mwc(const RaggedItem *items, uint64_t n_items, const uint64_t *t64,
                                                        const uint64_t *lane_maps, const uint8_t *st, uint64_t S,
                                                        uint64_t chunk, uint64_t *scratch, uint32_t *out) {
    const uint64_t q = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    if (q >= n_items) return;  // whole waves
    const RaggedItem it = items[q];
    const uint64_t y0 = reinterpret_cast<const uint64_t *>(st)[it.unit];
    const uint32_t a = DIFF ? reinterpret_cast<const uint32_t *>(st + 8 * S)[it.unit] : static_cast<uint32_t>(kMwcA);
    const uint32_t mis = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(out) >> 2) + it.out) & (kAffSpan - 1);
    const uint32_t pf = 4 * lane >= mis ? 4 * lane - mis : kAffSpan + 4 * lane - mis;
    uint64_t yc, x, a_span_m = 0;
    const Mont64 M(DIFF ? (static_cast<uint64_t>(a) << 32) - 1 : 3);  // (unused for MWC)
    if constexpr (DIFF) {
        yc = it.j ? mwc_jump_mod(y0, a, it.j * chunk) : y0;
        const uint64_t am = M.to(a);
        x = M.mul(yc, M.pow(am, pf + 1));
        a_span_m = M.pow(am, kAffSpan);
    } else {
        yc = mwc_mulmod(y0, t64[it.j]);
        x = mwc_mulmod(yc, lane_maps[pf]);
    }
    auto step = [=](uint64_t y) { return static_cast<uint64_t>(a) * static_cast<uint32_t>(y) + (y >> 32); };
    auto advance = [&](uint64_t y) { return DIFF ? M.mul(y, a_span_m) : mwc_mulmod(y, lane_maps[kAffSpan]); };
    const uint64_t s0 = step(yc);  // state of position 0
    const int64_t len = it.len;
    const uint32_t kend = static_cast<uint32_t>((len + mis + kAffSpan - 1) / kAffSpan);
    const uint32_t kb = mis ? 1u : 0u;
    const uint32_t kw = static_cast<uint32_t>((len + mis) / kAffSpan);
    const uint32_t kl = kend ? (kw < kend - 1 ? kw : kend - 1) : 0u;
    const uint32_t body_end = kl > kb ? kl : kb;
    uint32_t *o = out + (it.out - mis) + 4 * lane;
    auto checked = [&](uint32_t k) {
        const int64_t b = static_cast<int64_t>(kAffSpan) * k + 4 * lane - mis;
        uint64_t y = b >= 0 ? x : s0;
        for (int j = 0; j < 4; ++j) {
            const int64_t p = b + j;
            if (p < 0) continue;
            if (p < len) o[j] = static_cast<uint32_t>(y);
            if (it.last && p == len - 1) scratch[q] = y;
            y = step(y);
        }
        if (b >= 0) x = advance(x);
        o += kAffSpan;
    };
    uint32_t k = 0;
    for (; k < kb && k < kend; ++k) checked(k);
    for (; k < body_end; ++k) {
        const uint64_t y1 = step(x), y2 = step(y1), y3 = step(y2);
        const u32x4 v = {static_cast<uint32_t>(x), static_cast<uint32_t>(y1), static_cast<uint32_t>(y2),
                         static_cast<uint32_t>(y3)};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(o));
        x = advance(x);
        o += kAffSpan;
    }
    for (; k < kend; ++k) checked(k);
}

// Philox, counter-based, in the same span layout: lane i of step k makes
// the block holding positions P + 256 k + 4 i - mis .. +3 (P: the chunk's
// first stream position); when those are not block-aligned (d = (P - mis)
// mod 4 != 0) a slot's value comes from the lane's own block or, for its
// last d slots, from the next lane's (lane 63: lane 0's block of the next
// step, made one step ahead).  One block per lane per store.
__device__ __forceinline__ uint32_t pick4(const uint32_t (&v)[4], uint32_t i) {
    return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
}
template <int ROUNDS>
__global__ __launch_bounds__(kBlock) void k_ragged_philox(const RaggedItem *items, uint64_t n_items, const uint8_t *st,
                                                           uint64_t S, uint64_t chunk, uint64_t *scratch,
                                                           uint32_t *out) {
    const uint64_t q = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    if (q >= n_items) return;  // whole waves
    const RaggedItem it = items[q];
    const uint32_t *key = reinterpret_cast<const uint32_t *>(st);
    const uint32_t k0 = key[it.unit], k1 = key[S + it.unit];
    const uint64_t P = reinterpret_cast<const uint64_t *>(st + 8 * S)[it.unit] + it.j * chunk;
    const uint32_t mis = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(out) >> 2) + it.out) & (kAffSpan - 1);
    const uint64_t base = P - mis + 4 * lane;  // stream position of the lane's slot 0 in step 0 (mod 2^64)
    const uint32_t d = static_cast<uint32_t>(P - mis) & 3;
    const int64_t len = it.len;
    const uint32_t kend = static_cast<uint32_t>((len + mis + kAffSpan - 1) / kAffSpan);
    const uint32_t kb = mis ? 1u : 0u;
    const uint32_t kw = static_cast<uint32_t>((len + mis) / kAffSpan);
    const uint32_t kl = kend ? (kw < kend - 1 ? kw : kend - 1) : 0u;
    const uint32_t body_end = kl > kb ? kl : kb;
    uint32_t *o = out + (it.out - mis) + 4 * lane;
    uint32_t cur[4], nxt[4];
    philox_block<ROUNDS>(k0, k1, base >> 2, cur[0], cur[1], cur[2], cur[3]);
    // the four slot values of this step; every lane takes part (shuffles)
    auto values = [&](uint32_t k, uint32_t (&v)[4]) {
        philox_block<ROUNDS>(k0, k1, (base + kAffSpan * (static_cast<uint64_t>(k) + 1)) >> 2, nxt[0], nxt[1], nxt[2],
                             nxt[3]);
        uint32_t nb[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t down = static_cast<uint32_t>(__shfl_down(static_cast<int>(cur[w]), 1));
            const uint32_t first = static_cast<uint32_t>(__shfl(static_cast<int>(nxt[w]), 0));
            nb[w] = lane == 63 ? first : down;
        }
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) v[j] = d + j < 4 ? pick4(cur, d + j) : pick4(nb, d + j - 4);
#pragma unroll
        for (int w = 0; w < 4; ++w) cur[w] = nxt[w];
    };
    auto checked = [&](uint32_t k) {
        uint32_t v[4];
        values(k, v);
        const int64_t b = static_cast<int64_t>(kAffSpan) * k + 4 * lane - mis;
        for (int j = 0; j < 4; ++j) {
            const int64_t p = b + j;
            if (p < 0) continue;
            if (p < len) o[j] = v[j];
            if (it.last && p == len - 1) scratch[q] = P + static_cast<uint64_t>(len);
        }
        o += kAffSpan;
    };
    uint32_t k = 0;
    for (; k < kb && k < kend; ++k) checked(k);
    for (; k < body_end; ++k) {
        uint32_t v[4];
        values(k, v);
        const u32x4 w = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(o));
        o += kAffSpan;
    }
    for (; k < kend; ++k) checked(k);
}

// The final 64-bit state word of each stream (MWC: y; Philox: position) from
// scratch into the image's array `dst`.
__global__ __launch_bounds__(kBlock) void k_ragged_commit_u64(const RaggedItem *items, uint64_t n_items,
                                                               const uint64_t *scratch, uint64_t *dst) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_items || !items[i].last) return;
    dst[items[i].unit] = scratch[i];
}

template <bool L64>
__global__ __launch_bounds__(kBlock) void k_ragged_commit_affine(const RaggedItem *items, uint64_t n_items,
                                                                  const uint64_t *scratch, uint8_t *st) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_items || !items[i].last) return;
    if (L64) reinterpret_cast<uint64_t *>(st)[items[i].unit] = scratch[i];
    else reinterpret_cast<uint32_t *>(st)[items[i].unit] = static_cast<uint32_t>(scratch[i]);
}

// Start states of the chunks of the small-state kinds, written to scratch in
// the kind's structure-of-arrays layout with n_items streams.
__global__ __launch_bounds__(kBlock) void k_ragged_start_small(rngx_kind kind, const RaggedItem *items,
                                                                uint64_t n_items, const uint8_t *st, uint64_t S,
                                                                uint8_t *scratch, const uint64_t *t64,
                                                                const uint32_t *t32, uint64_t chunk) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const RaggedItem it = items[i];
    const uint64_t s = it.unit, j = it.j;
    switch (kind) {
    case RNGX_LCG32_SUB:  // the S-step map goes after the chunk states, as in the image
        if (i == 0) {
            const uint32_t *h = reinterpret_cast<const uint32_t *>(st) + S;
            reinterpret_cast<uint32_t *>(scratch)[n_items] = h[0];
            reinterpret_cast<uint32_t *>(scratch)[n_items + 1] = h[1];
        }
        [[fallthrough]];
    case RNGX_LCG32: {
        const uint32_t x = reinterpret_cast<const uint32_t *>(st)[s];
        reinterpret_cast<uint32_t *>(scratch)[i] =
            static_cast<uint32_t>(t64[2 * j]) * x + static_cast<uint32_t>(t64[2 * j + 1]);
        break;
    }
    case RNGX_LCG64_SUB:
        if (i == 0) {
            const uint64_t *h = reinterpret_cast<const uint64_t *>(st) + S;
            reinterpret_cast<uint64_t *>(scratch)[n_items] = h[0];
            reinterpret_cast<uint64_t *>(scratch)[n_items + 1] = h[1];
        }
        [[fallthrough]];
    case RNGX_LCG64: {
        const uint64_t x = reinterpret_cast<const uint64_t *>(st)[s];
        reinterpret_cast<uint64_t *>(scratch)[i] = t64[2 * j] * x + t64[2 * j + 1];
        break;
    }
    case RNGX_MWC: {
        const uint64_t y = reinterpret_cast<const uint64_t *>(st)[s];
        reinterpret_cast<uint64_t *>(scratch)[i] = mwc_mulmod(y, t64[j]);
        break;
    }
    case RNGX_MWC_DIFF: {  // the stream's own a^(jC) mod p, then its multiplier
        const uint64_t y = reinterpret_cast<const uint64_t *>(st)[s];
        const uint32_t a = reinterpret_cast<const uint32_t *>(st + 8 * S)[s];
        reinterpret_cast<uint64_t *>(scratch)[i] = j ? mwc_jump_mod(y, a, j * chunk) : y;
        reinterpret_cast<uint32_t *>(scratch + 8 * n_items)[i] = a;
        break;
    }
    case RNGX_XORWOW: {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        uint32_t v[5];
        for (int q = 0; q < 5; ++q) v[q] = p[q * S + s];
        if (j) xorwow_apply_poly(t32 + 5 * j, v);
        uint32_t *o = reinterpret_cast<uint32_t *>(scratch);
        for (int q = 0; q < 5; ++q) o[q * n_items + i] = v[q];
        o[5 * n_items + i] = p[5 * S + s] + static_cast<uint32_t>(j * chunk) * kWeylC;
        break;
    }
    case RNGX_PHILOX4X32_7:
    case RNGX_PHILOX4X32_10: {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        uint32_t *o = reinterpret_cast<uint32_t *>(scratch);
        o[i] = p[s];
        o[n_items + i] = p[S + s];
        reinterpret_cast<uint64_t *>(scratch + 8 * n_items)[i] =
            reinterpret_cast<const uint64_t *>(st + 8 * S)[s] + j * chunk;
        break;
    }
    default: break;
    }
}

// XS1024W: one 16-lane row per slot.  The row runs its slot's chunks
// (items slots[r] .. slots[r+1]-1) in turn: it takes the instance's state,
// jumps it by j*C if the chunk starts inside the instance (only a slot's
// first chunk can), and generates the chunk.  The states are only read here;
// after an instance's last chunk the row puts the final state in scratch
// (per item: 16 lane pairs, then the step counters at 128 * n_items) and a
// second kernel copies it back, so no row can read a state another row has
// already advanced.
//
// Stores are aligned to 32-word (128-byte) output lines: step k's 32 words
// go into a 64-word LDS ring and lane i writes the word pair at positions
// 2i, 2i+1 of line k of the chunk's aligned span, which holds the last `mis`
// words of step k-1 and the first 32-mis of step k (mis: the chunk's start
// modulo 32 words).  Inside a chunk every store is one whole line per row;
// only the first and last lines of a chunk are partial.
__global__ __launch_bounds__(kBlock) void k_ragged_xs(const RaggedItem *items, uint64_t n_items,
                                                       const uint32_t *slots, uint32_t n_slots, const uint8_t *st,
                                                       uint64_t S, const uint32_t *t32, uint64_t chunk,
                                                       uint8_t *scratch, uint32_t *out) {
    // 64-word ring per row, kept twice (word p at p and p + 64) so that a
    // lane's pair never wraps
    __shared__ uint32_t ring[kBlock / 16][128];
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t r = t >> 4;
    const uint32_t lane = static_cast<uint32_t>(t & 15), rl = threadIdx.x >> 4;
    if (r >= n_slots) return;  // whole rows
    const uint32_t q_end = slots[r + 1];
    const uint32_t y0 = *reinterpret_cast<const uint32_t *>(st + 4 * S + 8 * (S / 32));
    const uint64_t out_word = reinterpret_cast<uintptr_t>(out) >> 2;  // out is 4-byte aligned
    uint32_t *rg = ring[rl];
    // The row's chunks run in one flat loop (not a loop per chunk): the rows
    // of a wave switch chunks at different steps, and with a loop per chunk
    // the wave would run every chunk index as long as its longest row.
    uint32_t q = slots[r];
    RaggedItem it;
    uint32_t a, b, y, mis, len, kf, k;
    // ring positions of the lane's pair: written (step k's words 2 lane, 2
    // lane + 1 at 32 k mod 64) and read (line k at 32 k + 2 lane - mis mod 64),
    // for the current parity of k; xor with *_flip moves to the other parity
    uint32_t wcur, rcur, wflip, rflip;
    uint64_t n;
    int64_t nvals;
    uint32_t *o;
    auto begin = [&]() {  // load chunk q
        it = items[q];
        const uint2 w = reinterpret_cast<const uint2 *>(st)[16 * it.unit + lane];
        a = w.x;
        b = w.y;
        n = reinterpret_cast<const uint64_t *>(st + 4 * S)[it.unit];
        if (it.j) {
            xs1024_apply_poly(t32 + 32 * it.j, a, b);
            n += it.j * chunk;
        }
        y = y0 + static_cast<uint32_t>(n) * kWeylC;
        mis = static_cast<uint32_t>(out_word + it.out) & 31;
        o = out + (it.out - mis) + 2 * lane;  // lane's pair in line 0 (positions < mis unused)
        len = it.len;
        nvals = static_cast<int64_t>(it.nvals);
        // lines 1 .. kf are whole: 32 k - mis >= 0 and 32 k + 32 - mis <= nvals
        const int64_t kf_ = (nvals + mis - 32) / 32;
        kf = kf_ <= 0 ? 0 : static_cast<uint32_t>(min(kf_, static_cast<int64_t>(len) - 1));
        k = 0;
        wcur = 2 * lane;
        wflip = 32;
        rcur = (2 * lane - mis) & 63;
        rflip = rcur ^ ((32 + 2 * lane - mis) & 63);
        // Loads complete here: stores share the memory counter, so a wait
        // left to the step loop would also wait for the stores.
        __builtin_amdgcn_s_waitcnt(0x0F70);
    };
    begin();
    while (true) {
        if (k == len) {
            {  // line len: the last mis words of step len-1
                const uint32_t f0 = rg[rcur], f1 = rg[rcur + 1];
                __builtin_amdgcn_wave_barrier();
                const int64_t v0 = 32 * static_cast<int64_t>(len) + 2 * lane - mis;
                if (v0 < nvals) o[0] = f0;
                if (v0 + 1 < nvals) o[1] = f1;
            }
            if (it.last) {
                reinterpret_cast<uint2 *>(scratch)[16ull * q + lane] = make_uint2(a, b);
                if (lane == 0) reinterpret_cast<uint64_t *>(scratch + 128 * n_items)[q] = n + len;
            }
            if (++q == q_end) break;
            begin();
        }
        if (k >= 1 && k + 3 <= kf) {  // lines k .. k+3 whole: four steps with no tests
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xs1024_step(a, b);
                y += kWeylC;
                const uint32_t m = weyl_mix(y);
                const uint2 pv = make_uint2(a + m, b + m);
                *reinterpret_cast<uint2 *>(rg + wcur) = pv;
                *reinterpret_cast<uint2 *>(rg + wcur + 64) = pv;
                __builtin_amdgcn_wave_barrier();
                const uint32_t w0 = rg[rcur], w1 = rg[rcur + 1];
                __builtin_amdgcn_wave_barrier();
                wcur ^= wflip;
                rcur ^= rflip;
                __builtin_nontemporal_store(w0 | static_cast<uint64_t>(w1) << 32, reinterpret_cast<uint64_t *>(o + 32 * j));
            }
            o += 128;
            k += 4;
            continue;  // k <= kf + 1 <= len: the chunk may end here
        }
        // step k into the ring, then the lane's pair of line k
        xs1024_step(a, b);
        y += kWeylC;
        const uint32_t m = weyl_mix(y);
        const uint2 pv = make_uint2(a + m, b + m);
        *reinterpret_cast<uint2 *>(rg + wcur) = pv;
        *reinterpret_cast<uint2 *>(rg + wcur + 64) = pv;
        __builtin_amdgcn_wave_barrier();
        const uint32_t w0 = rg[rcur], w1 = rg[rcur + 1];
        __builtin_amdgcn_wave_barrier();
        wcur ^= wflip;
        rcur ^= rflip;
        if (k - 1 < kf) {  // 1 <= k <= kf: a whole line
            __builtin_nontemporal_store(w0 | static_cast<uint64_t>(w1) << 32, reinterpret_cast<uint64_t *>(o));
        } else {
            const int64_t v0 = 32 * static_cast<int64_t>(k) + 2 * lane - mis;
            if (v0 >= 0 && v0 < nvals) o[0] = w0;
            if (v0 + 1 >= 0 && v0 + 1 < nvals) o[1] = w1;
        }
        o += 32;
        ++k;
    }
}

// Final states of the instances, from the items that end them.
__global__ __launch_bounds__(kBlock) void k_ragged_commit_xs(const RaggedItem *items, uint64_t n_items,
                                                              const uint8_t *scratch, uint8_t *st, uint64_t S) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t i = t >> 4, lane = t & 15;
    if (i >= n_items || !items[i].last) return;
    const uint64_t u = items[i].unit;
    reinterpret_cast<uint2 *>(st)[16 * u + lane] = reinterpret_cast<const uint2 *>(scratch)[t];
    if (lane == 0)
        reinterpret_cast<uint64_t *>(st + 4 * S)[u] = reinterpret_cast<const uint64_t *>(scratch + 128 * n_items)[i];
}

unsigned blocks_for(uint64_t threads) { return static_cast<unsigned>((threads + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------- one stream
// The next N outputs of ONE stream (small kinds: contiguous; XS1024W: one
// instance in warp order) produced by many threads: chunk j of C outputs
// (XS1024W: C instance steps) starts from the state jumped by j*C.  The
// state is read from st_in and the final state written to st_out, a
// different buffer, so no chunk can read what the last one writes.
__device__ __forceinline__ void put(void *out, uint64_t idx, uint32_t u, int f32) {
    if (f32) static_cast<float *>(out)[idx] = static_cast<float>(u >> 8) * 0x1.0p-24f;
    else static_cast<uint32_t *>(out)[idx] = u;
}

template <class G>
__global__ __launch_bounds__(kBlock) void k_stream_fill_small(const uint8_t *st_in, uint8_t *st_out, uint64_t N,
                                                               uint64_t C, const uint64_t *t64, const uint32_t *t32,
                                                               void *out, int f32, uint32_t state_words) {
    __shared__ uint32_t tile[kBlock / 64][64][kSeg + 1];
    const uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t nch = (N + C - 1) / C;
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    const bool mine = j < nch;
    G g;
    uint32_t len = 0;
    if (mine) {
        g.load(st_in, 1, 0);
        jump(g, t64, t32, j, C);
        len = static_cast<uint32_t>(min(C, N - j * C));
    }
    uint32_t rounds = (len + kSeg - 1) / kSeg;
    for (int off = 32; off > 0; off >>= 1) rounds = max(rounds, static_cast<uint32_t>(__shfl_xor(static_cast<int>(rounds), off)));
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t base = rd * kSeg;
        const uint32_t cnt = len > base ? min(static_cast<uint32_t>(kSeg), len - base) : 0;
        for (uint32_t k = 0; k < cnt; ++k) tile[w][lane][k] = g.next();
        __builtin_amdgcn_wave_barrier();
        for (uint32_t q = 0; q < 64; q += 2) {
            const uint32_t src = q + half;
            const uint32_t len_q = static_cast<uint32_t>(__shfl(static_cast<int>(len), src));
            const uint64_t j_q = static_cast<uint64_t>(__shfl(static_cast<long long>(j), src));
            const uint32_t cnt_q = len_q > base ? min(static_cast<uint32_t>(kSeg), len_q - base) : 0;
            if (col < cnt_q) put(out, j_q * C + base + col, tile[w][src][col], f32);
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (mine && j == nch - 1) {
        // the whole one-stream image first: a generator's store writes only
        // what it changes (Philox: the position, not the key)
        for (uint32_t i = 0; i < state_words; ++i)
            reinterpret_cast<uint32_t *>(st_out)[i] = reinterpret_cast<const uint32_t *>(st_in)[i];
        g.store(st_out, 1, 0);
    }
}

// XS1024W instance (state: 32 words, step counter, Weyl seed): one 16-lane
// DPP row per chunk of C steps.
__global__ __launch_bounds__(kBlock) void k_stream_fill_xs(const uint8_t *st_in, uint8_t *st_out, uint64_t N,
                                                            uint64_t C, const uint32_t *t32, void *out, int f32) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t j = t >> 4, lane = t & 15;
    const uint64_t total_steps = (N + 31) / 32, nch = (total_steps + C - 1) / C;
    if (j >= nch) return;  // whole rows
    const uint2 w = reinterpret_cast<const uint2 *>(st_in)[lane];
    uint32_t a = w.x, b = w.y;
    if (j) xs1024_apply_poly(t32 + 32 * j, a, b);
    const uint64_t n0 = *reinterpret_cast<const uint64_t *>(st_in + 128);
    const uint32_t y0 = *reinterpret_cast<const uint32_t *>(st_in + 136);
    uint32_t y = y0 + static_cast<uint32_t>(n0 + j * C) * kWeylC;
    const uint64_t steps = min(C, total_steps - j * C);
    for (uint64_t k = 0; k < steps; ++k) {
        xs1024_step(a, b);
        y += kWeylC;
        const uint32_t m = weyl_mix(y);
        const uint64_t v = 32 * (j * C + k) + 2 * lane;
        if (v < N) put(out, v, a + m, f32);
        if (v + 1 < N) put(out, v + 1, b + m, f32);
    }
    if (j == nch - 1) {
        reinterpret_cast<uint2 *>(st_out)[lane] = make_uint2(a, b);
        if (lane == 0) {
            *reinterpret_cast<uint64_t *>(st_out + 128) = n0 + total_steps;
            *reinterpret_cast<uint32_t *>(st_out + 136) = y0;
        }
    }
}

}  // namespace

uint64_t stream_fill_chunk(rngx_kind) { return 4096; }

hipError_t launch_stream_fill(rngx_kind kind, const uint8_t *st_in, uint8_t *st_out, uint64_t N, int f32,
                              const uint64_t *t64, const uint32_t *t32, void *out, hipStream_t st) {
    if (N == 0) return hipSuccess;
    const uint64_t C = stream_fill_chunk(kind);
    if (kind == RNGX_XS1024W) {
        const uint64_t nch = ((N + 31) / 32 + C - 1) / C;
        hipLaunchKernelGGL(k_stream_fill_xs, dim3(blocks_for(16 * nch)), dim3(kBlock), 0, st, st_in, st_out, N, C, t32,
                           out, f32);
        return hipGetLastError();
    }
    const unsigned blocks = blocks_for((N + C - 1) / C);
    const uint32_t w = static_cast<uint32_t>(state_bytes(kind, 1) / 4);
    switch (kind) {
    case RNGX_LCG32: hipLaunchKernelGGL(k_stream_fill_small<Lcg32>, dim3(blocks), dim3(kBlock), 0, st, st_in, st_out, N, C, t64, t32, out, f32, w); break;
    case RNGX_LCG64: hipLaunchKernelGGL(k_stream_fill_small<Lcg64>, dim3(blocks), dim3(kBlock), 0, st, st_in, st_out, N, C, t64, t32, out, f32, w); break;
    case RNGX_MWC: hipLaunchKernelGGL(k_stream_fill_small<Mwc>, dim3(blocks), dim3(kBlock), 0, st, st_in, st_out, N, C, t64, t32, out, f32, w); break;
    case RNGX_XORWOW: hipLaunchKernelGGL(k_stream_fill_small<Xorwow>, dim3(blocks), dim3(kBlock), 0, st, st_in, st_out, N, C, t64, t32, out, f32, w); break;
    case RNGX_PHILOX4X32_10: hipLaunchKernelGGL(k_stream_fill_small<Philox>, dim3(blocks), dim3(kBlock), 0, st, st_in, st_out, N, C, t64, t32, out, f32, w); break;
    case RNGX_PHILOX4X32_7: hipLaunchKernelGGL(k_stream_fill_small<Philox7>, dim3(blocks), dim3(kBlock), 0, st, st_in, st_out, N, C, t64, t32, out, f32, w); break;
    default: break;
    }
    return hipGetLastError();
}

bool ragged_affine(rngx_kind kind) {
    return kind == RNGX_LCG32 || kind == RNGX_LCG64 || kind == RNGX_LCG32_SUB || kind == RNGX_LCG64_SUB;
}

bool ragged_wave(rngx_kind kind) {
    return ragged_affine(kind) || kind == RNGX_MWC || kind == RNGX_MWC_DIFF || kind == RNGX_PHILOX4X32_10 ||
           kind == RNGX_PHILOX4X32_7;
}

bool ragged_lane_table(rngx_kind kind) { return ragged_affine(kind) || kind == RNGX_MWC; }

// The tuned value of each shape: XS1024W rows per CU (the default fills every
// wave slot), else outputs per chunk, a lane's (4096) or, for the kinds
// written a whole wave span at a time, a wave's (65536).  Smaller chunks or
// fewer rows trade jumps for balance.
uint64_t ragged_shape_value(rngx_kind kind, int shape) {
    static constexpr uint64_t kXsRows[kRaggedShapes] = {kXsRowsPerCu, kXsRowsPerCu / 2, kXsRowsPerCu / 4};
    static constexpr uint64_t kWave[kRaggedShapes] = {65536, 16384, 262144};
    static constexpr uint64_t kLane[kRaggedShapes] = {4096, 1024, 16384};
    const int i = shape >= 0 && shape < kRaggedShapes ? shape : 0;
    if (kind == RNGX_XS1024W) return kXsRows[i];
    return ragged_wave(kind) ? kWave[i] : kLane[i];
}

uint64_t ragged_chunk(rngx_kind kind, int shape) { return ragged_shape_value(kind, shape); }

void ragged_plan(rngx_kind kind, const uint64_t *off, uint64_t n_units, int n_cu, RaggedPlan *plan, int shape) {
    std::vector<RaggedItem> &items = plan->items;
    items.clear();
    plan->slots.clear();
    plan->max_j = 0;
    if (kind != RNGX_XS1024W) {
        const uint64_t C = ragged_chunk(kind, shape);
        plan->step = C;
        for (uint64_t u = 0; u < n_units; ++u) {
            const uint64_t total = off[u + 1] - off[u];
            const uint64_t nch = (total + C - 1) / C;
            if (nch) plan->max_j = std::max(plan->max_j, nch - 1);
            for (uint64_t j = 0; j < nch; ++j) {
                RaggedItem it{};
                it.unit = u;
                it.j = j;
                it.len = static_cast<uint32_t>(std::min(C, total - j * C));
                it.last = j + 1 == nch;
                it.out = off[u] + j * C;
                it.nvals = it.len;
                items.push_back(it);
            }
        }
        return;
    }
    // XS1024W: concatenate the instances' steps and cut them into R slots of
    // about Q steps; a cut inside an instance is rounded to a multiple of J
    // steps (the jump table step), chosen so that the table stays small.
    uint64_t T = 0, max_steps = 0;
    for (uint64_t u = 0; u < n_units; ++u) {
        const uint64_t steps = (off[u + 1] - off[u] + 31) / 32;
        T += steps;
        max_steps = std::max(max_steps, steps);
    }
    uint64_t J = 128;
    while ((max_steps + J - 1) / J > 16384) J *= 2;
    plan->step = J;
    if (T == 0) return;
    const uint64_t R = std::max<uint64_t>(
        1, std::min<uint64_t>(ragged_shape_value(kind, shape) * std::max(n_cu, 1), (T + kXsMinSlotSteps - 1) / kXsMinSlotSteps));
    const uint64_t Q = (T + R - 1) / R;
    // Slot r should end at (r + 1) Q placed steps; G (steps placed) stays
    // below the open slot's target between pieces.
    uint64_t G = 0, r = 0;
    plan->slots.push_back(0);
    for (uint64_t u = 0; u < n_units; ++u) {
        const uint64_t total = off[u + 1] - off[u], steps = (total + 31) / 32;
        uint64_t p = 0;  // always 0 or a multiple of J
        while (p < steps) {
            const uint64_t target = (r + 1) * Q;
            uint64_t end = steps;
            bool close = false;
            if (G + (steps - p) >= target) {  // the slot ends in this instance
                close = true;
                const uint64_t want = p + (target - G);
                if (want < steps) {
                    uint64_t cut = (want + J / 2) / J * J;
                    if (cut <= p) cut = p + J;
                    if (cut < steps) end = cut;
                }
            }
            RaggedItem it{};
            it.unit = u;
            it.j = p / J;
            it.len = static_cast<uint32_t>(end - p);
            it.last = end == steps;
            it.out = off[u] + 32 * p;
            it.nvals = std::min<uint64_t>(32 * (end - p), total - 32 * p);
            plan->max_j = std::max(plan->max_j, it.j);
            items.push_back(it);
            G += end - p;
            p = end;
            if (close) {
                plan->slots.push_back(static_cast<uint32_t>(items.size()));
                r = std::max(r + 1, G / Q);
            }
        }
    }
    if (plan->slots.back() != items.size()) plan->slots.push_back(static_cast<uint32_t>(items.size()));
}

void ragged_lane_maps(const Gen *g, std::vector<uint64_t> *lane) {
    if (g->kind == RNGX_MWC) {  // a^(i+1) mod p for i < 256, then a^256
        std::vector<uint64_t> t64;
        std::vector<uint32_t> t32;
        jump_table(RNGX_MWC, 1, 257, &t64, &t32);  // a^0 .. a^256
        lane->assign(t64.begin() + 1, t64.begin() + 257);  // entries 0..255: a^1 .. a^256
        lane->push_back(t64[256]);                          // entry 256: the advance, a^256
        return;
    }
    // entry i: the (i+1)-step map (a lane whose first position is i); entry 256: the 256-step advance
    const uint64_t a = g->kind == RNGX_LCG32 ? kLcg32A : g->kind == RNGX_LCG64 ? kLcg64A : g->sub_a;
    const uint64_t c = g->kind == RNGX_LCG32 ? kLcg32C : g->kind == RNGX_LCG64 ? kLcg64C : g->sub_c;
    lane->assign(514, 0);
    for (int i = 0; i < 256; ++i) affine_power(a, c, i + 1, &(*lane)[2 * i], &(*lane)[2 * i + 1]);
    affine_power(a, c, 256, &(*lane)[512], &(*lane)[513]);
}

size_t ragged_scratch_bytes(rngx_kind kind, uint64_t n_items) {
    if (ragged_wave(kind)) return 8 * n_items;  // final states
    return kind == RNGX_XS1024W ? 136 * n_items : state_bytes(kind, n_items);
}

hipError_t launch_ragged(Ragged *r, uint32_t *d_out, hipStream_t st) {
    Gen *g = r->gen;
    const uint64_t n = r->n_items;
    if (n == 0) return hipSuccess;
    const uint64_t C = r->step;
    if (g->kind == RNGX_XS1024W) {
        hipLaunchKernelGGL(k_ragged_xs, dim3(blocks_for(16ull * r->n_slots)), dim3(kBlock), 0, st, r->d_items, n,
                           r->d_slots, r->n_slots, g->d_state, g->S, r->d_t32, C, r->d_scratch, d_out);
        hipLaunchKernelGGL(k_ragged_commit_xs, dim3(blocks_for(16 * n)), dim3(kBlock), 0, st, r->d_items, n,
                           r->d_scratch, g->d_state, g->S);
        return hipGetLastError();
    }
    if (ragged_affine(g->kind)) {
        const bool l64 = g->kind == RNGX_LCG64 || g->kind == RNGX_LCG64_SUB;
        uint64_t *scr = reinterpret_cast<uint64_t *>(r->d_scratch);
        if (l64) {
            hipLaunchKernelGGL(k_ragged_affine<true>, dim3(blocks_for(64 * n)), dim3(kBlock), 0, st, r->d_items, n,
                               r->d_t64, r->d_lane, g->d_state, scr, d_out);
            hipLaunchKernelGGL(k_ragged_commit_affine<true>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n,
                               scr, g->d_state);
        } else {
            hipLaunchKernelGGL(k_ragged_affine<false>, dim3(blocks_for(64 * n)), dim3(kBlock), 0, st, r->d_items, n,
                               r->d_t64, r->d_lane, g->d_state, scr, d_out);
            hipLaunchKernelGGL(k_ragged_commit_affine<false>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n,
                               scr, g->d_state);
        }
        return hipGetLastError();
    }
    if (ragged_wave(g->kind)) {
        uint64_t *scr = reinterpret_cast<uint64_t *>(r->d_scratch);
        uint64_t *dst = reinterpret_cast<uint64_t *>(g->d_state);  // MWC: y
        switch (g->kind) {
        case RNGX_MWC: hipLaunchKernelGGL(k_ragged_mwc<false>, dim3(blocks_for(64 * n)), dim3(kBlock), 0, st, r->d_items, n, r->d_t64, r->d_lane, g->d_state, g->S, C, scr, d_out); break;
        case RNGX_MWC_DIFF: hipLaunchKernelGGL(k_ragged_mwc<true>, dim3(blocks_for(64 * n)), dim3(kBlock), 0, st, r->d_items, n, r->d_t64, r->d_lane, g->d_state, g->S, C, scr, d_out); break;
        case RNGX_PHILOX4X32_10: hipLaunchKernelGGL(k_ragged_philox<10>, dim3(blocks_for(64 * n)), dim3(kBlock), 0, st, r->d_items, n, g->d_state, g->S, C, scr, d_out); break;
        case RNGX_PHILOX4X32_7: hipLaunchKernelGGL(k_ragged_philox<7>, dim3(blocks_for(64 * n)), dim3(kBlock), 0, st, r->d_items, n, g->d_state, g->S, C, scr, d_out); break;
        default: return hipErrorInvalidValue;
        }
        if (g->kind == RNGX_PHILOX4X32_10 || g->kind == RNGX_PHILOX4X32_7)
            dst = reinterpret_cast<uint64_t *>(g->d_state + 8 * g->S);  // positions
        hipLaunchKernelGGL(k_ragged_commit_u64, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, scr, dst);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_ragged_start_small, dim3(blocks_for(n)), dim3(kBlock), 0, st, g->kind, r->d_items, n,
                       g->d_state, g->S, r->d_scratch, r->d_t64, r->d_t32, C);
    switch (g->kind) {
    case RNGX_LCG32: hipLaunchKernelGGL(k_ragged_gen_small<Lcg32>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_LCG64: hipLaunchKernelGGL(k_ragged_gen_small<Lcg64>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_MWC: hipLaunchKernelGGL(k_ragged_gen_small<Mwc>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_MWC_DIFF: hipLaunchKernelGGL(k_ragged_gen_small<MwcDiff>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_XORWOW: hipLaunchKernelGGL(k_ragged_gen_small<Xorwow>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_PHILOX4X32_10: hipLaunchKernelGGL(k_ragged_gen_small<Philox>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_PHILOX4X32_7: hipLaunchKernelGGL(k_ragged_gen_small<Philox7>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_LCG32_SUB: hipLaunchKernelGGL(k_ragged_gen_small<Lcg32Sub>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    case RNGX_LCG64_SUB: hipLaunchKernelGGL(k_ragged_gen_small<Lcg64Sub>, dim3(blocks_for(n)), dim3(kBlock), 0, st, r->d_items, n, r->d_scratch, g->d_state, g->S, d_out); break;
    default: break;
    }
    return hipGetLastError();
}

}  // namespace rngx
