// Checkerboard Metropolis update of the 2D Ising ferromagnet (the paper's
// application test, Sec. 2) driven by the per-stream generators.
//
// Stream s = y*(L/4) + x/4 owns the 4-site run x0..x0+3 of row y.  In colour
// pass c it updates sites x0 + ((c+y)&1) and x0 + 2 + ((c+y)&1) with its next
// two outputs (XS1024W: one lane pair = streams 2u, 2u+1 = an 8-site run).
//
// Strip kernel (L up to ~5800): the lattice is cut into horizontal strips of
// R rows, one workgroup each.  A workgroup keeps its strip's spins in LDS and
// its streams' state in VGPRs for all sweeps of the call; only the two
// boundary rows of a strip go through global memory after each pass, and
// neighbouring strips synchronise through per-strip flags (release/acquire at
// agent scope).  Cooperative launch guarantees that every strip is resident,
// so every wait ends; the waits are also bounded.  A lattice that fits one
// workgroup (one strip, R = L) wraps its halo rows inside LDS.
//
// Per-pass kernels (larger L): one launch per colour pass, state and spins
// streamed from memory, energy reduced per block and then across blocks.
//
// Site update: with spins stored as int8 +1 = 0x01, -1 = 0xFF, bit 1 marks a
// down spin; the number m of neighbours that differ from a site is summed
// bytewise for a whole run (SWAR).  dE = 2 s h = 8 - 4 m, so a flip is
// accepted iff m >= 2, or m = 1 and r < T4, or m = 0 and r < T8.  After the
// colour-1 pass colour 0 is final and every bond has exactly one colour-1
// end, so E = -sum over colour-1 sites of s h = -sum (4 - 2 m_after).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <type_traits>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kOnes8 = 0x0101010101010101ull;

__global__ __launch_bounds__(kBlock) void k_hot_start(int8_t *spins, uint64_t n_words, uint64_t seed) {
    const uint64_t q = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= n_words) return;
    const uint64_t ss = seed ^ kSpinSeedXor;
    uint32_t w = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t site = 4 * q + i;
        const uint32_t v = (splitmix(ss, site + 1) >> 63) ? 0x01u : 0xFFu;  // +1 / -1 as int8
        w |= v << (8 * i);
    }
    reinterpret_cast<uint32_t *>(spins)[q] = w;
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t *p, uint64_t n) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Bytewise count (0..4) of neighbours that differ from each site of an
// NB-site run w; up/dn are the runs above and below, lb/rb the spins left of
// byte 0 and right of byte NB-1.
template <int NB>
__device__ __forceinline__ uint64_t mismatches(uint64_t w, uint64_t up, uint64_t dn, uint32_t lb, uint32_t rb) {
    constexpr uint64_t M = NB == 8 ? kOnes8 : 0x01010101ull;
    const uint64_t nw = (w >> 1) & M, nu = (up >> 1) & M, nd = (dn >> 1) & M;
    const uint64_t nl = ((nw << 8) | ((lb >> 1) & 1u)) & M;
    const uint64_t nr = (nw >> 8) | (static_cast<uint64_t>((rb >> 1) & 1u) << (8 * (NB - 1)));
    return (nu ^ nw) + (nd ^ nw) + (nl ^ nw) + (nr ^ nw);
}

// Metropolis decision for byte i; returns s_i h_i after the update.  Written
// without branches: the flip is a masked xor and the result a select.
__device__ __forceinline__ int metropolis(uint64_t &w, uint64_t m, int i, uint32_t r, uint64_t T4, uint64_t T8) {
    const uint32_t mi = static_cast<uint32_t>(m >> (8 * i)) & 0xFFu;
    const uint64_t thr = mi == 1 ? T4 : T8;
    const uint32_t acc = static_cast<uint32_t>(mi >= 2) | static_cast<uint32_t>(static_cast<uint64_t>(r) < thr);
    w ^= static_cast<uint64_t>(acc * 0xFEu) << (8 * i);
    const int e = 2 * static_cast<int>(mi) - 4;
    return acc ? e : -e;
}

// One Metropolis update of a site with mi (0..4) differing neighbours and
// draw r (multi-hit updates: the site's neighbours stay fixed between its
// hits); a taken flip turns mi into 4 - mi and toggles `flip`.
__device__ __forceinline__ void hit_mem(uint32_t &mi, uint32_t &flip, uint32_t r, uint64_t T4, uint64_t T8) {
    const uint64_t thr = mi == 1 ? T4 : T8;
    const bool acc = (mi >= 2) | (static_cast<uint64_t>(r) < thr);
    mi = acc ? 4 - mi : mi;
    flip ^= acc ? 1u : 0u;
}

// ---------------------------------------------------------------- units
// A unit is what one thread updates with one set of draws: a stream (4
// sites) for the small-state kinds, a lane pair of an XS1024W instance (8
// sites) for the paper's generator.  Units are numbered like the stream
// (small kinds) or stream/2 (XS1024W).
template <class G>
struct SmallUnit {
    static constexpr int kNB = 4;
    G g;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t u) { g.load(st, S, u); }
    __device__ void store(uint8_t *st, uint64_t S, uint64_t u, uint64_t) const { g.store(st, S, u); }
    __device__ void draw(uint32_t (&r)[2]) { r[0] = g.next(); r[1] = g.next(); }
    // multi-hit updates: n draws in order to f0, then n more to f1
    template <class F0, class F1>
    __device__ void draws2(uint32_t n, F0 &&f0, F1 &&f1) {
        for (uint32_t i = 0; i < n; ++i) f0(g.next());
        for (uint32_t i = 0; i < n; ++i) f1(g.next());
    }
};

// Philox with only key and position held: the two draws of a pass come from
// one block unless they straddle a block boundary.
template <int ROUNDS>
struct PhiloxUnitR {
    static constexpr int kNB = 4;
    uint32_t k0, k1;
    uint64_t pos;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t u) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        k0 = p[u]; k1 = p[S + u];
        pos = reinterpret_cast<const uint64_t *>(st + 8 * S)[u];
    }
    __device__ void store(uint8_t *st, uint64_t S, uint64_t u, uint64_t) const {
        reinterpret_cast<uint64_t *>(st + 8 * S)[u] = pos;
    }
    __device__ void draw(uint32_t (&r)[2]) {
        uint32_t b0, b1, b2, b3;
        philox_block<ROUNDS>(k0, k1, pos >> 2, b0, b1, b2, b3);
        const uint32_t j = static_cast<uint32_t>(pos) & 3;
        r[0] = j == 0 ? b0 : j == 1 ? b1 : j == 2 ? b2 : b3;
        if (j == 3) philox_block<ROUNDS>(k0, k1, (pos >> 2) + 1, b0, b1, b2, b3);
        r[1] = j == 0 ? b1 : j == 1 ? b2 : j == 2 ? b3 : b0;
        pos += 2;
    }
    // as SmallUnit::draws2, in one loop so that a block serves four draws in
    // a row also across the two runs
    template <class F0, class F1>
    __device__ void draws2(uint32_t n, F0 &&f0, F1 &&f1) {
        uint32_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
        for (uint32_t i = 0; i < 2 * n; ++i) {
            const uint32_t j = static_cast<uint32_t>(pos) & 3;
            if (i == 0 || j == 0) philox_block<ROUNDS>(k0, k1, pos >> 2, b0, b1, b2, b3);
            const uint32_t r = j == 0 ? b0 : j == 1 ? b1 : j == 2 ? b2 : b3;
            if (i < n) f0(r);
            else f1(r);
            ++pos;
        }
    }
};
using PhiloxUnit = PhiloxUnitR<10>;
using PhiloxUnit7 = PhiloxUnitR<7>;

// Philox in a strip whose streams all stand at the same block boundary at
// the start of a call (the usual case: seeded at 0, and every call advances
// every stream by the same multiple of 4).  A sweep takes the four words of
// one block: the colour-0 pass makes block blk0 + t, uses words 0 and 1 and
// keeps 2 and 3 for the colour-1 pass, so each block is made once rather
// than once per pass, and the position, the same for all units, is not held
// per unit.
template <int ROUNDS>
struct PhiloxSweepUnitR {
    static constexpr int kNB = 4;
    uint32_t k0, k1, c2, c3;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t u) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        k0 = p[u]; k1 = p[S + u];
        c2 = c3 = 0;
    }
    template <class Args>
    __device__ void store_at(uint8_t *st, uint64_t S, uint64_t u, const Args &g) const {
        reinterpret_cast<uint64_t *>(st + 8 * S)[u] = 4 * (g.blk0 + g.n_sweeps);
    }
    template <class Args>
    __device__ void draw_at(uint32_t (&r)[2], const Args &g, uint64_t sweep, int c) {
        if (c == 0) {
            philox_block<ROUNDS>(k0, k1, g.blk0 + sweep, r[0], r[1], c2, c3);
        } else {
            r[0] = c2;
            r[1] = c3;
        }
    }
};
template <class Unit> struct SweepCounter : std::false_type {};  // units that derive their pass from the call's start
template <int ROUNDS> struct SweepCounter<PhiloxSweepUnitR<ROUNDS>> : std::true_type {};

// Lagged Fibonacci units in strips (single-hit).  A strip holds whole
// instances (1024 units each) and runs 1024 threads, so slot i of thread t is
// stream t of the strip's instance i.  Before each colour pass the workgroup
// makes that pass's two rows of every instance of the strip in LDS rings of B
// words (value v at v mod B; runs of at most kRun values, a barrier each,
// whose reads and writes never share a ring word) and each thread takes
// value t of both rows for every slot; the unit only hands them out, in the
// order of the per-pass path (row 1 to the first colour-c site, row 2 to the
// second).
template <int LR, int LS>
struct LfgStripUnit {
    static constexpr int kNB = 4;
    static constexpr uint32_t kR = LR, kS = LS;
    static constexpr uint32_t B = LR < 1024 ? 1024 : 2048;
    static constexpr uint32_t kRun = (B - LR) < static_cast<uint32_t>(LS) ? B - LR : LS;
    static_assert(B >= LR + 1 && kRun >= 1, "ring too small");
    uint32_t d0, d1;
    __device__ void load(const uint8_t *, uint64_t, uint64_t) {}
    __device__ void store(uint8_t *, uint64_t, uint64_t, uint64_t) const {}
    __device__ void draw(uint32_t (&r)[2]) { r[0] = d0; r[1] = d1; }
};
template <class Unit> struct IsLfgStrip : std::false_type {};
template <int LR, int LS> struct IsLfgStrip<LfgStripUnit<LR, LS>> : std::true_type {};
// LDS of the rings of a strip's instances (after the strip's own bytes).
template <class Unit>
__host__ __device__ constexpr uint64_t lfg_ring_bytes(uint32_t units) {
    if constexpr (IsLfgStrip<Unit>::value) return 4ull * Unit::B * (units / 1024) + 16;
    else return 0;
}

// XS1024W lane pair u: lane u%16 of instance u/16 of the handle (words 2u,
// 2u+1 = streams 2u and 2u+1).  Two instance steps per pass; the draws are
// ordered stream 2u first, stream 2u+1 second, each in step order.
struct XsUnit {
    static constexpr int kNB = 8;
    uint32_t a, b, y;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t u) {
        const uint2 w = reinterpret_cast<const uint2 *>(st)[u];
        a = w.x; b = w.y;
        const uint64_t n = reinterpret_cast<const uint64_t *>(st + 4 * S)[u >> 4];
        y = *reinterpret_cast<const uint32_t *>(st + 4 * S + 8 * (S / 32)) + static_cast<uint32_t>(n) * kWeylC;
    }
    __device__ void store(uint8_t *st, uint64_t S, uint64_t u, uint64_t steps) const {
        reinterpret_cast<uint2 *>(st)[u] = make_uint2(a, b);
        if ((u & 15) == 0) reinterpret_cast<uint64_t *>(st + 4 * S)[u >> 4] += steps;
    }
    __device__ void draw(uint32_t (&r)[4]) {
        xs1024_step(a, b);
        y += kWeylC;
        uint32_t m = weyl_mix(y);
        r[0] = a + m; r[2] = b + m;
        xs1024_step(a, b);
        y += kWeylC;
        m = weyl_mix(y);
        r[1] = a + m; r[3] = b + m;
    }
    // one instance step: the next draw of stream 2u (ra) and of 2u+1 (rb)
    __device__ void pair(uint32_t &ra, uint32_t &rb) {
        xs1024_step(a, b);
        y += kWeylC;
        const uint32_t m = weyl_mix(y);
        ra = a + m;
        rb = b + m;
    }
};

// XS1024W in a strip whose instances have all taken the same number of
// steps at the start of a call (the usual case: every call advances every
// instance alike).  The Weyl word of a pass is then the same for every unit:
// it follows from the call's start (step count blk0, Weyl word y_start) and
// the sweep, instead of being held and stepped per unit.
struct XsSweepUnit {
    static constexpr int kNB = 8;
    uint32_t a, b;
    __device__ void load(const uint8_t *st, uint64_t, uint64_t u) {
        const uint2 w = reinterpret_cast<const uint2 *>(st)[u];
        a = w.x; b = w.y;
    }
    template <class Args>
    __device__ void store_at(uint8_t *st, uint64_t S, uint64_t u, const Args &g) const {
        reinterpret_cast<uint2 *>(st)[u] = make_uint2(a, b);
        if ((u & 15) == 0) reinterpret_cast<uint64_t *>(st + 4 * S)[u >> 4] = g.blk0 + 4 * g.n_sweeps;
    }
    // as XsUnit::draw for the pass (sweep, c): 4 sweep + 2 c steps after the start
    template <class Args>
    __device__ void draw_at(uint32_t (&r)[4], const Args &g, uint64_t sweep, int c) {
        const uint32_t y = g.y_start + static_cast<uint32_t>(4 * sweep + 2 * c) * kWeylC;
        xs1024_step(a, b);
        uint32_t m = weyl_mix(y + kWeylC);
        r[0] = a + m; r[2] = b + m;
        xs1024_step(a, b);
        m = weyl_mix(y + 2 * kWeylC);
        r[1] = a + m; r[3] = b + m;
    }
};
template <> struct SweepCounter<XsSweepUnit> : std::true_type {};
template <class Unit> struct SweepOf { using type = void; };  // the sweep form of a unit, if it has one
template <int ROUNDS> struct SweepOf<PhiloxUnitR<ROUNDS>> { using type = PhiloxSweepUnitR<ROUNDS>; };
template <> struct SweepOf<XsUnit> { using type = XsSweepUnit; };

template <int NB>
__device__ __forceinline__ uint64_t lds_run(const uint8_t *p) {
    if constexpr (NB == 8) return *reinterpret_cast<const uint64_t *>(p);
    else return *reinterpret_cast<const uint32_t *>(p);
}
template <int NB>
__device__ __forceinline__ void lds_put(uint8_t *p, uint64_t w) {
    if constexpr (NB == 8) *reinterpret_cast<uint64_t *>(p) = w;
    else *reinterpret_cast<uint32_t *>(p) = static_cast<uint32_t>(w);
}

// ---------------------------------------------------------------- strips
// A batch replica runs in one of three modes: in memory by one workgroup
// (kReplicaMemory), on chip by one workgroup (kReplicaOnChip, R = L), or as
// a gang of nwg strip workgroups of R rows each (kReplicaStrips) that
// exchange tagged halo words like the strips of one lattice.
constexpr uint32_t kReplicaMemory = 0, kReplicaOnChip = 1, kReplicaStrips = 2;
struct ReplicaDesc {
    int8_t *spins;
    uint8_t *st;
    uint64_t S;
    uint32_t L, mode;
    uint64_t T4, T8, n_sweeps;
    int32_t *trace;   // may be null
    uint32_t R, nwg, units;  // strips: rows and units per strip, strip count
    uint64_t *halo;   // strips: 2 slots x nwg x 2 rows x L/4 tagged words
    uint32_t *err;    // the lattice's error word (a strip gave up waiting)
    uint32_t R_last;  // strips: rows of the last strip (1..R; the others have R)
    uint32_t *gang;   // strips: arrival counter of the gang's workgroups (zeroed before each run)
    uint64_t start_ticks;  // strips: wall-clock ticks a gang member waits for the others to start
};

struct StripArgs {
    int8_t *spins;
    uint8_t *st;
    uint64_t S;
    uint32_t L, R, nwg, units;  // units per strip
    uint64_t T4, T8, n_sweeps;
    int32_t *trace;             // may be null
    uint64_t *halo;             // 2 slots x nwg x 2 rows x L/4 tagged words
    uint32_t epoch0;            // pass tags of this call are epoch0 + 1, epoch0 + 2, ...
    uint32_t *err;
    uint32_t hits;              // Metropolis updates per visited site (multi-hit kernels)
    uint32_t R0;                // rows of every strip but the last: strip r starts at row r*R0
    uint64_t blk0;              // sweep forms, at the start: Philox the common block index, XS1024W the step count
    uint32_t y_start;           // sweep-form XS1024W: the common Weyl word at the start
};

constexpr uint32_t kSpinLimit = 1u << 20;

// Halo words: 4 spins in the low half, the pass tag in the high half, both
// written by one 64-bit agent-scope atomic store, so a word read with the
// expected tag holds that pass's spins.  Polls one word until its tag is
// `tag`; gives up after kSpinLimit polls and records that in *err (once set,
// every later poll returns at once, so a failed exchange ends the kernel
// quickly with an invalid lattice instead of stalling it).
__device__ __forceinline__ uint32_t poll_word(const uint64_t *p, uint64_t v, uint32_t tag, uint32_t *err) {
    for (uint32_t it = 0; static_cast<uint32_t>(v >> 32) != tag; ++it) {
        if (it >= kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return static_cast<uint32_t>(v);
}

__device__ __forceinline__ void put_word(uint64_t *p, uint32_t spins, uint32_t tag) {
    __hip_atomic_store(p, (static_cast<uint64_t>(tag) << 32) | spins, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two rows of L bytes (src0 -> dst0, src1 -> dst1) by the whole block: all
// loads are issued before the first LDS write, one round trip in all.
__device__ __forceinline__ void copy_rows(uint8_t *dst0, const uint8_t *src0, uint8_t *dst1, const uint8_t *src1,
                                          uint32_t L, uint32_t t, uint32_t nt) {
    const uint32_t n = L / 16;  // 16-byte pieces per row
    for (uint32_t i = t; i < 2 * n; i += nt) {
        const bool second = i >= n;
        const uint32_t o = 16 * (second ? i - n : i);
        const uint4 v = *reinterpret_cast<const uint4 *>((second ? src1 : src0) + o);
        *reinterpret_cast<uint4 *>((second ? dst1 : dst0) + o) = v;
    }
}

// Sum of v over the block (result valid in thread 0).
__device__ __forceinline__ int block_sum(int v, int *scratch) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const uint32_t w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    int s = 0;
    if (threadIdx.x == 0)
        for (uint32_t i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- on-chip update
// LDS holds the strip's rows (and one halo row above and below) at a pitch
// of L + 2*kPad bytes with the spins at +kPad; the word just before a row's
// spins is a copy of its last four spins and the word just after them a copy
// of its first four ("ghost" words), so every run finds its left and right
// neighbours at fixed offsets.
constexpr uint32_t kPad = 16;
__host__ __device__ constexpr uint32_t lds_pitch(uint32_t L) { return L + 2 * kPad; }
// Rows: 0 and R+1 the rows above and below the strip (halo buffer 0),
// 1..R the strip, R+2 and R+3 halo buffer 1; then 64 bytes of per-wave sums
// and a zero word.
__host__ __device__ constexpr uint64_t strip_lds_bytes(uint32_t L, uint32_t R) {
    return static_cast<uint64_t>(R + 4) * lds_pitch(L) + 80;
}

// Acceptance in 32 bits.  With d = twice the number of a site's neighbours
// that differ from it (0, 2, .., 8), the flip is taken if d >= lo, else iff
// r < (d == 2 ? t4 : t8).  lo is 4 except when a threshold is 2^32 (every
// draw accepts), which 32 bits cannot hold: lo = 2 when that is T4, lo = 0
// when it is T8 (and then also T4, since T8 <= T4).
struct Accept {
    uint32_t t4, t8, lo;
};
__device__ __forceinline__ Accept make_accept(uint64_t T4, uint64_t T8) {
    constexpr uint64_t kAll = 1ull << 32;
    return Accept{T4 >= kAll ? 0xFFFFFFFFu : static_cast<uint32_t>(T4), T8 >= kAll ? 0xFFFFFFFFu : static_cast<uint32_t>(T8),
                  T8 >= kAll ? 0u : T4 >= kAll ? 2u : 4u};
}

// Twice the number of differing neighbours of each byte of a 4-spin word w
// (spins +-1 as int8: two differ iff bit 1 of their xor is set); l and r are
// the words left and right of w, u and d the words above and below.
__device__ __forceinline__ uint32_t mismatch2(uint32_t w, uint32_t l, uint32_t r, uint32_t u, uint32_t d) {
    constexpr uint32_t kBit1 = 0x02020202u;
    const uint32_t left = __builtin_amdgcn_alignbit(w, l, 24);  // byte i: spin i-1
    const uint32_t right = __builtin_amdgcn_alignbit(r, w, 8);  // byte i: spin i+1
    return ((w ^ u) & kBit1) + ((w ^ d) & kBit1) + ((w ^ left) & kBit1) + ((w ^ right) & kBit1);
}

// Metropolis decision for the byte at bit offset sh of a word with doubled
// counts m2 and draw r: returns f (the flip mask of that byte) if accepted,
// else 0.  With E, adds the byte's doubled count after the step to *esum.
template <bool E>
__device__ __forceinline__ uint32_t decide(uint32_t m2, uint32_t sh, uint32_t f, uint32_t r, const Accept &A,
                                           uint32_t &esum) {
    const uint32_t d = __builtin_amdgcn_ubfe(m2, sh, 8);
    // compares combined as lane masks (no select of the threshold): since
    // t8 <= t4, r < t8 accepts at d = 2 too, so it needs no d != 2 term
    const bool acc = (d >= A.lo) | (r < A.t8) | ((d == 2) & (r < A.t4));
    if constexpr (E) esum += acc ? 8 - d : d;
    return acc ? f : 0u;
}

// One update of a multi-hit site with doubled count d and draw r; a taken
// flip turns d into 8 - d and toggles `flip`.
__device__ __forceinline__ void hit_lds(uint32_t &d, uint32_t &flip, uint32_t r, const Accept &A) {
    const bool acc = (d >= A.lo) | (r < A.t8) | ((d == 2) & (r < A.t4));  // as in decide
    d = acc ? 8 - d : d;
    flip ^= acc ? 1u : 0u;
}

// Unit k of the strip starts at LDS offset `off` (its row yl+1); bit 27:
// unit in the strip's top row, bit 28: in its bottom row, bit 29: run starts
// the row, bit 30: run ends the row, bit 31: (row0+yl) odd, i.e. its
// colour-c sites are the odd bytes when c = 0.
constexpr uint32_t kOffMask = (1u << 27) - 1;
template <int NB>
__device__ __forceinline__ uint32_t unit_place(uint32_t k, uint32_t L, uint32_t R, uint64_t row0) {
    const uint32_t upr = L / NB;
    const uint32_t yl = k / upr, x0 = (k % upr) * NB;
    uint32_t off = (yl + 1) * lds_pitch(L) + kPad + x0;
    if (yl == 0) off |= 1u << 27;
    if (yl == R - 1) off |= 1u << 28;
    if (x0 == 0) off |= 1u << 29;
    if (x0 + NB == L) off |= 1u << 30;
    if ((row0 + yl) & 1) off |= 1u << 31;
    return off;
}

// Colour-c update of the unit at `pl` (place word, made opaque per pass);
// returns its new spins.  The rows above and below are read at off - P +
// up_add and off + P + dn_add (non-zero only to reach halo buffer 1).  The
// draws go to the colour-c bytes in increasing order.  MH: `hits` updates
// per site in a row, each stream's first site taking its first `hits`
// draws of the pass (XS1024W: instance steps 1..hits serve the first site
// of both streams of the lane pair, steps hits+1..2 hits the second).
template <class Unit, bool E, bool MH>
__device__ __forceinline__ uint64_t update_unit(uint8_t *lds, uint32_t pl, uint32_t P, uint32_t up_add, uint32_t dn_add,
                                                int c, Unit &u, const Accept &A, uint32_t &esum, uint32_t hits,
                                                const StripArgs &g, uint64_t sweep) {
    constexpr int NB = Unit::kNB;
    const uint32_t off = pl & kOffMask;
    const uint32_t sh0 = ((pl >> 31) ^ static_cast<uint32_t>(c)) << 3;  // bit offset of the first colour-c byte
    const uint32_t f0 = 0xFEu << sh0, f1 = f0 << 16;                     // flip masks (+1 <-> -1)
    const uint32_t *l32 = reinterpret_cast<const uint32_t *>(lds + off);
    if constexpr (MH) {
        if constexpr (NB == 4) {
            const uint32_t w = l32[0];
            const uint32_t m2 = mismatch2(w, l32[-1], l32[1], *reinterpret_cast<const uint32_t *>(lds + off - P + up_add),
                                          *reinterpret_cast<const uint32_t *>(lds + off + P + dn_add));
            uint32_t d0 = __builtin_amdgcn_ubfe(m2, sh0, 8), d1 = __builtin_amdgcn_ubfe(m2, sh0 + 16, 8);
            uint32_t x0 = 0, x1 = 0;
            u.draws2(hits, [&](uint32_t r) { hit_lds(d0, x0, r, A); }, [&](uint32_t r) { hit_lds(d1, x1, r, A); });
            if constexpr (E) esum += d0 + d1;
            const uint32_t nw = w ^ (x0 ? f0 : 0u) ^ (x1 ? f1 : 0u);
            *reinterpret_cast<uint32_t *>(lds + off) = nw;
            return nw;
        } else {
            const uint2 w = *reinterpret_cast<const uint2 *>(lds + off);
            const uint2 up = *reinterpret_cast<const uint2 *>(lds + off - P + up_add);
            const uint2 dn = *reinterpret_cast<const uint2 *>(lds + off + P + dn_add);
            const uint32_t m2a = mismatch2(w.x, l32[-1], w.y, up.x, dn.x);
            const uint32_t m2b = mismatch2(w.y, w.x, l32[2], up.y, dn.y);
            uint32_t d0 = __builtin_amdgcn_ubfe(m2a, sh0, 8), d1 = __builtin_amdgcn_ubfe(m2a, sh0 + 16, 8);
            uint32_t d2 = __builtin_amdgcn_ubfe(m2b, sh0, 8), d3 = __builtin_amdgcn_ubfe(m2b, sh0 + 16, 8);
            uint32_t x0 = 0, x1 = 0, x2 = 0, x3 = 0;
            for (uint32_t i = 0; i < hits; ++i) {
                uint32_t ra, rb;
                u.pair(ra, rb);
                hit_lds(d0, x0, ra, A);
                hit_lds(d2, x2, rb, A);
            }
            for (uint32_t i = 0; i < hits; ++i) {
                uint32_t ra, rb;
                u.pair(ra, rb);
                hit_lds(d1, x1, ra, A);
                hit_lds(d3, x3, rb, A);
            }
            if constexpr (E) esum += d0 + d1 + d2 + d3;
            const uint2 nw = make_uint2(w.x ^ (x0 ? f0 : 0u) ^ (x1 ? f1 : 0u), w.y ^ (x2 ? f0 : 0u) ^ (x3 ? f1 : 0u));
            *reinterpret_cast<uint2 *>(lds + off) = nw;
            return (static_cast<uint64_t>(nw.y) << 32) | nw.x;
        }
    }
    uint32_t rr[NB / 2];
    if constexpr (SweepCounter<Unit>::value) u.draw_at(rr, g, sweep, c);
    else u.draw(rr);
    if constexpr (NB == 4) {
        const uint32_t w = l32[0];
        const uint32_t m2 = mismatch2(w, l32[-1], l32[1], *reinterpret_cast<const uint32_t *>(lds + off - P + up_add),
                                      *reinterpret_cast<const uint32_t *>(lds + off + P + dn_add));
        const uint32_t g0 = decide<E>(m2, sh0, f0, rr[0], A, esum);
        const uint32_t g1 = decide<E>(m2, sh0 + 16, f1, rr[1], A, esum);
        const uint32_t nw = w ^ (g0 | g1);
        *reinterpret_cast<uint32_t *>(lds + off) = nw;
        return nw;
    } else {
        const uint2 w = *reinterpret_cast<const uint2 *>(lds + off);
        const uint2 up = *reinterpret_cast<const uint2 *>(lds + off - P + up_add);
        const uint2 dn = *reinterpret_cast<const uint2 *>(lds + off + P + dn_add);
        const uint32_t m2a = mismatch2(w.x, l32[-1], w.y, up.x, dn.x);
        const uint32_t m2b = mismatch2(w.y, w.x, l32[2], up.y, dn.y);
        const uint32_t g0 = decide<E>(m2a, sh0, f0, rr[0], A, esum);
        const uint32_t g1 = decide<E>(m2a, sh0 + 16, f1, rr[1], A, esum);
        const uint32_t g2 = decide<E>(m2b, sh0, f0, rr[2], A, esum);
        const uint32_t g3 = decide<E>(m2b, sh0 + 16, f1, rr[3], A, esum);
        const uint2 nw = make_uint2(w.x ^ (g0 | g1), w.y ^ (g2 | g3));
        *reinterpret_cast<uint2 *>(lds + off) = nw;
        return (static_cast<uint64_t>(nw.y) << 32) | nw.x;
    }
}

// Ghost words of LDS rows [y0, y1) from the same rows' spins.
__device__ __forceinline__ void refresh_ghosts(uint8_t *lds, uint32_t L, uint32_t y0, uint32_t y1, uint32_t t,
                                               uint32_t nt) {
    const uint32_t P = lds_pitch(L);
    for (uint32_t i = 2 * y0 + t; i < 2 * y1; i += nt) {
        uint8_t *row = lds + (i >> 1) * P + kPad;
        if (i & 1) *reinterpret_cast<uint32_t *>(row + L) = *reinterpret_cast<const uint32_t *>(row);
        else *reinterpret_cast<uint32_t *>(row - 4) = *reinterpret_cast<const uint32_t *>(row + L - 4);
    }
}

// R rows of L spins between global memory (L apart) and LDS (pitch apart).
template <bool TO_LDS>
__device__ __forceinline__ void copy_strip(uint8_t *lds_row1, int8_t *g, uint32_t L, uint32_t R, uint32_t t, uint32_t nt) {
    const uint32_t n16 = L / 16, P = lds_pitch(L);
    for (uint32_t i = t; i < R * n16; i += nt) {
        const uint32_t y = i / n16, x = (i - y * n16) * 16;
        uint4 *l = reinterpret_cast<uint4 *>(lds_row1 + y * P + x);
        uint4 *m = reinterpret_cast<uint4 *>(g + static_cast<uint64_t>(y) * L + x);
        if constexpr (TO_LDS) *l = *m;
        else *m = *l;
    }
}

// A unit whose run starts (bit 29) or ends (bit 30) its row also refreshes
// the row's ghost word on that side (run: the run's first spin in LDS).
// Other threads may read that ghost during the pass, but only its
// other-colour byte, which this update does not change.
template <int NB>
__device__ __forceinline__ void edge_ghosts(uint8_t *run, uint32_t pl, uint32_t L, uint64_t nw) {
    if ((pl >> 29) & 1) *reinterpret_cast<uint32_t *>(run + L) = static_cast<uint32_t>(nw);  // first 4 spins
    if ((pl >> 30) & 1)                                                                      // last 4 spins
        *reinterpret_cast<uint32_t *>(run + NB - L - 4) = static_cast<uint32_t>(nw >> (8 * (NB - 4)));
}

// All sweeps of strip r (R rows at row r*R) held in `lds`
// (strip_lds_bytes(L, R)) by the calling workgroup.
//
// Pass q reads the halo rows of buffer q&1 and fills buffer (q+1)&1, so a
// pass needs a single barrier (before it starts):
//   - every unit updates its sites and, at a row end, the row's ghost word;
//   - with one strip (periodic in y) the units of the top and bottom rows
//     also write their new runs into the other side's row of the next
//     buffer;
//   - with several strips they store them as tagged words into pass q's
//     halo slot in global memory, and every thread pulls its share of the
//     neighbours' tagged words (loads issued some slots before the end,
//     polled until the tags say pass q) into the next buffer.
// Sites of one colour are independent within a pass, so the slot order changes
// no result; the slots holding the top and bottom rows go first so that the
// neighbours' words are ready when pulled.
// Place words in LDS (after the per-wave sums) instead of registers when a
// thread's unit states are large: frees SPT registers for kinds that would
// otherwise spill.  The batch kernel keeps them in registers (its LDS budget
// is tighter).
template <class Unit, int SPT>
__host__ __device__ constexpr bool place_in_lds() {
    return !IsLfgStrip<Unit>::value && SPT * (sizeof(Unit) / 4 + 1) >= 40;
}

template <class Unit, int SPT, bool EARLY, bool PLDS, bool MH = false>
__device__ __forceinline__ void strip_body(const StripArgs &a, uint32_t r, uint8_t *lds) {
    constexpr int NB = Unit::kNB;
    const uint32_t L = a.L, R = a.R, nwg = a.nwg, t = threadIdx.x, nt = blockDim.x;
    const uint32_t P = lds_pitch(L);
    const uint64_t row0 = static_cast<uint64_t>(r) * a.R0;
    const uint32_t upr = L / NB;             // units per row
    const uint32_t W = L / 4;                // halo words per row
    int *wave_e = reinterpret_cast<int *>(lds + (R + 4) * P);
    uint32_t *zero_word = reinterpret_cast<uint32_t *>(lds + (R + 4) * P + 64);
    if (t == 0) *zero_word = 0;
    // interiors of the halo rows (above, below) of buffers 0 and 1
    const uint32_t h_up[2] = {kPad, (R + 2) * P + kPad}, h_dn[2] = {(R + 1) * P + kPad, (R + 3) * P + kPad};

    // strip and halo rows (buffer 0) from the lattice, then every ghost word
    const uint8_t *gs = reinterpret_cast<const uint8_t *>(a.spins);
    copy_strip<true>(lds + P + kPad, a.spins + row0 * L, L, R, t, nt);
    const uint64_t up_row = (row0 + L - 1) % L, dn_row = (row0 + R) % L;
    copy_rows(lds + h_up[0], gs + up_row * L, lds + h_dn[0], gs + dn_row * L, L, t, nt);
    __syncthreads();
    refresh_ghosts(lds, L, 0, R + 2, t, nt);

    const uint64_t ubase = row0 * upr;  // first unit (and stream) of the strip
    Unit u[SPT];
    uint32_t place[PLDS ? 1 : SPT];
    uint32_t *place_lds = reinterpret_cast<uint32_t *>(lds + (R + 4) * P + 80);  // [slot][thread] when PLDS
    uint32_t my_units = 0;
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
        const uint32_t k = t + i * nt;
        if (k < a.units) {
            u[i].load(a.st, a.S, ubase + k);
            const uint32_t pw = unit_place<NB>(k, L, R, row0);
            if constexpr (PLDS) place_lds[i * nt + t] = pw;
            else place[i] = pw;
            ++my_units;
        }
    }
    const Accept A = make_accept(a.T4, a.T8);

    // lagged Fibonacci: the windows of the strip's instances into their rings
    // (ordered before use by the barrier that starts every pass)
    uint32_t *rings = reinterpret_cast<uint32_t *>(lds + ((strip_lds_bytes(L, R) + 15) & ~15ull));
    uint32_t lq = 0;  // index of the next value of every instance of the strip
    if constexpr (IsLfgStrip<Unit>::value) {
        constexpr uint32_t LR = Unit::kR, RB = Unit::B;
        const uint32_t n_inst = a.units / 1024;
        const uint32_t *X = reinterpret_cast<const uint32_t *>(a.st) + (ubase / 1024) * LR;
        for (uint32_t idx = t; idx < n_inst * LR; idx += nt) {
            const uint32_t i = idx / LR, j = idx - i * LR;
            rings[i * RB + RB - LR + j] = X[idx];
        }
    }

    const uint32_t up_wg = (r + nwg - 1) % nwg, dn_wg = (r + 1) % nwg;
    // EARLY: top row entirely in slot 0 and bottom row entirely in slot
    // SPT-1, so only those two slots hold boundary units (the host picks the
    // instantiation with the same test).
    constexpr bool early = EARLY;
    constexpr int kPullAt = SPT >= 4 ? SPT * 5 / 8 : SPT - 1;  // neighbours' words requested after this slot
    uint32_t q = 0;  // pass counter

    // trace[sweep] from the wave sums of that sweep's colour-1 pass (read
    // after the barrier that follows them), by the last wavefront.
    auto flush_energy = [&](uint64_t sweep) {
        if (a.trace && t >= nt - 64) {
            const uint32_t lane = t & 63;
            int v = lane < (nt >> 6) ? wave_e[lane] : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) {
                if (nwg == 1) a.trace[sweep] = -v;  // the only contributor
                else atomicAdd(a.trace + sweep, -v);
            }
        }
    };

    // One colour pass; E: accumulate the energy terms (colour 1).
    auto pass = [&](auto e_tag, int c, uint64_t sweep) {
        constexpr bool E = decltype(e_tag)::value;
        __syncthreads();  // pass q-1 done, buffer q&1 complete
        if (c == 0 && sweep > 0) flush_energy(sweep - 1);  // colour 1 of the previous sweep
        const uint32_t cur = q & 1, nxt = cur ^ 1;
        const uint32_t tag = a.epoch0 + q + 1;
        const uint32_t up_add = h_up[cur] - h_up[0], dn_add = h_dn[cur] - h_dn[0];
        uint64_t *mine = nwg > 1 ? a.halo + (static_cast<uint64_t>(cur) * nwg + r) * 2 * W : nullptr;  // [top][bottom]
        const uint64_t *from_up = nwg > 1 ? a.halo + ((static_cast<uint64_t>(cur) * nwg + up_wg) * 2 + 1) * W : nullptr;
        const uint64_t *from_dn = nwg > 1 ? a.halo + (static_cast<uint64_t>(cur) * nwg + dn_wg) * 2 * W : nullptr;
        // my pulled words: i = t + m nt (< 2W), i < W from the strip above
        auto src_word = [&](uint32_t i) { return i < W ? from_up + i : from_dn + (i - W); };
        uint64_t pre0 = 0, pre1 = 0;
        auto request = [&]() {
            if (t < 2 * W) pre0 = __hip_atomic_load(src_word(t), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t + nt < 2 * W) pre1 = __hip_atomic_load(src_word(t + nt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        if constexpr (IsLfgStrip<Unit>::value) {
            constexpr uint32_t LR = Unit::kR, LS = Unit::kS, RB = Unit::B, RUN = Unit::kRun;
            constexpr uint32_t NR = (1024 + RUN - 1) / RUN;
            const uint32_t n_inst = a.units / 1024;
            const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63, n_waves = nt >> 6;
            constexpr uint32_t kLast = 1024 - (NR - 1) * RUN;
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (n_inst >= n_waves) {
                    // as many instances as waves or more: wave w makes the
                    // runs of instances w, w + waves, ... in turn; a run
                    // reads only earlier runs of its own instance, written
                    // by the same wave, whose LDS accesses complete in order
                    for (uint32_t i = wave; i < n_inst; i += n_waves) {
                        uint32_t *rg = rings + i * RB;
#pragma unroll
                        for (uint32_t rr = 0; rr < NR; ++rr) {
                            const uint32_t len = rr + 1 < NR ? RUN : kLast;
                            const uint32_t v0 = lq + rr * RUN;
                            for (uint32_t j = lane; j < len; j += 64) {
                                const uint32_t v = v0 + j;
                                rg[v & (RB - 1)] = rg[(v - LR) & (RB - 1)] + rg[(v - LS) & (RB - 1)];
                            }
                            __builtin_amdgcn_wave_barrier();
                        }
                    }
                    __syncthreads();
                } else {
#pragma unroll
                    for (uint32_t rr = 0; rr < NR; ++rr) {
                        const uint32_t len = rr + 1 < NR ? RUN : kLast;
                        const uint32_t nblk = (len + 63) / 64;  // 64-value blocks of the run per instance
                        const uint32_t v0 = lq + rr * RUN;
                        // block b = (instance i, block m) goes to wave b mod
                        // (waves): i and m are wave-uniform, lane l makes
                        // value 64 m + l
                        for (uint32_t b = wave; b < n_inst * nblk; b += n_waves) {
                            const uint32_t i = b / nblk, m = b - i * nblk;
                            const uint32_t j = 64 * m + lane;
                            if (j < len) {
                                uint32_t *rg = rings + i * RB;
                                const uint32_t v = v0 + j;
                                rg[v & (RB - 1)] = rg[(v - LR) & (RB - 1)] + rg[(v - LS) & (RB - 1)];
                            }
                        }
                        __syncthreads();
                    }
                }
#pragma unroll
                for (int i = 0; i < SPT; ++i)  // slot i: instance i, stream t (1024 threads)
                    if (t + i * nt < a.units) {
                        const uint32_t val = rings[i * RB + ((lq + t) & (RB - 1))];
                        if (d == 0) u[i].d0 = val;
                        else u[i].d1 = val;
                    }
                if (RB < 2048 && d == 0) __syncthreads();  // row 1 read before row 2 overwrites it
                lq += 1024;
            }
        }
        uint32_t esum = 0;
        const uint32_t zero = *zero_word;
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int i = j == 0 ? SPT - 1 : j - 1;  // bottom-row slot, top-row slot, then the rest
            const uint32_t k = t + i * nt;
            const bool bslot = !early || j <= 1;      // may hold top- or bottom-row units
            if (k < a.units) {
                // `zero` is reloaded from LDS every pass, so the addresses
                // derived from `pl` cannot be hoisted out of the sweep loop
                // and held per unit in registers.
                uint32_t pl;
                if constexpr (PLDS) pl = place_lds[i * nt + t];
                else pl = place[i] + zero;
                const bool top = bslot && ((pl >> 27) & 1), bot = bslot && ((pl >> 28) & 1);
                const uint64_t nw = update_unit<Unit, E, MH>(lds, pl, P, top ? up_add : 0u, bot ? dn_add : 0u, c, u[i], A, esum,
                                                                   a.hits, a, sweep);
                const uint32_t off = pl & kOffMask;
                const uint32_t yrow = top ? 1 : bot ? R : 0;   // only used for boundary units
                const uint32_t x0 = off - kPad - yrow * P;
                if ((pl >> 29) & 3) edge_ghosts<NB>(lds + off, pl, L, nw);
                if (top || bot) {
                    if (nwg > 1) {
                        uint64_t *dst = mine + (bot ? W : 0) + x0 / 4;
                        put_word(dst, static_cast<uint32_t>(nw), tag);
                        if constexpr (NB == 8) put_word(dst + 1, static_cast<uint32_t>(nw >> 32), tag);
                    } else {
                        // periodic in y: the top row is the row below the bottom row
                        uint8_t *row = lds + (top ? h_dn[nxt] : h_up[nxt]);
                        lds_put<NB>(row + x0, nw);
                        if ((pl >> 29) & 3) edge_ghosts<NB>(row + x0, pl, L, nw);
                    }
                }
            }
            // keep units apart: only the held states stay live across units
            __builtin_amdgcn_sched_barrier(0);
            if (nwg > 1 && early && j == kPullAt) request();
        }
        if (nwg > 1) {
            if (!early) request();
            // the neighbours' pass-q words into buffer nxt, with ghosts
            for (uint32_t i = t, m = 0; i < 2 * W; i += nt, ++m) {
                const uint64_t *sp = src_word(i);
                const uint64_t v0 = m == 0 ? pre0 : m == 1 ? pre1 : __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t v = poll_word(sp, v0, tag, a.err);
                const uint32_t wi = i < W ? i : i - W;
                uint8_t *row = lds + (i < W ? h_up[nxt] : h_dn[nxt]);
                *reinterpret_cast<uint32_t *>(row + 4 * wi) = v;
                if (wi == 0) *reinterpret_cast<uint32_t *>(row + L) = v;
                if (wi == W - 1) *reinterpret_cast<uint32_t *>(row - 4) = v;
            }
        }
        if constexpr (E) {
            // each colour-1 site adds s*h = 4 - (doubled count after the step)
            int v = static_cast<int>(2 * NB * my_units) - static_cast<int>(esum);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if ((t & 63) == 0) wave_e[t >> 6] = v;
        }
        ++q;
    };

    // Colour 1 always accumulates the energy terms (they are only reduced
    // when a trace is asked for): a single colour-1 body keeps the register
    // assignment of the unit states the same on every path through the loop,
    // which a traced/untraced branch here would not.
    for (uint64_t sweep = 0; sweep < a.n_sweeps; ++sweep) {
        pass(std::false_type{}, 0, sweep);
        pass(std::true_type{}, 1, sweep);
    }
    __syncthreads();
    if (a.n_sweeps > 0) flush_energy(a.n_sweeps - 1);

    // write back spins and state
    copy_strip<false>(lds + P + kPad, a.spins + row0 * L, L, R, t, nt);
    if constexpr (IsLfgStrip<Unit>::value) {  // the last r values of every instance
        constexpr uint32_t LR = Unit::kR, RB = Unit::B;
        const uint32_t n_inst = a.units / 1024;
        uint32_t *X = reinterpret_cast<uint32_t *>(a.st) + (ubase / 1024) * LR;
        for (uint32_t idx = t; idx < n_inst * LR; idx += nt) {
            const uint32_t i = idx / LR, j = idx - i * LR;
            X[idx] = rings[i * RB + ((lq - LR + j) & (RB - 1))];
        }
    }
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
        const uint32_t k = t + i * nt;
        if (k < a.units) {
            if constexpr (SweepCounter<Unit>::value) u[i].store_at(a.st, a.S, ubase + k, a);
            else u[i].store(a.st, a.S, ubase + k, 4 * a.n_sweeps * (MH ? a.hits : 1));
        }
    }
}

// Whether every stream of strip r stands at the same position, a multiple of
// 4 (Philox): then *blk0 is that position's block.
__device__ inline bool strip_positions_aligned(const StripArgs &a, uint32_t r, uint64_t *blk0) {
    const uint64_t ubase = static_cast<uint64_t>(r) * a.R0 * (a.L / 4);
    const uint64_t *pos = reinterpret_cast<const uint64_t *>(a.st + 8 * a.S) + ubase;
    const uint64_t p0 = pos[0];
    int ok = (p0 & 3) == 0;
    for (uint32_t k = threadIdx.x; k < a.units; k += blockDim.x) ok &= pos[k] == p0;
    *blk0 = p0 >> 2;
    return __syncthreads_and(ok) != 0;
}

// Whether every XS1024W instance with a unit in strip r has taken the same
// number of steps: then *n0 is that count and *y_start the common Weyl word.
__device__ inline bool strip_steps_uniform(const StripArgs &a, uint32_t r, uint64_t *n0, uint32_t *y_start) {
    const uint64_t ubase = static_cast<uint64_t>(r) * a.R0 * (a.L / 8);
    const uint64_t *N = reinterpret_cast<const uint64_t *>(a.st + 4 * a.S);
    const uint64_t g0 = ubase >> 4, g1 = (ubase + a.units - 1) >> 4;
    const uint64_t n = N[g0];
    int ok = 1;
    for (uint64_t g = g0 + threadIdx.x; g <= g1; g += blockDim.x) ok &= N[g] == n;
    *n0 = n;
    *y_start = *reinterpret_cast<const uint32_t *>(a.st + 4 * a.S + 8 * (a.S / 32)) + static_cast<uint32_t>(n) * kWeylC;
    return __syncthreads_and(ok) != 0;
}

// EARLY: the strip's top row lies in slot 0 and its bottom row in slot SPT-1.
template <int SPT>
__host__ __device__ constexpr bool early_slots(uint32_t upr, uint32_t units, uint32_t nt) {
    return SPT > 2 && upr <= nt && units - upr >= (SPT - 1) * nt;
}

template <class Unit, int SPT, bool EARLY, bool MH>
__global__ __launch_bounds__(1024) void k_ising_strip(StripArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    // Blocks b, b+8, b+16, ... share an XCD: give them consecutive strips so
    // that most neighbour exchanges stay inside one L2.
    const uint32_t b = blockIdx.x, nwg = a.nwg;
    const uint32_t r = (nwg % 8 == 0) ? (b % 8) * (nwg / 8) + b / 8 : b;
    if (early_slots<SPT>(a.L / Unit::kNB, a.units, blockDim.x) != EARLY) {  // plan and kernel disagree
        if (threadIdx.x == 0) __hip_atomic_fetch_or(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    using Sweep = typename SweepOf<Unit>::type;
    if constexpr (!std::is_void<Sweep>::value && !MH) {
        static_assert(place_in_lds<Sweep, SPT>() == place_in_lds<Unit, SPT>(), "the two forms share the LDS plan");
        StripArgs b2 = a;
        bool uniform;
        if constexpr (std::is_same<Unit, XsUnit>::value) uniform = strip_steps_uniform(a, r, &b2.blk0, &b2.y_start);
        else uniform = strip_positions_aligned(a, r, &b2.blk0);
        if (uniform) {
            strip_body<Sweep, SPT, EARLY, place_in_lds<Sweep, SPT>(), false>(b2, r, lds);
            return;
        }
    }
    strip_body<Unit, SPT, EARLY, place_in_lds<Unit, SPT>(), MH>(a, r, lds);
}

// ---------------------------------------------------------------- per pass
struct PassArgs {
    int8_t *spins;
    uint8_t *st;
    uint64_t S;
    uint32_t L;
    int c;
    uint64_t T4, T8;
    int32_t *partial;  // one per block, or null
    uint32_t hits;     // multi-hit kernels only
};

// Update unit k of colour c with spins and state in global memory; returns
// the sum of s*h over the updated sites.  A unit reads only other-colour
// bytes of its neighbour runs, which no thread writes during the pass.
template <class Unit, bool MH = false>
__device__ __forceinline__ int unit_in_memory_with(Unit &u, uint8_t *sp, uint8_t *st, uint64_t S, uint32_t L,
                                                   uint64_t k, int c, uint64_t T4, uint64_t T8, uint32_t hits);

template <class Unit, bool MH = false>
__device__ __forceinline__ int unit_in_memory(uint8_t *sp, uint8_t *st, uint64_t S, uint32_t L, uint64_t k, int c,
                                              uint64_t T4, uint64_t T8, uint32_t hits = 1) {
    Unit u;
    u.load(st, S, k);
    return unit_in_memory_with<Unit, MH>(u, sp, st, S, L, k, c, T4, T8, hits);
}

// The update with the unit's generator already loaded (it stores it back).
template <class Unit, bool MH>
__device__ __forceinline__ int unit_in_memory_with(Unit &u, uint8_t *sp, uint8_t *st, uint64_t S, uint32_t L,
                                                   uint64_t k, int c, uint64_t T4, uint64_t T8, uint32_t hits) {
    constexpr int NB = Unit::kNB;
    // L <= 16384: unit indices and site offsets fit 32 bits (no 64-bit division)
    const uint32_t upr = L / NB, k32 = static_cast<uint32_t>(k);
    const uint32_t y = k32 / upr;
    const uint32_t x0 = (k32 - y * upr) * NB;
    const uint32_t row = y * L, up_row = (y == 0 ? L - 1 : y - 1) * L;
    const uint32_t dn_row = (y == L - 1 ? 0 : y + 1) * L;
    uint64_t w = lds_run<NB>(sp + row + x0);
    const uint64_t upw = lds_run<NB>(sp + up_row + x0), dnw = lds_run<NB>(sp + dn_row + x0);
    const uint32_t lb = sp[row + (x0 == 0 ? L - 1 : x0 - 1)];
    const uint32_t rb = sp[row + (x0 + NB == L ? 0 : x0 + NB)];
    const uint64_t m = mismatches<NB>(w, upw, dnw, lb, rb);
    const int p = static_cast<int>((c + y) & 1);
    int sh = 0;
    if constexpr (MH) {
        // byte p + 2h is site h; the same draw order as the on-chip update
        uint32_t mi[NB / 2], fl[NB / 2];
#pragma unroll
        for (int h = 0; h < NB / 2; ++h) {
            mi[h] = static_cast<uint32_t>(m >> (8 * (p + 2 * h))) & 0xFFu;
            fl[h] = 0;
        }
        if constexpr (NB == 4) {
            u.draws2(hits, [&](uint32_t r) { hit_mem(mi[0], fl[0], r, T4, T8); },
                     [&](uint32_t r) { hit_mem(mi[1], fl[1], r, T4, T8); });
        } else {
            for (uint32_t i = 0; i < hits; ++i) {
                uint32_t ra, rb;
                u.pair(ra, rb);
                hit_mem(mi[0], fl[0], ra, T4, T8);
                hit_mem(mi[2], fl[2], rb, T4, T8);
            }
            for (uint32_t i = 0; i < hits; ++i) {
                uint32_t ra, rb;
                u.pair(ra, rb);
                hit_mem(mi[1], fl[1], ra, T4, T8);
                hit_mem(mi[3], fl[3], rb, T4, T8);
            }
        }
        u.store(st, S, k, 2 * hits);
#pragma unroll
        for (int h = 0; h < NB / 2; ++h) {
            w ^= static_cast<uint64_t>(fl[h] * 0xFEu) << (8 * (p + 2 * h));
            sh += 4 - 2 * static_cast<int>(mi[h]);
        }
    } else {
        uint32_t rr[NB / 2];
        u.draw(rr);
        u.store(st, S, k, 2);
#pragma unroll
        for (int h = 0; h < NB / 2; ++h) sh += metropolis(w, m, p + 2 * h, rr[h], T4, T8);
    }
    lds_put<NB>(sp + row + x0, w);
    return sh;
}

template <class Unit, bool MH>
__global__ __launch_bounds__(kBlock) void k_ising_pass(PassArgs a, uint64_t n_units) {
    const uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int sh = 0;
    if (k < n_units)  // XS1024W: n_units is a multiple of 16, so rows stay whole
        sh = unit_in_memory<Unit, MH>(reinterpret_cast<uint8_t *>(a.spins), a.st, a.S, a.L, k, a.c, a.T4, a.T8,
                                      a.hits);
    if (a.partial) {
        __shared__ int red[kBlock / 64];
        const int tot = block_sum(sh, red);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = tot;
    }
}

// ---------------------------------------------------------------- lagged Fibonacci
// A lagged Fibonacci instance is shared by 1024 streams, i.e. 1024
// consecutive units (L a multiple of 64), so a lattice is swept one launch
// per colour pass with one 1024-thread workgroup per instance: it loads the
// instance's last r values into an LDS ring, and each draw of the pass is a
// row of 1024 new values made by the whole workgroup (runs of at most s
// values, one barrier each; thread i then takes value i of the row), after
// which the window goes back to memory.  Every thread has a unit, so all
// reach each row's barriers together.
template <int R, int SL>
struct LfgPassUnit {
    static constexpr int kNB = 4;
    static constexpr uint32_t B = R + 1024 <= 2048 ? 2048 : 4096;  // a row plus the r values before it
    uint32_t *ring;  // LDS: value q at ring[q mod B]
    uint32_t q;      // index of the next row's first value
    __device__ void load(const uint8_t *, uint64_t, uint64_t) {}
    __device__ void store(uint8_t *, uint64_t, uint64_t, uint64_t) const {}
    __device__ uint32_t next() {
        const uint32_t t = threadIdx.x;
        for (uint32_t b = 0; b < 1024; b += SL) {
            const uint32_t len = min(static_cast<uint32_t>(SL), 1024 - b);
            const uint32_t qq = q + b + t;
            if (t < len) ring[qq & (B - 1)] = ring[(qq - R) & (B - 1)] + ring[(qq - SL) & (B - 1)];
            __syncthreads();
        }
        const uint32_t v = ring[(q + t) & (B - 1)];
        q += 1024;
        return v;
    }
    __device__ void draw(uint32_t (&r)[2]) { r[0] = next(); r[1] = next(); }
    template <class F0, class F1>
    __device__ void draws2(uint32_t n, F0 &&f0, F1 &&f1) {
        for (uint32_t i = 0; i < n; ++i) f0(next());
        for (uint32_t i = 0; i < n; ++i) f1(next());
    }
};

template <int R, int SL, bool MH>
__global__ __launch_bounds__(1024) void k_ising_pass_lfg(PassArgs a) {
    using U = LfgPassUnit<R, SL>;
    __shared__ uint32_t ring[U::B];
    __shared__ int red[16];
    uint32_t *X = reinterpret_cast<uint32_t *>(a.st) + static_cast<uint64_t>(blockIdx.x) * R;
    for (uint32_t j = threadIdx.x; j < R; j += blockDim.x) ring[U::B - R + j] = X[j];
    __syncthreads();
    U u{ring, 0};
    const uint64_t k = static_cast<uint64_t>(blockIdx.x) * 1024 + threadIdx.x;
    const int sh = unit_in_memory_with<U, MH>(u, reinterpret_cast<uint8_t *>(a.spins), a.st, a.S, a.L, k, a.c,
                                              a.T4, a.T8, a.hits);
    // the last row's barrier has passed and no thread writes the ring again
    for (uint32_t j = threadIdx.x; j < R; j += blockDim.x) X[j] = ring[(u.q - R + j) & (U::B - 1)];
    if (a.partial) {
        const int tot = block_sum(sh, red);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = tot;
    }
}

// Single-hit passes with T < 1024 threads per instance, U = 1024 / T units
// per thread (unit j of the instance on thread j mod T): every workgroup is a
// chain of dependent steps (window and spin loads, a barrier per run of new
// values, stores) whose latency one 1024-thread workgroup per SIMD pair
// cannot hide; smaller workgroups put several instances on each CU.  The
// units' spin words are loaded before the window so that both loads are in
// flight together, and each row is made in runs of at most s values as in
// LfgPassUnit.  Same draws, spins and energies as k_ising_pass_lfg.
template <int R, int SL, int T>
__global__ __launch_bounds__(T) void k_ising_pass_lfg_n(PassArgs a) {
    constexpr int U = 1024 / T;
    constexpr uint32_t B = LfgPassUnit<R, SL>::B;
    __shared__ uint32_t ring[B];
    __shared__ int red[T / 64];
    const uint32_t t = threadIdx.x, L = a.L, upr = L / 4;
    uint8_t *sp = reinterpret_cast<uint8_t *>(a.spins);
    uint64_t w[U], m[U];
    uint32_t at[U];
    int p[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
        // L <= 16384: unit indices and site offsets fit 32 bits
        const uint32_t k = blockIdx.x * 1024 + t + i * T;
        const uint32_t y = k / upr;
        const uint32_t x0 = (k - y * upr) * 4;
        const uint32_t row = y * L, up_row = (y == 0 ? L - 1 : y - 1) * L;
        const uint32_t dn_row = (y == L - 1 ? 0 : y + 1) * L;
        w[i] = lds_run<4>(sp + row + x0);
        const uint64_t upw = lds_run<4>(sp + up_row + x0), dnw = lds_run<4>(sp + dn_row + x0);
        const uint32_t lb = sp[row + (x0 == 0 ? L - 1 : x0 - 1)];
        const uint32_t rb = sp[row + (x0 + 4 == L ? 0 : x0 + 4)];
        m[i] = mismatches<4>(w[i], upw, dnw, lb, rb);
        p[i] = static_cast<int>((a.c + y) & 1);
        at[i] = row + x0;
    }
    uint32_t *X = reinterpret_cast<uint32_t *>(a.st) + static_cast<uint64_t>(blockIdx.x) * R;
    for (uint32_t j = t; j < R; j += T) ring[B - R + j] = X[j];
    __syncthreads();
    // the pass's two rows: value j of row d is draw d of unit j
    uint32_t r[U][2];
    uint32_t q = 0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        for (uint32_t b = 0; b < 1024; b += SL) {
            const uint32_t len = min(static_cast<uint32_t>(SL), 1024 - b);
            for (uint32_t j = t; j < len; j += T) {
                const uint32_t qq = q + b + j;
                ring[qq & (B - 1)] = ring[(qq - R) & (B - 1)] + ring[(qq - SL) & (B - 1)];
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < U; ++i) r[i][d] = ring[(q + t + i * T) & (B - 1)];
        q += 1024;
    }
    int sh = 0;
#pragma unroll
    for (int i = 0; i < U; ++i) {
        sh += metropolis(w[i], m[i], p[i], r[i][0], a.T4, a.T8);
        sh += metropolis(w[i], m[i], p[i] + 2, r[i][1], a.T4, a.T8);
        lds_put<4>(sp + at[i], w[i]);
    }
    // the second row's barrier has passed and no thread writes the ring again
    for (uint32_t j = t; j < R; j += T) X[j] = ring[(q - R + j) & (B - 1)];
    if (a.partial) {
        const int tot = block_sum(sh, red);
        if (t == 0) a.partial[blockIdx.x] = tot;
    }
}

// L = 64: the lattice is one instance, so one workgroup runs every sweep of
// the call in one launch, the window staying in LDS throughout; the spins
// stay in memory and a barrier separates the passes.
template <int R, int SL, bool MH>
__global__ __launch_bounds__(1024) void k_ising_lfg_one(PassArgs a, uint64_t n_sweeps, int32_t *trace) {
    using U = LfgPassUnit<R, SL>;
    __shared__ uint32_t ring[U::B];
    __shared__ int red[16];
    uint32_t *X = reinterpret_cast<uint32_t *>(a.st);
    for (uint32_t j = threadIdx.x; j < R; j += blockDim.x) ring[U::B - R + j] = X[j];
    __syncthreads();
    U u{ring, 0};
    uint8_t *sp = reinterpret_cast<uint8_t *>(a.spins);
    for (uint64_t t = 0; t < n_sweeps; ++t) {
        int sh = 0;
        for (int c = 0; c < 2; ++c) {
            sh = unit_in_memory_with<U, MH>(u, sp, a.st, a.S, a.L, threadIdx.x, c, a.T4, a.T8, a.hits);
            __syncthreads();  // this pass's spins before the next pass reads them
        }
        if (trace) {
            const int tot = block_sum(sh, red);
            if (threadIdx.x == 0) trace[t] = -tot;
        }
    }
    for (uint32_t j = threadIdx.x; j < R; j += blockDim.x) X[j] = ring[(u.q - R + j) & (U::B - 1)];
}

// ---------------------------------------------------------------- batches
// A batch is a fixed list of replicas (same kind) swept in one launch: each
// workgroup takes the next replica from a counter (replicas ordered by
// decreasing work) and runs all its sweeps alone -- on chip when the
// lattice fits, otherwise streaming it through memory -- so no workgroup
// ever waits for another.
template <class Unit>
__device__ void replica_in_memory(const ReplicaDesc &d, int *red) {
    constexpr int NB = Unit::kNB;
    const uint64_t n_units = static_cast<uint64_t>(d.L) * d.L / NB;
    uint8_t *sp = reinterpret_cast<uint8_t *>(d.spins);
    for (uint64_t sweep = 0; sweep < d.n_sweeps; ++sweep) {
        for (int c = 0; c < 2; ++c) {
            int sh = 0;
            // XS1024W: n_units and blockDim are multiples of 16, rows stay whole
            for (uint64_t k = threadIdx.x; k < n_units; k += blockDim.x)
                sh += unit_in_memory<Unit>(sp, d.st, d.S, d.L, k, c, d.T4, d.T8);
            __syncthreads();
            if (c == 1 && d.trace) {
                const int tot = block_sum(sh, red);
                if (threadIdx.x == 0) d.trace[sweep] = -tot;
            }
        }
    }
}

// A gang's strips wait on each other every pass, so none of them may start
// its sweeps before all of them run.  Items are claimed one at a time, so the
// first strips of a gang can be claimed long before the last ones (the other
// workgroups may be busy with long independent items): each member checks in
// and waits here, bounded by wall-clock time rather than a poll count, until
// all nwg have arrived.  They always do, as every other claimed item finishes
// on its own and frees its workgroup for the gang's next strip; if the bound
// is reached anyway (the device held by other work for that long), the
// lattice is marked invalid and its strips end quickly.
__device__ void gang_start(const ReplicaDesc &d) {
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(d.gang, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = static_cast<uint64_t>(wall_clock64());
        while (__hip_atomic_load(d.gang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < d.nwg) {
            if (static_cast<uint64_t>(wall_clock64()) - t0 > d.start_ticks || __hip_atomic_load(d.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_fetch_or(d.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(127);
        }
    }
    __syncthreads();
}

// Units per thread of an on-chip replica (at most 16384 four-site or 8192
// eight-site units, i.e. L <= 256, with 1024 threads).
template <class Unit>
constexpr int batch_spt() { return Unit::kNB == 8 ? 8 : 16; }

// Work items are (replica, strip) pairs; a gang's strips are consecutive in
// the list, which the workgroups take in order from a counter.  Every
// workgroup of the launch is resident, so when a strip waits for a neighbour
// that neighbour is either running or will be taken by the next workgroup to
// finish its (independent) item; gangs are far smaller than the grid.
// MAXT: the most threads per workgroup the instantiation is compiled for
// (1024 caps a thread at 128 VGPRs, 512 at 256, so fewer spills).
template <class Unit, int MAXT>
__global__ __launch_bounds__(MAXT) void k_ising_batch(const ReplicaDesc *reps, const uint2 *items, uint32_t n_items,
                                                     uint32_t *next) {
    constexpr int NB = Unit::kNB;
    constexpr int spt = batch_spt<Unit>();
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t idx_s;
    __shared__ int red_s[16];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) idx_s = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t idx = idx_s;
        if (idx >= n_items) break;  // every workgroup leaves once the list is drained
        const uint2 item = items[idx];
        const ReplicaDesc d = reps[item.x];
        if (d.mode == kReplicaMemory) {
            replica_in_memory<Unit>(d, red_s);
            continue;
        }
        if (d.mode == kReplicaStrips) gang_start(d);
        const uint32_t R = item.y + 1 == d.nwg ? d.R_last : d.R;
        const uint32_t units = R * (d.L / NB);
        const StripArgs a{d.spins, d.st, d.S, d.L, R, d.nwg, units, d.T4, d.T8, d.n_sweeps, d.trace,
                          d.halo, 0, d.err, 1, d.R};
        if (early_slots<spt>(d.L / NB, units, blockDim.x)) strip_body<Unit, spt, true, false>(a, item.y, lds);
        else strip_body<Unit, spt, false, false>(a, item.y, lds);
    }
}

// Before each batch run: the work counter, and for every gang its halo
// tags (so that the pass tags can restart at 1 on every run, also on graph
// replays) and its energy trace (strips add their parts).  Block i: replica i.
__global__ __launch_bounds__(kBlock) void k_batch_prologue(const ReplicaDesc *reps, uint32_t *next) {
    const ReplicaDesc d = reps[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) *next = 0;
    if (d.mode != kReplicaStrips) return;
    uint32_t *h = reinterpret_cast<uint32_t *>(d.halo);
    const uint64_t words = 2ull * d.nwg * d.L;
    for (uint64_t i = threadIdx.x; i < words; i += kBlock) h[i] = 0;
    if (threadIdx.x == 0) *d.gang = 0;
    if (d.trace)
        for (uint64_t i = threadIdx.x; i < d.n_sweeps; i += kBlock) d.trace[i] = 0;
}

// trace[t] = -(sum of n partials); one block, deterministic order.
__global__ __launch_bounds__(1024) void k_reduce_partials(const int32_t *partial, uint64_t n, int32_t *out) {
    __shared__ int red[16];
    int s = 0;
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
    const int tot = block_sum(s, red);
    if (threadIdx.x == 0) *out = -tot;
}

// ---------------------------------------------------------------- host side
constexpr uint32_t kLdsMax = 160 * 1024;
constexpr uint32_t kMaxThreads = 1024;

template <class Unit, int SPT, bool EARLY, bool MH>
const void *strip_kernel() { return reinterpret_cast<const void *>(&k_ising_strip<Unit, SPT, EARLY, MH>); }

template <class Unit, bool MH = false>
const void *strip_kernel_for(int spt, bool early) {
    switch (spt) {
    case 1: return strip_kernel<Unit, 1, false, MH>();
    case 2: return strip_kernel<Unit, 2, false, MH>();
    case 4: return early ? strip_kernel<Unit, 4, true, MH>() : strip_kernel<Unit, 4, false, MH>();
    case 8: return early ? strip_kernel<Unit, 8, true, MH>() : strip_kernel<Unit, 8, false, MH>();
    case 16: return early ? strip_kernel<Unit, 16, true, MH>() : strip_kernel<Unit, 16, false, MH>();
    }
    return nullptr;
}

template <class Unit>
bool place_lds_for(int spt) {
    switch (spt) {
    case 1: return place_in_lds<Unit, 1>();
    case 2: return place_in_lds<Unit, 2>();
    case 4: return place_in_lds<Unit, 4>();
    case 8: return place_in_lds<Unit, 8>();
    case 16: return place_in_lds<Unit, 16>();
    }
    return false;
}

// Host twin of early_slots for a run-time SPT.
inline bool plan_early(int spt, uint32_t upr, uint32_t units, uint32_t nt) {
    switch (spt) {
    case 4: return early_slots<4>(upr, units, nt);
    case 8: return early_slots<8>(upr, units, nt);
    case 16: return early_slots<16>(upr, units, nt);
    }
    return false;
}

template <class Unit, bool MH>
hipError_t run_passes(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st, uint32_t hits) {
    constexpr int NB = Unit::kNB;
    const uint64_t L = lat->L, n_units = L * L / NB;
    const unsigned blocks = static_cast<unsigned>((n_units + kBlock - 1) / kBlock);
    PassArgs pa{lat->d_spins, lat->gen->d_state, lat->gen->S, lat->L, 0, T4, T8, nullptr, hits};
    for (uint64_t t = 0; t < n; ++t) {
        for (int c = 0; c < 2; ++c) {
            pa.c = c;
            pa.partial = (c == 1 && tr) ? lat->d_partial : nullptr;
            hipLaunchKernelGGL((k_ising_pass<Unit, MH>), dim3(blocks), dim3(kBlock), 0, st, pa, n_units);
        }
        if (tr) hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, st, lat->d_partial,
                                   static_cast<uint64_t>(blocks), tr + t);
    }
    return hipGetLastError();
}

template <class Unit, bool MH>
hipError_t run_strips(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st, uint32_t hits) {
    const IsingPlan &pl = lat->plan;
    const void *fn = strip_kernel_for<Unit, MH>(pl.spt, pl.early);
    if (MH) {
        // The plan was sized with the single-hit kernel: give this one the
        // same LDS and check that every strip can still be resident.
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(pl.lds));
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, static_cast<int>(pl.threads), pl.lds) != hipSuccess ||
            static_cast<uint64_t>(occ) * lat->gen->n_cu < pl.nwg) {
            (void)hipGetLastError();
            return run_passes<Unit, MH>(lat, T4, T8, n, tr, st, hits);
        }
    }
    if (tr && pl.nwg > 1) {
        hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint32_t *>(tr), n);
    }
    if (pl.nwg > 1 && lat->epoch + 2 * n + 2 >= (1ull << 31)) {  // restart the pass tags before they wrap
        const uint64_t words = 2ull * pl.nwg * lat->L;              // halo size in uint32
        hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<unsigned>((words + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint32_t *>(lat->d_halo), words);
        lat->epoch = 0;
    }
    StripArgs a{lat->d_spins, lat->gen->d_state, lat->gen->S, lat->L, pl.R, pl.nwg, pl.units, T4, T8, n,
                tr, lat->d_halo, static_cast<uint32_t>(lat->epoch), lat->d_err, hits, pl.R};
    void *args[] = {&a};
    hipError_t e;
    if (pl.nwg == 1)
        e = hipLaunchKernel(fn, dim3(1), dim3(pl.threads), args, pl.lds, st);
    else
        e = hipLaunchCooperativeKernel(fn, dim3(pl.nwg), dim3(pl.threads), args, pl.lds, st);
    if (e != hipSuccess) return e;
    lat->epoch += 2 * n;
    return hipGetLastError();
}

// Try one decomposition into nwg strips; fills *out if it fits on chip.
template <class Unit>
bool try_strips(uint32_t L, uint32_t nwg, int max_spt, int n_cu, IsingPlan *out) {
    constexpr uint32_t NB = Unit::kNB;
    if (nwg == 0 || L % nwg) return false;
    const uint32_t R = L / nwg;
    if (R < 2) return false;  // a strip's top and bottom rows are distinct
    uint64_t lds = strip_lds_bytes(L, R);
    if (lds > kLdsMax) return false;
    const uint64_t sites = static_cast<uint64_t>(R) * L;
    if (NB == 8 && sites % 128) return false;  // whole XS1024W instances per strip
    const uint32_t units = static_cast<uint32_t>(sites / NB);
    int spt = 1;
    while (spt <= max_spt && (units + spt - 1) / spt > kMaxThreads) spt *= 2;
    if (spt > max_spt) return false;
    // The fewest units per thread that fit; if the strips are then not all
    // resident (more strips than CUs), more units per thread and fewer
    // threads per strip put several strips on each CU.
    for (; spt <= max_spt; spt *= 2) {
        uint32_t threads = (units + spt - 1) / spt;
        threads = (threads + 63) / 64 * 64;
        uint64_t b = lds;
        if constexpr (IsLfgStrip<Unit>::value) {  // whole instances, slot i = instance i on 1024 threads
            if (units % 1024 || threads != 1024 || static_cast<uint32_t>(spt) * 1024 != units) return false;
            b = (b + 15) / 16 * 16 + lfg_ring_bytes<Unit>(units);
        }
        const bool early = plan_early(spt, L / NB, units, threads);
        if (place_lds_for<Unit>(spt)) b += 4ull * spt * threads;
        if (b > kLdsMax) return false;
        const void *fn = strip_kernel_for<Unit>(spt, early);
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(b));
        (void)hipGetLastError();
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, static_cast<int>(threads), b) != hipSuccess ||
            occ < 1) {
            (void)hipGetLastError();
            return false;
        }
        if (static_cast<uint64_t>(occ) * n_cu >= nwg) {
            *out = IsingPlan{true, R, nwg, units, static_cast<uint32_t>(spt), threads, static_cast<uint32_t>(b), early};
            return true;
        }
    }
    return false;
}

// Lattices up to 256 x 256 run in one workgroup (barriers stay inside the
// CU).  Larger ones take the most strips (at most one per CU) that still
// leave each strip >= 2048 sites, else the fewest strips that fit.
template <class Unit>
bool plan_strips(uint32_t L, int max_spt, int n_cu, IsingPlan *out) {
    *out = IsingPlan{};
    if (n_cu < 1) return false;
    if (L <= 256 && try_strips<Unit>(L, 1, max_spt, n_cu, out)) return true;
    const uint32_t top = std::min<uint32_t>(L, static_cast<uint32_t>(n_cu));
    for (uint32_t nwg = top; nwg >= 1; --nwg)
        if (static_cast<uint64_t>(L / nwg) * L >= 2048 && try_strips<Unit>(L, nwg, max_spt, n_cu, out)) return true;
    for (uint32_t nwg = 1; nwg <= top; ++nwg)
        if (try_strips<Unit>(L, nwg, max_spt, n_cu, out)) return true;
    *out = IsingPlan{};
    return false;
}

template <class Unit>
hipError_t run(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st, uint32_t hits) {
    if (hits == 1) {
        if (lat->plan.strips) return run_strips<Unit, false>(lat, T4, T8, n, tr, st, 1);
        return run_passes<Unit, false>(lat, T4, T8, n, tr, st, 1);
    }
    if (lat->plan.strips) return run_strips<Unit, true>(lat, T4, T8, n, tr, st, hits);
    return run_passes<Unit, true>(lat, T4, T8, n, tr, st, hits);
}

constexpr uint32_t kMaxGang = 64;             // most strips of one batch replica
constexpr uint64_t kGangWordBytes = 64;       // a gang's arrival counter, after its halo words
constexpr double kGangStartSeconds = 60.0;    // longest wait of a gang member for the others to start

template <class Unit>
const void *batch_kernel(uint32_t threads) {
    if (threads > 512) return reinterpret_cast<const void *>(&k_ising_batch<Unit, 1024>);
    return reinterpret_cast<const void *>(&k_ising_batch<Unit, 512>);
}

const void *batch_kernel_for(rngx_kind kind, uint32_t threads) {
    switch (kind) {
    case RNGX_LCG32: return batch_kernel<SmallUnit<Lcg32>>(threads);
    case RNGX_LCG32_SUB: return batch_kernel<SmallUnit<Lcg32Sub>>(threads);
    case RNGX_LCG64: return batch_kernel<SmallUnit<Lcg64>>(threads);
    case RNGX_LCG64_SUB: return batch_kernel<SmallUnit<Lcg64Sub>>(threads);
    case RNGX_MWC: return batch_kernel<SmallUnit<Mwc>>(threads);
    case RNGX_MWC_DIFF: return batch_kernel<SmallUnit<MwcDiff>>(threads);
    case RNGX_XORWOW: return batch_kernel<SmallUnit<Xorwow>>(threads);
    case RNGX_PHILOX4X32_10: return batch_kernel<PhiloxUnit>(threads);
    case RNGX_PHILOX4X32_7: return batch_kernel<PhiloxUnit7>(threads);
    case RNGX_XS1024W: return batch_kernel<XsUnit>(threads);
    default: break;  // lagged Fibonacci lattices are not batched
    }
    return nullptr;
}

uint64_t threshold(double beta, int dE) {
    return static_cast<uint64_t>(std::floor(std::exp(-beta * dE) * 4294967296.0));
}

}  // namespace

const BatchShape kBatchShape[kBatchShapes] = {
    {1024, 64, 80 * 1024},  // the default: fewest strips, two strip workgroups' LDS per CU
    {1024, 32, 80 * 1024},  // half the sites per workgroup: twice the strips per replica
    {512, 64, 80 * 1024},
    {512, 32, 40 * 1024},
    {256, 64, 40 * 1024},   // small workgroups for many small replicas
};

void batch_release(IsingBatch *b) {
    (void)hipFree(b->d_reps);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_next);
    (void)hipFree(b->d_halo);
    b->d_reps = b->d_items = b->d_halo = nullptr;
    b->d_next = nullptr;
    b->n_items = b->grid = b->resident = b->lds = 0;
    b->gangs = false;
}

hipError_t batch_prepare(IsingBatch *b, const uint64_t *sweeps, bool with_traces) {
    batch_release(b);
    const uint32_t n = b->n;
    const BatchShape &sh = kBatchShape[b->shape];
    const uint32_t nb = b->kind == RNGX_XS1024W ? 8 : 4;
    const uint64_t max_units = static_cast<uint64_t>(sh.sites_per_thread) * sh.threads / nb;
    std::vector<ReplicaDesc> reps(n);
    uint32_t lds = 80;
    uint64_t halo_bytes = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const Ising *l = b->lats[i];
        const uint32_t L = l->L;
        int32_t *tr = with_traces ? b->traces[i] : nullptr;
        ReplicaDesc d{l->d_spins, l->gen->d_state, l->gen->S, L, kReplicaMemory, threshold(b->betas[i], 4),
                      threshold(b->betas[i], 8), sweeps[i], tr, 0, 0, 0, nullptr, l->d_err};
        // Fewest strips (one if possible) that fit the workgroup's LDS and
        // unit slots: strips of R rows and a last one of R_last = L - (nwg-1) R
        // rows (2 <= R_last <= R), so that L need not be a multiple of R.
        // XS1024W strips hold whole instances (128 sites), so R is a multiple
        // of g = 128 / gcd(L, 128) (L is a multiple of 16, hence of g).
        const uint32_t g = nb == 8 ? 128u / std::gcd(L, 128u) : 1u;
        for (uint32_t want = 1; want <= kMaxGang; ++want) {
            uint32_t R = (L + want - 1) / want;
            R = std::min((R + g - 1) / g * g, L);
            const uint32_t nwg = (L + R - 1) / R;
            const uint32_t R_last = L - (nwg - 1) * R;
            if (nwg > 1 && R_last < 2) continue;  // a strip's top and bottom rows are distinct
            const uint64_t units = static_cast<uint64_t>(R) * L / nb;
            if (units > max_units || strip_lds_bytes(L, R) > sh.lds_cap) continue;
            if (nb == 8 && ((static_cast<uint64_t>(R) * L) % 128 || (static_cast<uint64_t>(R_last) * L) % 128))
                continue;
            d.mode = nwg == 1 ? kReplicaOnChip : kReplicaStrips;
            d.R = R;
            d.R_last = R_last;
            d.nwg = nwg;
            d.units = static_cast<uint32_t>(units);
            lds = std::max<uint32_t>(lds, static_cast<uint32_t>(strip_lds_bytes(L, R)));
            if (nwg > 1) halo_bytes += 8ull * nwg * L + kGangWordBytes;
            break;
        }
        reps[i] = d;
    }
    // items: replicas by decreasing work per item, each gang's strips together
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    auto work = [&](uint32_t x) {
        return static_cast<double>(reps[x].L) * reps[x].L * reps[x].n_sweeps / std::max<uint32_t>(reps[x].nwg, 1);
    };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return work(x) > work(y); });
    std::vector<uint2> items;
    for (uint32_t x : order)
        for (uint32_t j = 0; j < std::max<uint32_t>(reps[x].nwg, 1); ++j) items.push_back(make_uint2(x, j));
    const void *fn = batch_kernel_for(b->kind, sh.threads);
    // the largest strip LDS of any shape, so that batches planned with other
    // shapes keep launching
    uint32_t lds_top = 0;
    for (const BatchShape &x : kBatchShape) lds_top = std::max(lds_top, x.lds_cap);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_top));
    (void)hipGetLastError();
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, sh.threads, lds);
    if (e != hipSuccess) return e;
    if (occ < 1) return hipErrorOutOfMemory;
    const uint32_t resident = static_cast<uint32_t>(occ * std::max(b->n_cu, 1));
    if (resident < 2 * kMaxGang) {  // too few workgroups to run gangs safely: strips go to memory
        halo_bytes = 0;
        for (auto &d : reps)
            if (d.mode == kReplicaStrips) d = ReplicaDesc{d.spins, d.st, d.S, d.L, kReplicaMemory, d.T4, d.T8,
                                                          d.n_sweeps, d.trace, 0, 0, 0, nullptr, d.err};
        items.clear();
        for (uint32_t x : order) items.push_back(make_uint2(x, 0));
    }
    int clock_khz = 0;  // wall_clock64() rate
    if ((e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, b->device)) != hipSuccess) return e;
    const uint64_t start_ticks = static_cast<uint64_t>(kGangStartSeconds * 1e3 * std::max(clock_khz, 1));
    if (halo_bytes) {
        if ((e = hipMalloc(&b->d_halo, halo_bytes)) != hipSuccess) return e;
        uint64_t off = 0;
        for (auto &d : reps)
            if (d.mode == kReplicaStrips) {
                d.halo = reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(b->d_halo) + off);
                d.gang = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(b->d_halo) + off + 8ull * d.nwg * d.L);
                d.start_ticks = start_ticks;
                off += 8ull * d.nwg * d.L + kGangWordBytes;
            }
    }
    if ((e = hipMalloc(&b->d_reps, sizeof(ReplicaDesc) * n)) != hipSuccess) return e;
    if ((e = hipMalloc(&b->d_items, sizeof(uint2) * items.size())) != hipSuccess) return e;
    if ((e = hipMalloc(&b->d_next, 4)) != hipSuccess) return e;
    if ((e = hipMemcpy(b->d_reps, reps.data(), sizeof(ReplicaDesc) * n, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(b->d_items, items.data(), sizeof(uint2) * items.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    b->lds = lds;
    b->n_items = static_cast<uint32_t>(items.size());
    b->resident = resident;
    b->gangs = halo_bytes != 0;
    b->grid = std::min<uint32_t>(b->n_items, resident);
    return hipSuccess;
}

hipError_t launch_batch(IsingBatch *b, hipStream_t st) {
    if (b->n == 0) return hipSuccess;
    if (!b->d_reps || !b->d_items || !b->d_next) return hipErrorNotReady;  // a failed re-plan left no plan
    const auto *reps = static_cast<const ReplicaDesc *>(b->d_reps);
    const auto *items = static_cast<const uint2 *>(b->d_items);
    hipLaunchKernelGGL(k_batch_prologue, dim3(b->n), dim3(kBlock), 0, st, reps, b->d_next);
    const void *fn = batch_kernel_for(b->kind, kBatchShape[b->shape].threads);
    if (!fn) return hipErrorInvalidValue;
    uint32_t n_items = b->n_items;
    uint32_t *next = b->d_next;
    const uint32_t threads = kBatchShape[b->shape].threads;
    void *args[] = {&reps, &items, &n_items, &next};
    // With gangs, and outside graph capture, the launch is cooperative, which
    // makes the whole grid resident together whatever else runs on the
    // device; a captured launch relies on the grid fitting (it is sized to
    // what is resident at once) and on the gang start wait.  Without gangs no
    // workgroup waits for another, and a plain launch can overlap with other
    // work.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cap);
    if (e != hipSuccess) return e;
    if (b->gangs && cap == hipStreamCaptureStatusNone)
        return hipLaunchCooperativeKernel(fn, dim3(b->grid), dim3(threads), args, b->lds, st);
    return hipLaunchKernel(fn, dim3(b->grid), dim3(threads), args, b->lds, st);
}

namespace {
// Every strip count the planner accepts for side L, most strips first (at
// most `max`): the autotuner's candidates besides the per-pass path.
template <class Unit>
int list_plans(uint32_t L, int max_spt, int n_cu, IsingPlan *out, int max) {
    int n = 0;
    // up to two strips per CU (smaller workgroups, several per CU)
    const uint32_t top = std::min<uint32_t>(L, 2 * static_cast<uint32_t>(std::max(n_cu, 1)));
    for (uint32_t nwg = top; nwg >= 1 && n < max; --nwg) {
        if (L % nwg) continue;
        if (nwg > 1 && static_cast<uint64_t>(L / nwg) * L < 2048) continue;
        IsingPlan p;
        if (try_strips<Unit>(L, nwg, max_spt, n_cu, &p)) out[n++] = p;
    }
    return n;
}
}  // namespace

int ising_plan_list(uint32_t L, rngx_kind kind, int n_cu, IsingPlan *out, int max) {
    switch (kind) {
    case RNGX_LCG32: return list_plans<SmallUnit<Lcg32>>(L, 16, n_cu, out, max);
    case RNGX_LCG32_SUB: return list_plans<SmallUnit<Lcg32Sub>>(L, 16, n_cu, out, max);
    case RNGX_LCG64: return list_plans<SmallUnit<Lcg64>>(L, 16, n_cu, out, max);
    case RNGX_LCG64_SUB: return list_plans<SmallUnit<Lcg64Sub>>(L, 16, n_cu, out, max);
    case RNGX_MWC: return list_plans<SmallUnit<Mwc>>(L, 16, n_cu, out, max);
    case RNGX_MWC_DIFF: return list_plans<SmallUnit<MwcDiff>>(L, 16, n_cu, out, max);
    case RNGX_XORWOW: return list_plans<SmallUnit<Xorwow>>(L, 16, n_cu, out, max);
    case RNGX_PHILOX4X32_10: return list_plans<PhiloxUnit>(L, 16, n_cu, out, max);
    case RNGX_PHILOX4X32_7: return list_plans<PhiloxUnit7>(L, 16, n_cu, out, max);
    case RNGX_XS1024W: return list_plans<XsUnit>(L, 16, n_cu, out, max);
    case RNGX_LFG521: return list_plans<LfgStripUnit<521, 353>>(L, 16, n_cu, out, max);
    case RNGX_LFG1279: return list_plans<LfgStripUnit<1279, 861>>(L, 16, n_cu, out, max);
    default: break;
    }
    return 0;
}

bool ising_plan(uint32_t L, rngx_kind kind, int n_cu, IsingPlan *out) {
    switch (kind) {
    case RNGX_LCG32: return plan_strips<SmallUnit<Lcg32>>(L, 16, n_cu, out);
    case RNGX_LCG32_SUB: return plan_strips<SmallUnit<Lcg32Sub>>(L, 16, n_cu, out);
    case RNGX_LCG64: return plan_strips<SmallUnit<Lcg64>>(L, 16, n_cu, out);
    case RNGX_LCG64_SUB: return plan_strips<SmallUnit<Lcg64Sub>>(L, 16, n_cu, out);
    case RNGX_MWC: return plan_strips<SmallUnit<Mwc>>(L, 16, n_cu, out);
    case RNGX_MWC_DIFF: return plan_strips<SmallUnit<MwcDiff>>(L, 16, n_cu, out);
    case RNGX_XORWOW: return plan_strips<SmallUnit<Xorwow>>(L, 16, n_cu, out);
    case RNGX_PHILOX4X32_10: return plan_strips<PhiloxUnit>(L, 16, n_cu, out);
    case RNGX_PHILOX4X32_7: return plan_strips<PhiloxUnit7>(L, 16, n_cu, out);
    case RNGX_XS1024W: return plan_strips<XsUnit>(L, 16, n_cu, out);
    case RNGX_LFG521: return plan_strips<LfgStripUnit<521, 353>>(L, 16, n_cu, out);
    case RNGX_LFG1279: return plan_strips<LfgStripUnit<1279, 861>>(L, 16, n_cu, out);
    default: break;
    }
    return false;
}

namespace {
constexpr int kLfgPassThreads = 256;  // single-hit LFG passes: four units per thread

template <int R, int SL, bool MH>
hipError_t run_passes_lfg(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st,
                          uint32_t hits) {
    const uint64_t G = lat->gen->S / kLfgLanes;
    PassArgs pa{lat->d_spins, lat->gen->d_state, lat->gen->S, lat->L, 0, T4, T8, nullptr, hits};
    for (uint64_t t = 0; t < n; ++t) {
        for (int c = 0; c < 2; ++c) {
            pa.c = c;
            pa.partial = (c == 1 && tr) ? lat->d_partial : nullptr;
            if constexpr (MH)
                hipLaunchKernelGGL((k_ising_pass_lfg<R, SL, true>), dim3(static_cast<unsigned>(G)), dim3(1024), 0, st, pa);
            else
                hipLaunchKernelGGL((k_ising_pass_lfg_n<R, SL, kLfgPassThreads>), dim3(static_cast<unsigned>(G)),
                                   dim3(kLfgPassThreads), 0, st, pa);
        }
        if (tr) hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, st, lat->d_partial, G, tr + t);
    }
    return hipGetLastError();
}

template <int R, int SL, bool MH>
hipError_t run_one_lfg(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st, uint32_t hits) {
    PassArgs pa{lat->d_spins, lat->gen->d_state, lat->gen->S, lat->L, 0, T4, T8, nullptr, hits};
    hipLaunchKernelGGL((k_ising_lfg_one<R, SL, MH>), dim3(1), dim3(1024), 0, st, pa, n, tr);
    return hipGetLastError();
}

template <int R, int SL>
hipError_t run_lfg(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st, uint32_t hits) {
    if (n == 0) return hipSuccess;
    // single-hit sweeps on chip when a strip plan holds whole instances
    if (hits == 1 && lat->plan.strips) return run_strips<LfgStripUnit<R, SL>, false>(lat, T4, T8, n, tr, st, 1);
    if (lat->gen->S == kLfgLanes) {
        if (hits == 1) return run_one_lfg<R, SL, false>(lat, T4, T8, n, tr, st, 1);
        return run_one_lfg<R, SL, true>(lat, T4, T8, n, tr, st, hits);
    }
    if (hits == 1) return run_passes_lfg<R, SL, false>(lat, T4, T8, n, tr, st, 1);
    return run_passes_lfg<R, SL, true>(lat, T4, T8, n, tr, st, hits);
}
}  // namespace

uint64_t ising_partials(uint32_t L) { return (static_cast<uint64_t>(L) * L / 4 + kBlock - 1) / kBlock; }

hipError_t launch_hot_start(Ising *lat, uint64_t seed, hipStream_t st) {
    const uint64_t n_words = static_cast<uint64_t>(lat->L) * lat->L / 4;
    const unsigned blocks = static_cast<unsigned>((n_words + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_hot_start, dim3(blocks), dim3(kBlock), 0, st, lat->d_spins, n_words, seed);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t *p, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_ising(Ising *lat, double beta, uint64_t n_sweeps, int32_t *d_trace, hipStream_t st,
                        uint32_t hits) {
    // Thresholds floor(exp(-beta dE) 2^32) in IEEE double on the host.
    const uint64_t T4 = static_cast<uint64_t>(std::floor(std::exp(-4.0 * beta) * 4294967296.0));
    const uint64_t T8 = static_cast<uint64_t>(std::floor(std::exp(-8.0 * beta) * 4294967296.0));
    switch (lat->gen->kind) {
    case RNGX_LCG32: return run<SmallUnit<Lcg32>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_LCG32_SUB: return run<SmallUnit<Lcg32Sub>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_LCG64: return run<SmallUnit<Lcg64>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_LCG64_SUB: return run<SmallUnit<Lcg64Sub>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_MWC: return run<SmallUnit<Mwc>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_MWC_DIFF: return run<SmallUnit<MwcDiff>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_XORWOW: return run<SmallUnit<Xorwow>>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_PHILOX4X32_10: return run<PhiloxUnit>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_PHILOX4X32_7: return run<PhiloxUnit7>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_XS1024W: return run<XsUnit>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_LFG521: return run_lfg<521, 353>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    case RNGX_LFG1279: return run_lfg<1279, 861>(lat, T4, T8, n_sweeps, d_trace, st, hits);
    default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace rngx
