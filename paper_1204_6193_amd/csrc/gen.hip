// Seeding, bulk fill and consume kernels for all generator kinds.
//
// Fills are HBM-write-bound: each thread keeps its streams' state in VGPRs
// for the whole launch (loaded once, stored once) and writes output k of
// stream s to out[k*S + s], so a wavefront's stores cover one contiguous
// span per step.  Small-state kinds run V consecutive streams per thread
// (V = 4: one 16-byte store per step); XS1024W runs one instance per
// 16-lane DPP row with two words per lane (one 8-byte store per step).
#include <algorithm>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kXsSync = 16;  // rows between its barriers when not paced (a power of two)
// --------------------------------------------------------------------------
// Seeding (definitions in rngx.h).
__global__ __launch_bounds__(kBlock) void k_seed_small(rngx_kind kind, uint8_t *st, uint64_t S, uint64_t seed) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint32_t *u32 = reinterpret_cast<uint32_t *>(st);
    uint64_t *u64 = reinterpret_cast<uint64_t *>(st);
    switch (kind) {
    case RNGX_LCG32: u32[s] = static_cast<uint32_t>(splitmix(seed, 1 + s)); break;
    case RNGX_LCG64: u64[s] = splitmix(seed, 1 + s); break;
    case RNGX_LCG32_SUB:
    case RNGX_LCG64_SUB: {
        // stream s at position s of the sequence from the plain stream-0 value;
        // the S-step map after the states
        const bool l32 = kind == RNGX_LCG32_SUB;
        const uint64_t a = l32 ? kLcg32A : kLcg64A, c = l32 ? kLcg32C : kLcg64C;
        const uint64_t g0 = l32 ? static_cast<uint32_t>(splitmix(seed, 1)) : splitmix(seed, 1);
        uint64_t A, C;
        affine_power(a, c, s, &A, &C);
        if (l32) u32[s] = static_cast<uint32_t>(A * g0 + C);
        else u64[s] = A * g0 + C;
        if (s == 0) {
            affine_power(a, c, S, &A, &C);
            if (l32) { u32[S] = static_cast<uint32_t>(A); u32[S + 1] = static_cast<uint32_t>(C); }
            else { u64[S] = A; u64[S + 1] = C; }
        }
        break;
    }
    case RNGX_MWC: {
        const uint64_t z = splitmix(seed, 1 + s);
        uint64_t x = z & 0xFFFFFFFFull, c = (z >> 32) % (kMwcA - 1);
        if (x == 0 && c == 0) x = 1;
        u64[s] = (c << 32) | x;
        break;
    }
    case RNGX_MWC_DIFF: {  // the multipliers are already in place after the states
        const uint64_t a = reinterpret_cast<const uint32_t *>(st + 8 * S)[s];
        const uint64_t z = splitmix(seed, 1 + s);
        uint64_t x = z & 0xFFFFFFFFull, c = (z >> 32) % (a - 1);
        if (x == 0 && c == 0) x = 1;
        u64[s] = (c << 32) | x;
        break;
    }
    case RNGX_XORWOW: {
        const uint64_t p = splitmix(seed, 1 + 3 * s), q = splitmix(seed, 2 + 3 * s), r = splitmix(seed, 3 + 3 * s);
        uint32_t w[6] = {static_cast<uint32_t>(p), static_cast<uint32_t>(p >> 32), static_cast<uint32_t>(q),
                         static_cast<uint32_t>(q >> 32), static_cast<uint32_t>(r), static_cast<uint32_t>(r >> 32)};
        if ((w[0] | w[1] | w[2] | w[3] | w[4]) == 0) w[0] = 1;
        for (int i = 0; i < 6; ++i) u32[i * S + s] = w[i];
        break;
    }
    case RNGX_PHILOX4X32_7:
    case RNGX_PHILOX4X32_10: {
        const uint64_t z = splitmix(seed, 1 + s);
        u32[s] = static_cast<uint32_t>(z);
        u32[S + s] = static_cast<uint32_t>(z >> 32);
        reinterpret_cast<uint64_t *>(st + 8 * S)[s] = 0;
        break;
    }
    default: break;
    }
}

// XS1024W: one thread per 64-bit seed word (two state words).  Among the 16
// words SM(1+16g .. 16+16g) of an instance at most one can be zero (mix64 is
// a bijection with mix64(0) = 0), so no instance is seeded all-zero.
__global__ __launch_bounds__(kBlock) void k_seed_xs(uint8_t *st, uint64_t S, uint64_t seed) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;  // pair index
    const uint64_t G = S / 32;
    if (t >= 16 * G) return;
    const uint64_t z = splitmix(seed, 1 + t);  // t = 16 g + i/2
    reinterpret_cast<uint2 *>(st)[t] = make_uint2(static_cast<uint32_t>(z), static_cast<uint32_t>(z >> 32));
    if ((t & 15) == 0) reinterpret_cast<uint64_t *>(st + 4 * S)[t >> 4] = 0;
    if (t == 0) *reinterpret_cast<uint32_t *>(st + 4 * S + 8 * G) = static_cast<uint32_t>(splitmix(seed, 0) >> 32);
}

// --------------------------------------------------------------------------
// Output stores.
__device__ __forceinline__ float to_unit(uint32_t u) { return static_cast<float>(u >> 8) * 0x1.0p-24f; }

// Non-temporal stores: the outputs are streamed out and not read back by
// this kernel (XS1024W u32 fill at 2^20 x 4096: 6.30 -> 6.55 TB/s).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int MODE, int V>
__device__ __forceinline__ void store_out(void *out, uint64_t idx, const uint32_t (&u)[V]) {
    uint32_t w[V];
    for (int v = 0; v < V; ++v) w[v] = MODE == kOutU32 ? u[v] : __float_as_uint(to_unit(u[v]));
    uint32_t *o = static_cast<uint32_t *>(out) + idx;
    if constexpr (V == 4) {
        const u32x4 x = {w[0], w[1], w[2], w[3]};
        __builtin_nontemporal_store(x, reinterpret_cast<u32x4 *>(o));
    } else if constexpr (V == 2) {
        __builtin_nontemporal_store(w[0] | static_cast<uint64_t>(w[1]) << 32, reinterpret_cast<uint64_t *>(o));
    } else {
        __builtin_nontemporal_store(w[0], o);
    }
}

// Small-state kinds: V consecutive streams per thread.
template <class G, int MODE, int V>
__global__ __launch_bounds__(kBlock) void k_fill_small(uint8_t *st, uint64_t S, uint64_t count, void *out) {
    const uint64_t s0 = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * V;
    if (s0 >= S) return;
    G g[V];
#pragma unroll
    for (int v = 0; v < V; ++v) g[v].load(st, S, s0 + v);
    uint32_t acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0;
    auto emit = [&](uint64_t k, const uint32_t (&u)[V]) {
        if constexpr (MODE == kOutXor) {
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] ^= u[v];
        } else {
            store_out<MODE, V>(out, k * S + s0, u);
        }
    };
    uint64_t k = 0;
    if constexpr (HasNext8<G>::value) {  // 8 outputs of each stream at a time
        for (; k + 8 <= count; k += 8) {
            uint32_t d[V][8];
#pragma unroll
            for (int v = 0; v < V; ++v) g[v].next8(d[v]);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                uint32_t u[V];
#pragma unroll
                for (int v = 0; v < V; ++v) u[v] = d[v][kk];
                emit(k + kk, u);
            }
        }
    }
    for (; k < count; ++k) {
        uint32_t u[V];
#pragma unroll
        for (int v = 0; v < V; ++v) u[v] = g[v].next();
        emit(k, u);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) g[v].store(st, S, s0 + v);
    if constexpr (MODE == kOutXor) {
        uint32_t *o = static_cast<uint32_t *>(out);
#pragma unroll
        for (int v = 0; v < V; ++v) o[s0 + v] = acc[v];
    }
}

// Small-state kinds, paced: V consecutive streams per thread, BLK threads
// per workgroup (S % V == 0; threads past the last stream stay in the loop
// with their stores masked, since they take part in the barriers).
template <class G, int MODE, int V, int BLK>
__global__ __launch_bounds__(BLK) void k_fill_paced(uint8_t *st, uint64_t S, uint64_t count, void *out,
                                                    uint32_t *ring) {
    const uint64_t s0 = (static_cast<uint64_t>(blockIdx.x) * BLK + threadIdx.x) * V;
    const bool live = s0 < S;
    G g[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (live) g[v].load(st, S, s0 + v);
    __shared__ uint32_t s_free;
    Pacer pc(ring);
    for (uint64_t k0 = 0, band = 0; k0 < count; k0 += kBand, ++band) {
        pc.before(band, &s_free);
        auto row = [&](uint64_t k) {
            uint32_t u[V];
#pragma unroll
            for (int v = 0; v < V; ++v) u[v] = g[v].next();
            if (live) store_out<MODE, V>(out, k * S + s0, u);
        };
        const uint64_t k1 = k0 + kBand < count ? k0 + kBand : count;
        if (k1 - k0 == kBand) {
            if constexpr (HasNext8<G>::value) {  // a band is 8 outputs of each stream
                static_assert(kBand == 8, "next8 covers one band");
                uint32_t d[V][8];
#pragma unroll
                for (int v = 0; v < V; ++v) g[v].next8(d[v]);
#pragma unroll
                for (uint32_t kk = 0; kk < kBand; ++kk) {
                    uint32_t u[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) u[v] = d[v][kk];
                    if (live) store_out<MODE, V>(out, (k0 + kk) * S + s0, u);
                }
            } else {
#pragma unroll
                for (uint32_t kk = 0; kk < kBand; ++kk) row(k0 + kk);
            }
        } else {
            for (uint64_t k = k0; k < k1; ++k) row(k);
        }
        pc.after(band);
    }
    if (!live) return;
#pragma unroll
    for (int v = 0; v < V; ++v) g[v].store(st, S, s0 + v);
}

// XS1024W: thread t runs lane j = t % 16 of instance g = t / 16.  The output
// is written row by row across all streams.  How fast HBM takes these rows
// depends on how many distinct rows the chip writes at once, i.e. on how far
// the workgroups drift apart, so a paced launch (ring != null, whole grid
// resident) keeps them together: rows go in bands of kBand, and before band b
// a workgroup waits until every workgroup has finished band b - kSlack.
// Completion is counted in a ring of kRing band entries of kPaceSlots
// counters (workgroup w adds 1 to slot w % kPaceSlots), so that no counter is
// hit by more than a few workgroups; an entry's target after its u-th use is
// u times the workgroups of its slot (Pacer).  Waits are bounded: a workgroup
// that waited kPollLimit polls runs free for the rest of the launch.  Pacing
// only decides when a row is written, never what is written.  Unpaced launches
// meet at a block barrier every kXsSync rows instead.  Rows past the last
// instance stay in the loop with their loads and stores masked, since every
// wave of the block has to reach each barrier; they are whole 16-lane rows,
// so no active instance sees one of their words.
template <int MODE, int BLK>
__global__ __launch_bounds__(BLK) void k_fill_xs(uint8_t *st, uint64_t S, uint64_t count, void *out,
                                                 uint32_t *ring) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t G = S / 32, g = t >> 4;
    const bool live = g < G;
    if (MODE == kOutXor && !live) return;                 // no barriers in this mode
    uint2 *W = reinterpret_cast<uint2 *>(st);
    uint64_t *N = reinterpret_cast<uint64_t *>(st + 4 * S);
    const uint32_t y0 = *reinterpret_cast<const uint32_t *>(st + 4 * S + 8 * G);
    const uint2 w = live ? W[t] : make_uint2(0, 0);
    uint32_t a = w.x, b = w.y;
    const uint64_t n = live ? N[g] : 0;
    uint32_t y = y0 + static_cast<uint32_t>(n) * kWeylC;
    uint32_t acc0 = 0, acc1 = 0;
    __shared__ uint32_t s_free;
    Pacer pc(MODE != kOutXor ? ring : nullptr);
    for (uint64_t k0 = 0, band = 0; k0 < count; k0 += kBand, ++band) {
        if constexpr (MODE != kOutXor) pc.before(band, &s_free);
        auto row = [&](uint64_t k) {
            xs1024_step(a, b);
            y += kWeylC;
            const uint32_t m = weyl_mix(y);
            const uint32_t u[2] = {a + m, b + m};
            if constexpr (MODE == kOutXor) {
                acc0 ^= u[0];
                acc1 ^= u[1];
            } else {
                if (live) store_out<MODE, 2>(out, k * S + 2 * t, u);
            }
        };
        const uint64_t k1 = k0 + kBand < count ? k0 + kBand : count;
        if (k1 - k0 == kBand) {
#pragma unroll
            for (uint32_t kk = 0; kk < kBand; ++kk) row(k0 + kk);
        } else {
            for (uint64_t k = k0; k < k1; ++k) row(k);
        }
        if constexpr (MODE != kOutXor) {
            if (pc.ring) pc.after(band);
            else if ((k1 & (kXsSync - 1)) == 0) __syncthreads();
        }
    }
    if (!live) return;
    W[t] = make_uint2(a, b);
    if ((t & 15) == 0) N[g] = n + count;
    if constexpr (MODE == kOutXor) reinterpret_cast<uint2 *>(out)[t] = make_uint2(acc0, acc1);
}

__global__ __launch_bounds__(kBlock) void k_zero_ring(uint32_t *ring) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < kRing * kPaceSlots) ring[i] = 0;
}

// ---------------------------------------------------------------- configurations
// The fill configurations the autotuner chooses from; every one of them
// produces the same values.  Small-state kinds: paced or not, streams per
// thread, threads per workgroup (the unpaced one is k_fill_small).
// XS1024W: always one lane pair per thread; paced or not, threads per
// workgroup.  The first entry of each list is the default (XORWOW: the
// second), as measured at 2^20 streams x 4096.
constexpr rngx_fill_config kSmallConfigs[] = {{1, 4, 512}, {1, 4, 1024}, {1, 4, 256}, {1, 2, 1024},
                                              {1, 2, 512}, {1, 2, 256},  {0, 4, 256}};
constexpr rngx_fill_config kXsConfigs[] = {{1, 2, 1024}, {1, 2, 512}, {0, 2, 1024}, {0, 2, 256}};
// Lagged Fibonacci kinds: one wave per 1024-stream instance (16 streams per
// lane), four waves per workgroup, free-running.
constexpr rngx_fill_config kLfgConfigs[] = {{1, 16, 256}, {0, 16, 256}};
constexpr int kNumSmall = sizeof(kSmallConfigs) / sizeof(kSmallConfigs[0]);
constexpr int kNumXs = sizeof(kXsConfigs) / sizeof(kXsConfigs[0]);
static_assert(kNumSmall <= kMaxFillConfigs && kNumXs <= kMaxFillConfigs, "Gen::resident too small");

int default_config(rngx_kind kind) { return kind == RNGX_XORWOW ? 1 : 0; }

// Kernel of a configuration (U32 or F32), for launches and occupancy.
template <class G, int MODE>
const void *paced_kernel(int v, int blk) {
    if (v == 4 && blk == 256) return reinterpret_cast<const void *>(&k_fill_paced<G, MODE, 4, 256>);
    if (v == 4 && blk == 512) return reinterpret_cast<const void *>(&k_fill_paced<G, MODE, 4, 512>);
    if (v == 4 && blk == 1024) return reinterpret_cast<const void *>(&k_fill_paced<G, MODE, 4, 1024>);
    if (v == 2 && blk == 256) return reinterpret_cast<const void *>(&k_fill_paced<G, MODE, 2, 256>);
    if (v == 2 && blk == 512) return reinterpret_cast<const void *>(&k_fill_paced<G, MODE, 2, 512>);
    if (v == 2 && blk == 1024) return reinterpret_cast<const void *>(&k_fill_paced<G, MODE, 2, 1024>);
    return nullptr;
}
template <int MODE>
const void *xs_kernel(int blk) {
    if (blk == 256) return reinterpret_cast<const void *>(&k_fill_xs<MODE, 256>);
    if (blk == 512) return reinterpret_cast<const void *>(&k_fill_xs<MODE, 512>);
    if (blk == 1024) return reinterpret_cast<const void *>(&k_fill_xs<MODE, 1024>);
    return nullptr;
}
template <class G>
const void *config_kernel(int mode, const rngx_fill_config &c) {
    return mode == kOutU32 ? paced_kernel<G, kOutU32>(c.streams_per_thread, c.block)
                           : paced_kernel<G, kOutF32>(c.streams_per_thread, c.block);
}
const void *config_kernel(rngx_kind kind, int mode, const rngx_fill_config &c) {
    switch (kind) {
    case RNGX_LCG32: return config_kernel<Lcg32>(mode, c);
    case RNGX_LCG64: return config_kernel<Lcg64>(mode, c);
    case RNGX_MWC: return config_kernel<Mwc>(mode, c);
    case RNGX_MWC_DIFF: return config_kernel<MwcDiff>(mode, c);
    case RNGX_XORWOW: return config_kernel<Xorwow>(mode, c);
    case RNGX_PHILOX4X32_10: return config_kernel<Philox>(mode, c);
    case RNGX_PHILOX4X32_7: return config_kernel<Philox7>(mode, c);
    case RNGX_LCG32_SUB: return config_kernel<Lcg32Sub>(mode, c);
    case RNGX_LCG64_SUB: return config_kernel<Lcg64Sub>(mode, c);
    case RNGX_XS1024W: return mode == kOutU32 ? xs_kernel<kOutU32>(c.block) : xs_kernel<kOutF32>(c.block);
    default: break;  // lagged Fibonacci kinds have their own kernel
    }
    return nullptr;
}

// Workgroups of configuration i that fit on the device at once (cached).
uint32_t resident(Gen *g, int i, const rngx_fill_config &c) {
    if (g->resident[i] >= 0) return static_cast<uint32_t>(g->resident[i]);
    int u = 0, f = 0;
    const void *ku = config_kernel(g->kind, kOutU32, c), *kf = config_kernel(g->kind, kOutF32, c);
    if (!ku || !kf || hipOccupancyMaxActiveBlocksPerMultiprocessor(&u, ku, c.block, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&f, kf, c.block, 0) != hipSuccess) {
        (void)hipGetLastError();
        u = f = 0;
    }
    g->resident[i] = std::min(u, f) * std::max(g->n_cu, 0);
    return static_cast<uint32_t>(g->resident[i]);
}

// Pace a launch of `blocks` workgroups of configuration i: large enough and
// every workgroup resident at once.
bool pace_ok(Gen *g, int i, const rngx_fill_config &c, uint64_t blocks, uint64_t count) {
    return g->d_ring && count >= 4 * kBand && blocks >= 128 && blocks <= resident(g, i, c);
}

void clear_ring(Gen *g, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_ring, dim3((kRing * kPaceSlots + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g->d_ring);
}

template <class G, int MODE>
hipError_t fill_small(Gen *g, void *out, uint64_t count, hipStream_t st) {
    const uint64_t S = g->S;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(out);
    const bool vec4 = (S % 4 == 0) && (addr % 16 == 0);
    if constexpr (MODE != kOutXor) {
        const int i = g->fill_cfg >= 0 ? g->fill_cfg : default_config(g->kind);
        const rngx_fill_config c = kSmallConfigs[i];
        const int V = c.streams_per_thread;
        if (c.paced && S % V == 0 && addr % (4 * V) == 0) {
            const uint64_t blocks = (S / V + c.block - 1) / c.block;
            const bool pace = pace_ok(g, i, c, blocks, count);
            if (pace) clear_ring(g, st);
            uint32_t *ring = pace ? g->d_ring : nullptr;
            void *args[] = {&g->d_state, const_cast<uint64_t *>(&S), &count, &out, &ring};
            const hipError_t e = hipLaunchKernel(config_kernel<G>(MODE, c), dim3(static_cast<unsigned>(blocks)),
                                                 dim3(c.block), args, 0, st);
            return e != hipSuccess ? e : hipGetLastError();
        }
    }
    if (vec4) {
        const uint64_t threads = S / 4;
        const unsigned blocks = static_cast<unsigned>((threads + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_fill_small<G, MODE, 4>), dim3(blocks), dim3(kBlock), 0, st, g->d_state, S, count, out);
    } else {
        const unsigned blocks = static_cast<unsigned>((S + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_fill_small<G, MODE, 1>), dim3(blocks), dim3(kBlock), 0, st, g->d_state, S, count, out);
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t fill_xs(Gen *g, void *out, uint64_t count, hipStream_t st) {
    const int i = MODE == kOutXor ? 2 : (g->fill_cfg >= 0 ? g->fill_cfg : default_config(g->kind));
    const rngx_fill_config c = kXsConfigs[i];
    const uint64_t blocks = (g->S / 2 + c.block - 1) / c.block;
    const bool pace = MODE != kOutXor && c.paced && pace_ok(g, i, c, blocks, count);
    if (pace) clear_ring(g, st);
    uint32_t *ring = pace ? g->d_ring : nullptr;
    const void *fn = MODE == kOutXor ? reinterpret_cast<const void *>(&k_fill_xs<kOutXor, 1024>) : xs_kernel<MODE>(c.block);
    void *args[] = {&g->d_state, &g->S, &count, &out, &ring};
    const hipError_t e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(blocks)), dim3(c.block), args, 0, st);
    return e != hipSuccess ? e : hipGetLastError();
}

template <int MODE>
hipError_t fill_mode(Gen *g, void *out, uint64_t count, hipStream_t st) {
    switch (g->kind) {
    case RNGX_LCG32: return fill_small<Lcg32, MODE>(g, out, count, st);
    case RNGX_LCG64: return fill_small<Lcg64, MODE>(g, out, count, st);
    case RNGX_MWC: return fill_small<Mwc, MODE>(g, out, count, st);
    case RNGX_MWC_DIFF: return fill_small<MwcDiff, MODE>(g, out, count, st);
    case RNGX_XORWOW: return fill_small<Xorwow, MODE>(g, out, count, st);
    case RNGX_PHILOX4X32_10: return fill_small<Philox, MODE>(g, out, count, st);
    case RNGX_PHILOX4X32_7: return fill_small<Philox7, MODE>(g, out, count, st);
    case RNGX_LCG32_SUB: return fill_small<Lcg32Sub, MODE>(g, out, count, st);
    case RNGX_LCG64_SUB: return fill_small<Lcg64Sub, MODE>(g, out, count, st);
    case RNGX_XS1024W: return fill_xs<MODE>(g, out, count, st);
    default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_seed(Gen *g, uint64_t seed, hipStream_t st) {
    if (is_lfg(g->kind)) return launch_seed_lfg(g, seed, st);
    if (g->kind == RNGX_XS1024W) {
        const uint64_t pairs = g->S / 2;
        const unsigned blocks = static_cast<unsigned>((pairs + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_seed_xs, dim3(blocks), dim3(kBlock), 0, st, g->d_state, g->S, seed);
    } else {
        if (g->kind == RNGX_MWC_DIFF) {
            const hipError_t e = mwc_diff_multipliers(g->S, reinterpret_cast<uint32_t *>(g->d_state + 8 * g->S), st);
            if (e != hipSuccess) return e;
        }
        const unsigned blocks = static_cast<unsigned>((g->S + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_seed_small, dim3(blocks), dim3(kBlock), 0, st, g->kind, g->d_state, g->S, seed);
    }
    return hipGetLastError();
}

hipError_t launch_clear_ring(Gen *g, hipStream_t st) {
    clear_ring(g, st);
    return hipGetLastError();
}

hipError_t fill_setup(Gen *g, int n_cu) {
    g->d_ring = nullptr;
    g->n_cu = n_cu;
    g->fill_cfg = -1;
    for (int i = 0; i < kMaxFillConfigs; ++i) g->resident[i] = -1;
    return hipMalloc(&g->d_ring, 4ull * kRing * kPaceSlots);
}

int fill_configs(rngx_kind kind, const rngx_fill_config **list) {
    if (is_lfg(kind)) { *list = kLfgConfigs; return 2; }
    *list = kind == RNGX_XS1024W ? kXsConfigs : kSmallConfigs;
    return kind == RNGX_XS1024W ? kNumXs : kNumSmall;
}

int fill_default(rngx_kind kind) { return default_config(kind); }

hipError_t launch_fill(Gen *g, void *d_out, uint64_t count, int mode, hipStream_t st) {
    if (is_lfg(g->kind)) return launch_fill_lfg(g, d_out, count, mode, st);
    if (mode == kOutU32) return fill_mode<kOutU32>(g, d_out, count, st);
    if (mode == kOutF32) return fill_mode<kOutF32>(g, d_out, count, st);
    return fill_mode<kOutXor>(g, d_out, count, st);
}

}  // namespace rngx
