// Checkerboard Metropolis update of the 2D Ising ferromagnet (the paper's
// application test, Sec. 2) driven by the per-stream generators.
//
// Stream s = y*(L/4) + x/4 owns the 4-site word x0..x0+3 of row y.  In colour
// pass c it updates sites x0 + ((c+y)&1) and x0 + 2 + ((c+y)&1) with its next
// two outputs.  One launch per colour pass: a thread loads its stream
// state, its spin word and the neighbouring words, makes both updates and
// writes back.  The energy after a sweep is accumulated in the colour-1 pass:
// every bond has exactly one colour-1 end, and colour 0 is final by then, so
// E = -sum over colour-1 sites of s_i * (sum of its 4 neighbours).
#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kBlock = 256;

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

__device__ __forceinline__ int spin_at(uint64_t word, int i) { return static_cast<int8_t>(word >> (8 * i)); }

// Update byte i of `word` (a 4- or 8-site run of one row).  lft/rgt are the
// spins just outside the run, up/dn the words of the rows above and below.
// Returns the post-update s_i * (neighbour sum) for the energy.
template <int NBYTES>
__device__ __forceinline__ int update_site(uint64_t &word, int i, int lft, int rgt, uint64_t up, uint64_t dn,
                                           uint32_t r, uint64_t T4, uint64_t T8) {
    const int s = spin_at(word, i);
    const int l = i > 0 ? spin_at(word, i - 1) : lft;
    const int rr = i < NBYTES - 1 ? spin_at(word, i + 1) : rgt;
    const int nb = l + rr + spin_at(up, i) + spin_at(dn, i);
    const int dE = 2 * s * nb;
    const uint64_t thr = dE == 4 ? T4 : T8;
    const bool acc = dE <= 0 || static_cast<uint64_t>(r) < thr;
    const int s_new = acc ? -s : s;
    const uint64_t m = 0xFFull << (8 * i);
    word = (word & ~m) | (static_cast<uint64_t>(static_cast<uint8_t>(s_new)) << (8 * i));
    return s_new * nb;
}

__device__ __forceinline__ void block_energy_add(int e, int32_t *dst) {
    // wave reduction, then one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0 && e != 0) atomicAdd(dst, -e);
}

// Small-state kinds: one stream (4-site word) per thread.
template <class G>
__global__ __launch_bounds__(kBlock) void k_pass_small(int8_t *spins, uint8_t *st, uint64_t S, uint32_t L, int c,
                                                        uint64_t T4, uint64_t T8, int32_t *trace_t) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c == 0 && trace_t && s == 0) *trace_t = 0;
    int e = 0;
    if (s < S) {
        const uint32_t spr = L >> 2;
        const uint32_t y = static_cast<uint32_t>(s / spr), x0 = 4 * static_cast<uint32_t>(s % spr);
        const uint64_t row = static_cast<uint64_t>(y) * L;
        const uint64_t up_row = static_cast<uint64_t>(y == 0 ? L - 1 : y - 1) * L;
        const uint64_t dn_row = static_cast<uint64_t>(y == L - 1 ? 0 : y + 1) * L;
        uint64_t word = *reinterpret_cast<const uint32_t *>(spins + row + x0);
        const uint64_t up = *reinterpret_cast<const uint32_t *>(spins + up_row + x0);
        const uint64_t dn = *reinterpret_cast<const uint32_t *>(spins + dn_row + x0);
        const int lft = spins[row + (x0 == 0 ? L - 1 : x0 - 1)];
        const int rgt = spins[row + (x0 + 4 == L ? 0 : x0 + 4)];
        const int p = (c + y) & 1;
        G g;
        g.load(st, S, s);
        const uint32_t r0 = g.next();
        const uint32_t r1 = g.next();
        g.store(st, S, s);
        e += update_site<4>(word, p, lft, rgt, up, dn, r0, T4, T8);
        e += update_site<4>(word, p + 2, lft, rgt, up, dn, r1, T4, T8);
        *reinterpret_cast<uint32_t *>(spins + row + x0) = static_cast<uint32_t>(word);
    }
    if (c == 1 && trace_t) block_energy_add(e, trace_t);
}

// XS1024W: lane j of instance g (one 16-lane row) owns streams 32g+2j and
// 32g+2j+1, i.e. the 8-site run x0..x0+7 of one row.  Two instance steps
// give every lane its two draws for the pass.
__global__ __launch_bounds__(kBlock) void k_pass_xs(int8_t *spins, uint8_t *st, uint64_t S, uint32_t L, int c,
                                                     uint64_t T4, uint64_t T8, int32_t *trace_t) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t G = S / 32, g = t >> 4;
    if (c == 0 && trace_t && t == 0) *trace_t = 0;
    int e = 0;
    if (g < G) {  // whole rows are in or out
        uint2 *W = reinterpret_cast<uint2 *>(st);
        uint64_t *N = reinterpret_cast<uint64_t *>(st + 4 * S);
        const uint32_t y0 = *reinterpret_cast<const uint32_t *>(st + 4 * S + 8 * G);
        const uint2 w = W[t];
        uint32_t a = w.x, b = w.y;
        const uint64_t n = N[g];
        uint32_t yw = y0 + static_cast<uint32_t>(n) * kWeylC;
        xs1024_step(a, b);
        yw += kWeylC;
        uint32_t m = weyl_mix(yw);
        const uint32_t ra0 = a + m, rb0 = b + m;
        xs1024_step(a, b);
        yw += kWeylC;
        m = weyl_mix(yw);
        const uint32_t ra1 = a + m, rb1 = b + m;
        W[t] = make_uint2(a, b);
        if ((t & 15) == 0) N[g] = n + 2;

        const uint64_t sa = 2 * t;  // = 32 g + 2 j
        const uint32_t spr = L >> 2;
        const uint32_t y = static_cast<uint32_t>(sa / spr), x0 = 4 * static_cast<uint32_t>(sa % spr);
        const uint64_t row = static_cast<uint64_t>(y) * L;
        const uint64_t up_row = static_cast<uint64_t>(y == 0 ? L - 1 : y - 1) * L;
        const uint64_t dn_row = static_cast<uint64_t>(y == L - 1 ? 0 : y + 1) * L;
        uint64_t word = *reinterpret_cast<const uint64_t *>(spins + row + x0);
        const uint64_t up = *reinterpret_cast<const uint64_t *>(spins + up_row + x0);
        const uint64_t dn = *reinterpret_cast<const uint64_t *>(spins + dn_row + x0);
        const int lft = spins[row + (x0 == 0 ? L - 1 : x0 - 1)];
        const int rgt = spins[row + (x0 + 8 == L ? 0 : x0 + 8)];
        const int p = (c + y) & 1;
        e += update_site<8>(word, p, lft, rgt, up, dn, ra0, T4, T8);
        e += update_site<8>(word, p + 2, lft, rgt, up, dn, ra1, T4, T8);
        e += update_site<8>(word, p + 4, lft, rgt, up, dn, rb0, T4, T8);
        e += update_site<8>(word, p + 6, lft, rgt, up, dn, rb1, T4, T8);
        *reinterpret_cast<uint64_t *>(spins + row + x0) = word;
    }
    if (c == 1 && trace_t) block_energy_add(e, trace_t);
}

template <class G>
hipError_t sweeps_small(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st) {
    const uint64_t S = lat->gen->S;
    const unsigned blocks = static_cast<unsigned>((S + kBlock - 1) / kBlock);
    for (uint64_t t = 0; t < n; ++t) {
        int32_t *tt = tr ? tr + t : nullptr;
        for (int c = 0; c < 2; ++c) {
            hipLaunchKernelGGL((k_pass_small<G>), dim3(blocks), dim3(kBlock), 0, st, lat->d_spins, lat->gen->d_state,
                               S, lat->L, c, T4, T8, tt);
        }
    }
    return hipGetLastError();
}

hipError_t sweeps_xs(Ising *lat, uint64_t T4, uint64_t T8, uint64_t n, int32_t *tr, hipStream_t st) {
    const uint64_t S = lat->gen->S;
    const unsigned blocks = static_cast<unsigned>((S / 2 + kBlock - 1) / kBlock);
    for (uint64_t t = 0; t < n; ++t) {
        int32_t *tt = tr ? tr + t : nullptr;
        for (int c = 0; c < 2; ++c) {
            hipLaunchKernelGGL(k_pass_xs, dim3(blocks), dim3(kBlock), 0, st, lat->d_spins, lat->gen->d_state, S,
                               lat->L, c, T4, T8, tt);
        }
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hot_start(Ising *lat, uint64_t seed, hipStream_t st) {
    const uint64_t n_words = static_cast<uint64_t>(lat->L) * lat->L / 4;
    const unsigned blocks = static_cast<unsigned>((n_words + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_hot_start, dim3(blocks), dim3(kBlock), 0, st, lat->d_spins, n_words, seed);
    return hipGetLastError();
}

hipError_t launch_ising(Ising *lat, double beta, uint64_t n_sweeps, int32_t *d_trace, hipStream_t st) {
    // Thresholds floor(exp(-beta dE) 2^32) in IEEE double on the host.
    const uint64_t T4 = static_cast<uint64_t>(std::floor(std::exp(-4.0 * beta) * 4294967296.0));
    const uint64_t T8 = static_cast<uint64_t>(std::floor(std::exp(-8.0 * beta) * 4294967296.0));
    switch (lat->gen->kind) {
    case RNGX_LCG32: return sweeps_small<Lcg32>(lat, T4, T8, n_sweeps, d_trace, st);
    case RNGX_LCG64: return sweeps_small<Lcg64>(lat, T4, T8, n_sweeps, d_trace, st);
    case RNGX_MWC: return sweeps_small<Mwc>(lat, T4, T8, n_sweeps, d_trace, st);
    case RNGX_XORWOW: return sweeps_small<Xorwow>(lat, T4, T8, n_sweeps, d_trace, st);
    case RNGX_PHILOX4X32_10: return sweeps_small<Philox>(lat, T4, T8, n_sweeps, d_trace, st);
    case RNGX_XS1024W: return sweeps_xs(lat, T4, T8, n_sweeps, d_trace, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace rngx
