// Additive lagged Fibonacci generators (Lagged Fibonacci section):
// x_n = x_{n-r} + x_{n-s} mod 2^32 with (r, s) = (521, 353) or (1279, 861),
// the exact fixed-point form of u_n = u_{n-r} + u_{n-s} mod 1.  One sequence
// (instance) serves 1024 streams in warp order: stream lane i of instance g
// takes the instance's values 1024 k + i, k = 0, 1, ...
//
// The instance's state is its last r values, which a kernel stages in LDS as
// a ring: value q lives at ring[q mod B] (B a power of two >= r + the largest
// run of values written at once), so the window never moves.  Any run of at
// most s consecutive new values depends only on older values, so a run is
// one parallel step: every lane adds two ring words and writes one.
//
// Fill / consume: one wave per instance (workgroups of four waves, four
// instances), runs of 64 V values (V per lane), wave-synchronous with no
// barrier.  At 2^20 streams there are only 1024 instances, one wave per SIMD,
// so nothing hides a run's LDS latency and the run's instruction count sets
// the rate: the fill keeps every value twice, at q mod B and q mod B + B, so
// that a run's reads [x, x + 64 V) never wrap and every LDS address of a run
// is one base (uniform plus the lane) and an immediate offset.  Seeding and
// jump-ahead are plain per-instance kernels.  The Ising consumer is in
// ising.hip.
#include <algorithm>
#include <mutex>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kWaves = 4;  // instances (waves) per fill workgroup

__device__ __forceinline__ float to_unit_lfg(uint32_t u) { return static_cast<float>(u >> 8) * 0x1.0p-24f; }

// Orders the wave's LDS writes of one run before its reads of the next
// (lanes of a wave read words other lanes wrote).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ring geometry of the fill kernel: runs of 64 V values, V per lane; B a
// power of two >= r + P (and a multiple of P, so a run's writes never wrap).
template <int R, int SL>
struct LfgFill {
    static constexpr int V = SL >= 512 ? 8 : 4;  // 64 V <= s
    static constexpr int P = 64 * V;             // values per run (divides 1024)
    static constexpr int B = (R + P) <= 1024 ? 1024 : (R + P) <= 2048 ? 2048 : 4096;
    static_assert(P <= SL && 1024 % P == 0 && B % P == 0, "run longer than the short lag");
};

// `count` rows (1024 values) of every instance; MODE as the other fills.
// With a ring the workgroups are paced in bands of kBand rows like the other
// fills (Pacer); waves past the last instance stay for the barriers.
template <int R, int SL, int MODE>
__global__ __launch_bounds__(64 * kWaves) void k_fill_lfg(uint8_t *st, uint64_t S, uint64_t count, void *out,
                                                         uint32_t *ring) {
    using F = LfgFill<R, SL>;
    constexpr int V = F::V, P = F::P, B = F::B, RUNS = 1024 / P;
    __shared__ uint32_t rings[kWaves][2 * B];  // value q at [q mod B] and [q mod B + B]
    __shared__ uint32_t s_free;
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * kWaves + w;
    const uint64_t G = S / 1024;
    const bool live = g < G;
    if (!ring && !live) return;  // whole waves; without pacing there are no barriers
    uint32_t *rg = rings[w];
    uint32_t *X = reinterpret_cast<uint32_t *>(st) + (live ? g : 0) * R;
    if (live)
        for (int j = lane; j < R; j += 64) {  // x_{j-r} at (j - r) mod B, twice
            const uint32_t x = X[j];
            rg[B - R + j] = x;
            rg[2 * B - R + j] = x;
        }
    wave_lds_sync();
    uint32_t acc[RUNS * V];
#pragma unroll
    for (int i = 0; i < RUNS * V; ++i) acc[i] = 0;
    uint32_t q = 0;  // value index modulo 2^32 (only q mod B is used)
    Pacer pc(ring);
    for (uint64_t k0 = 0, band = 0; k0 < count; k0 += kBand, ++band) {
        pc.before(band, &s_free);
        const uint64_t k1 = k0 + kBand < count ? k0 + kBand : count;
        for (uint64_t k = k0; k < k1; ++k) {
#pragma unroll
            for (int f = 0; f < RUNS; ++f) {
                // q is a multiple of P and B of P: the run writes [q mod B,
                // q mod B + P) < B, and reads from bases below B that the
                // second copy extends past B
                const uint32_t *lag_r = rg + ((q - R) & (B - 1)) + lane;
                const uint32_t *lag_s = rg + ((q - SL) & (B - 1)) + lane;
                uint32_t *dst = rg + (q & (B - 1)) + lane;
                uint32_t v[V];
#pragma unroll
                for (int j = 0; j < V; ++j) v[j] = lag_r[64 * j] + lag_s[64 * j];
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    dst[64 * j] = v[j];
                    dst[64 * j + B] = v[j];
                }
                if constexpr (MODE == kOutXor) {
#pragma unroll
                    for (int j = 0; j < V; ++j) acc[f * V + j] ^= v[j];
                } else if (live) {
                    uint32_t *o = static_cast<uint32_t *>(out) + k * S + g * 1024 + f * P + lane;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const uint32_t word = MODE == kOutU32 ? v[j] : __float_as_uint(to_unit_lfg(v[j]));
                        __builtin_nontemporal_store(word, o + 64 * j);
                    }
                }
                q += P;
                wave_lds_sync();
            }
        }
        pc.after(band);
    }
    if (!live) return;
    if constexpr (MODE == kOutXor) {
        uint32_t *o = static_cast<uint32_t *>(out) + g * 1024 + lane;
#pragma unroll
        for (int i = 0; i < RUNS * V; ++i) o[64 * i] = acc[i];  // stream lane f P + 64 j + lane
    }
    for (int j = lane; j < R; j += 64) X[j] = rg[(q - R + j) & (B - 1)];
}

// Seeding: word j of instance g from SM(1 + H g + j/2), H = (r + 1)/2.
template <int R>
__global__ __launch_bounds__(256) void k_seed_lfg(uint8_t *st, uint64_t G, uint64_t seed) {
    constexpr uint64_t H = (R + 1) / 2;
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;  // (instance, pair)
    if (t >= G * H) return;
    const uint64_t g = t / H, i = t % H;
    const uint64_t z = splitmix(seed, 1 + H * g + i);
    uint32_t *X = reinterpret_cast<uint32_t *>(st) + g * R;
    X[2 * i] = static_cast<uint32_t>(z);
    if (2 * i + 1 < R) X[2 * i + 1] = static_cast<uint32_t>(z >> 32);
}

// An instance whose words are all even keeps its low bits zero for ever:
// give word 0 its low bit (one wave per instance).
template <int R>
__global__ __launch_bounds__(64) void k_seed_lfg_odd(uint8_t *st) {
    uint32_t *X = reinterpret_cast<uint32_t *>(st) + static_cast<uint64_t>(blockIdx.x) * R;
    uint32_t odd = 0;
    for (int j = threadIdx.x; j < R; j += 64) odd |= X[j] & 1u;
    if (!__any(odd) && threadIdx.x == 0) X[0] |= 1u;
}

// Jump: x_{m+N+j} = sum_i J_i x_{m+j+i} (J = x^N mod the characteristic
// polynomial), from the window extended by r - 1 values.  One workgroup per
// instance.
template <int R, int SL>
__global__ __launch_bounds__(1024) void k_skip_lfg(uint8_t *st, const uint32_t *J) {
    __shared__ uint32_t E[2 * R];
    __shared__ uint32_t Js[R];
    uint32_t *X = reinterpret_cast<uint32_t *>(st) + static_cast<uint64_t>(blockIdx.x) * R;
    for (int j = threadIdx.x; j < R; j += blockDim.x) { E[j] = X[j]; Js[j] = J[j]; }
    __syncthreads();
    for (int base = R; base < 2 * R - 1; base += SL) {  // runs of at most s new values
        const int k = base + threadIdx.x;
        uint32_t v = 0;
        const bool mine = threadIdx.x < SL && k < 2 * R - 1;
        if (mine) v = E[k - R] + E[k - SL];
        __syncthreads();
        if (mine) E[k] = v;
        __syncthreads();
    }
    for (int j = threadIdx.x; j < R; j += blockDim.x) {
        uint32_t acc = 0;
        for (int i = 0; i < R; ++i) acc += Js[i] * E[j + i];
        X[j] = acc;
    }
}

// ------------------------------------------------------------------ host
// Polynomials over Z/2^32 modulo P(x) = x^r - x^(r-s) - 1 (coefficient i at
// index i, degree < r).
struct LfgPoly {
    int r, s;
    void mulmod(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b, std::vector<uint32_t> *out) const {
        std::vector<uint32_t> t(2 * r - 1, 0);
        for (int i = 0; i < r; ++i) {
            if (!a[i]) continue;
            const uint32_t ai = a[i];
            uint32_t *ti = t.data() + i;
            for (int j = 0; j < r; ++j) ti[j] += ai * b[j];
        }
        for (int d = 2 * r - 2; d >= r; --d) {  // x^d = x^(d-s) + x^(d-r)
            t[d - s] += t[d];
            t[d - r] += t[d];
        }
        t.resize(r);
        *out = std::move(t);
    }
};

// x^(1024 * 2^i) mod P for i < 64, per kind, made once.
const std::vector<std::vector<uint32_t>> &row_powers(int r, int s) {
    static std::mutex mu;
    static std::vector<std::vector<uint32_t>> tab521, tab1279;
    std::lock_guard<std::mutex> lk(mu);
    auto &tab = r == 521 ? tab521 : tab1279;
    if (tab.empty()) {
        const LfgPoly P{r, s};
        std::vector<uint32_t> x(r, 0);  // x^1024 by 1024 multiplications by x
        x[0] = 1;
        for (int k = 0; k < 1024; ++k) {
            const uint32_t top = x[r - 1];
            for (int i = r - 1; i > 0; --i) x[i] = x[i - 1];
            x[0] = top;
            x[r - s] += top;
        }
        tab.push_back(x);
        for (int i = 1; i < 64; ++i) {
            std::vector<uint32_t> sq;
            P.mulmod(tab.back(), tab.back(), &sq);
            tab.push_back(std::move(sq));
        }
    }
    return tab;
}

template <int R, int SL>
hipError_t fill_lfg(Gen *g, void *out, uint64_t count, int mode, hipStream_t st) {
    const unsigned blocks = static_cast<unsigned>((g->S / 1024 + kWaves - 1) / kWaves);
    const dim3 block(64 * kWaves);
    // paced (the default configuration) when large enough and every
    // workgroup fits on the device at once
    uint32_t *ring = nullptr;
    if (mode != kOutXor && g->fill_cfg <= 0 && g->d_ring && count >= 4 * kBand && blocks >= 128) {
        int occ = 0;
        const void *fn = mode == kOutU32 ? reinterpret_cast<const void *>(&k_fill_lfg<R, SL, kOutU32>)
                                         : reinterpret_cast<const void *>(&k_fill_lfg<R, SL, kOutF32>);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * kWaves, 0) == hipSuccess &&
            static_cast<uint64_t>(occ) * std::max(g->n_cu, 0) >= blocks)
            ring = g->d_ring;
        (void)hipGetLastError();
    }
    if (ring) {
        const hipError_t e = launch_clear_ring(g, st);
        if (e != hipSuccess) return e;
    }
    if (mode == kOutU32) hipLaunchKernelGGL((k_fill_lfg<R, SL, kOutU32>), dim3(blocks), block, 0, st, g->d_state, g->S, count, out, ring);
    else if (mode == kOutF32) hipLaunchKernelGGL((k_fill_lfg<R, SL, kOutF32>), dim3(blocks), block, 0, st, g->d_state, g->S, count, out, ring);
    else hipLaunchKernelGGL((k_fill_lfg<R, SL, kOutXor>), dim3(blocks), block, 0, st, g->d_state, g->S, count, out, static_cast<uint32_t *>(nullptr));
    return hipGetLastError();
}

}  // namespace

int lfg_lag_r(rngx_kind kind) { return kind == RNGX_LFG521 ? 521 : 1279; }
int lfg_lag_s(rngx_kind kind) { return kind == RNGX_LFG521 ? 353 : 861; }

hipError_t launch_seed_lfg(Gen *g, uint64_t seed, hipStream_t st) {
    const uint64_t G = g->S / 1024;
    if (g->kind == RNGX_LFG521) {
        hipLaunchKernelGGL(k_seed_lfg<521>, dim3(static_cast<unsigned>((G * 261 + 255) / 256)), dim3(256), 0, st,
                           g->d_state, G, seed);
        hipLaunchKernelGGL(k_seed_lfg_odd<521>, dim3(static_cast<unsigned>(G)), dim3(64), 0, st, g->d_state);
    } else {
        hipLaunchKernelGGL(k_seed_lfg<1279>, dim3(static_cast<unsigned>((G * 640 + 255) / 256)), dim3(256), 0, st,
                           g->d_state, G, seed);
        hipLaunchKernelGGL(k_seed_lfg_odd<1279>, dim3(static_cast<unsigned>(G)), dim3(64), 0, st, g->d_state);
    }
    return hipGetLastError();
}

hipError_t launch_fill_lfg(Gen *g, void *out, uint64_t count, int mode, hipStream_t st) {
    return g->kind == RNGX_LFG521 ? fill_lfg<521, 353>(g, out, count, mode, st)
                                  : fill_lfg<1279, 861>(g, out, count, mode, st);
}

// Jump every instance by n rows (1024 n values); synchronous (the
// polynomial is staged through the handle's auxiliary device buffer).
hipError_t launch_skip_lfg(Gen *g, uint64_t n, hipStream_t st) {
    const int r = lfg_lag_r(g->kind), s = lfg_lag_s(g->kind);
    const LfgPoly P{r, s};
    const auto &tab = row_powers(r, s);
    std::vector<uint32_t> J(r, 0), T;
    J[0] = 1;
    for (int i = 0; i < 64; ++i)
        if ((n >> i) & 1) { P.mulmod(J, tab[i], &T); J.swap(T); }
    hipError_t e = hipMemcpyAsync(g->d_aux, J.data(), 4ull * r, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>(g->S / 1024)), block(1024);
    if (g->kind == RNGX_LFG521) hipLaunchKernelGGL((k_skip_lfg<521, 353>), grid, block, 0, st, g->d_state, g->d_aux);
    else hipLaunchKernelGGL((k_skip_lfg<1279, 861>), grid, block, 0, st, g->d_state, g->d_aux);
    e = hipGetLastError();
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
}

}  // namespace rngx
