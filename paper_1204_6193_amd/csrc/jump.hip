// Jump-ahead: advance every stream by n outputs without producing them.
//
// LCG (eq. lcg_skipping): the n-step map is affine, x -> A_n x + C_n, with
//   (A_n, C_n) from repeated squaring of the one-step map (x -> a x + c).
// MWC: with y = carry 2^32 + x one step is y -> a y mod p, p = a 2^32 - 1, so
//   the n-step map is y -> (a^n mod p) y mod p.
// XORWOW / XS1024W: the xorshift parts are GF(2)-linear with transition
//   matrix M (XORShift section).  M^n = J(M) with J(x) = x^n mod P(x), P the
//   minimal polynomial of M (degree 160 resp. 1024, found once on the host by
//   Berlekamp-Massey from a bit of the state sequence).  The device evaluates
//   J(M) v by Horner's rule, i.e. deg(P) generator steps per stream, instead
//   of the paper's product with a stored 1024 x 1024 bit matrix.  The Weyl
//   parts advance in closed form (d += n c; the XS1024W step counter += n).
// Philox: the position advances by n.
#include <mutex>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kBlock = 256;

// ----------------------------------------------------------------- host GF(2)
using Poly = std::vector<uint64_t>;  // bit i = coefficient of x^i

int poly_deg(const Poly &p) {
    for (int w = static_cast<int>(p.size()) - 1; w >= 0; --w)
        if (p[w]) return 64 * w + 63 - __builtin_clzll(p[w]);
    return -1;
}
bool poly_bit(const Poly &p, int i) { return (p[i / 64] >> (i % 64)) & 1u; }
void poly_flip(Poly &p, int i) { p[i / 64] ^= 1ull << (i % 64); }

// r ^= p << sh
void poly_xor_shifted(Poly &r, const Poly &p, int sh) {
    const int ws = sh / 64, bs = sh % 64;
    for (size_t w = 0; w < p.size(); ++w) {
        if (!p[w]) continue;
        if (w + ws < r.size()) r[w + ws] ^= p[w] << bs;
        if (bs && w + ws + 1 < r.size()) r[w + ws + 1] ^= p[w] >> (64 - bs);
    }
}

// a mod P, with a of any length; result has P's word count.
Poly poly_mod(Poly a, const Poly &P) {
    const int d = poly_deg(P);
    for (int i = poly_deg(a); i >= d; --i)
        if (poly_bit(a, i)) poly_xor_shifted(a, P, i - d);
    Poly r(P.size(), 0);
    for (size_t w = 0; w < r.size() && w < a.size(); ++w) r[w] = a[w];
    return r;
}

Poly poly_square(const Poly &a) {  // the cross terms vanish over GF(2)
    Poly r(2 * a.size(), 0);
    for (size_t w = 0; w < a.size(); ++w)
        for (int i = 0; i < 64; ++i)
            if ((a[w] >> i) & 1u) r[(128 * w + 2 * i) / 64] |= 1ull << ((128 * w + 2 * i) % 64);
    return r;
}

// x^n mod P, left-to-right: square, then multiply by x when the bit is set.
Poly x_pow_mod(uint64_t n, const Poly &P) {
    Poly r(P.size(), 0);
    r[0] = 1;
    const int d = poly_deg(P);
    for (int bit = 63; bit >= 0; --bit) {
        r = poly_mod(poly_square(r), P);
        if ((n >> bit) & 1u) {
            Poly s(P.size() + 1, 0);
            poly_xor_shifted(s, r, 1);
            r = poly_mod(s, P);
        }
    }
    (void)d;
    return r;
}

// a * b mod P (carry-less product, then reduction).
Poly poly_mulmod(const Poly &a, const Poly &b, const Poly &P) {
    Poly r(a.size() + b.size() + 1, 0);
    for (size_t w = 0; w < a.size(); ++w)
        for (int i = 0; i < 64; ++i)
            if ((a[w] >> i) & 1u) poly_xor_shifted(r, b, static_cast<int>(64 * w + i));
    return poly_mod(r, P);
}

// Minimal polynomial of a bit sequence (Berlekamp-Massey), as x^L C(1/x).
Poly berlekamp_massey(const std::vector<uint8_t> &s, int words) {
    const int n = static_cast<int>(s.size());
    std::vector<uint8_t> C(n + 1, 0), B(n + 1, 0), T;
    C[0] = B[0] = 1;
    int L = 0, m = 1;
    for (int i = 0; i < n; ++i) {
        uint8_t d = s[i];
        for (int j = 1; j <= L; ++j) d ^= C[j] & s[i - j];
        if (!d) { ++m; continue; }
        T = C;
        for (int j = 0; j + m <= n; ++j) C[j + m] ^= B[j];
        if (2 * L <= i) { L = i + 1 - L; B = T; m = 1; } else { ++m; }
    }
    Poly P(words, 0);
    for (int i = 0; i <= L; ++i)
        if (C[i]) poly_flip(P, L - i);
    return P;
}

// Host copies of the two GF(2)-linear steps (used only to find P).
void host_xs1024_step(uint32_t *W) {
    auto shl = [](const uint32_t *in, int q, int r, uint32_t *out) {
        for (int i = 0; i < 32; ++i) {
            uint32_t hi = i + q < 32 ? in[i + q] : 0, lo = i + q + 1 < 32 ? in[i + q + 1] : 0;
            out[i] = (hi << r) | (lo >> (32 - r));
        }
    };
    auto shr = [](const uint32_t *in, int q, int r, uint32_t *out) {
        for (int i = 0; i < 32; ++i) {
            uint32_t lo = i - q >= 0 ? in[i - q] : 0, hi = i - q - 1 >= 0 ? in[i - q - 1] : 0;
            out[i] = (lo >> r) | (hi << (32 - r));
        }
    };
    uint32_t t[32];
    shl(W, 10, 9, t);
    for (int i = 0; i < 32; ++i) W[i] ^= t[i];
    shr(W, 10, 27, t);
    for (int i = 0; i < 32; ++i) W[i] ^= t[i];
    shl(W, 10, 24, t);
    for (int i = 0; i < 32; ++i) W[i] ^= t[i];
}

void host_xorwow_step(uint32_t *s) {
    uint32_t t = s[0] ^ (s[0] >> 2);
    s[0] = s[1]; s[1] = s[2]; s[2] = s[3]; s[3] = s[4];
    s[4] = (s[4] ^ (s[4] << 4)) ^ (t ^ (t << 1));
}

const Poly &xs1024_minpoly() {
    static Poly P;
    static std::once_flag once;
    std::call_once(once, [] {
        uint32_t W[32];
        for (int i = 0; i < 32; ++i) W[i] = static_cast<uint32_t>(splitmix(12345, i + 1));
        for (int bit = 0;; ++bit) {
            std::vector<uint8_t> seq(2 * 1024 + 64);
            uint32_t V[32];
            for (int i = 0; i < 32; ++i) V[i] = W[i];
            for (auto &x : seq) { host_xs1024_step(V); x = (V[31 - bit / 32] >> (bit % 32)) & 1u; }
            P = berlekamp_massey(seq, 17);
            if (poly_deg(P) == 1024) break;
        }
    });
    return P;
}

const Poly &xorwow_minpoly() {
    static Poly P;
    static std::once_flag once;
    std::call_once(once, [] {
        uint32_t W[5];
        for (int i = 0; i < 5; ++i) W[i] = static_cast<uint32_t>(splitmix(777, i + 1));
        for (int bit = 0;; ++bit) {
            std::vector<uint8_t> seq(2 * 160 + 64);
            uint32_t V[5];
            for (int i = 0; i < 5; ++i) V[i] = W[i];
            for (auto &x : seq) { host_xorwow_step(V); x = (V[4 - bit / 32] >> (bit % 32)) & 1u; }
            P = berlekamp_massey(seq, 3);
            if (poly_deg(P) == 160) break;
        }
    });
    return P;
}

// ---------------------------------------------------------------- kernels
struct JumpPoly1024 { uint32_t c[32]; };  // coefficient i at bit i%32 of c[i/32]
struct JumpPoly160 { uint32_t c[5]; };


__global__ __launch_bounds__(kBlock) void k_skip_affine32(uint32_t *x, uint64_t S, uint32_t A, uint32_t C) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s < S) x[s] = A * x[s] + C;
}
__global__ __launch_bounds__(kBlock) void k_skip_affine64(uint64_t *x, uint64_t S, uint64_t A, uint64_t C) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s < S) x[s] = A * x[s] + C;
}

__global__ __launch_bounds__(kBlock) void k_skip_mwc(uint64_t *y, uint64_t S, uint64_t A) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s < S) y[s] = mwc_mulmod(y[s], A);
}

__global__ __launch_bounds__(kBlock) void k_skip_philox(uint64_t *pos, uint64_t S, uint64_t n) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s < S) pos[s] += n;
}

__global__ __launch_bounds__(kBlock) void k_skip_xorwow(uint32_t *st, uint64_t S, JumpPoly160 J, uint32_t dAdd) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint32_t v[5];
    for (int i = 0; i < 5; ++i) v[i] = st[i * S + s];
    xorwow_apply_poly(J.c, v);
    for (int i = 0; i < 5; ++i) st[i * S + s] = v[i];
    st[5 * S + s] += dAdd;
}

__global__ __launch_bounds__(kBlock) void k_skip_xs(uint8_t *st, uint64_t S, JumpPoly1024 J, uint64_t n) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t G = S / 32, g = t >> 4;
    if (g >= G) return;  // whole 16-lane rows
    uint2 *W = reinterpret_cast<uint2 *>(st);
    const uint2 w = W[t];
    uint32_t a = w.x, b = w.y;
    xs1024_apply_poly(J.c, a, b);
    W[t] = make_uint2(a, b);
    if ((t & 15) == 0) reinterpret_cast<uint64_t *>(st + 4 * S)[g] += n;
}

// Sub-stream seeding (XORShift section): instance g (g >= 1) takes instance
// 0's xorshift words and skips g * 2^137 steps, applying x^(2^(137+i)) mod P
// (polys[32 i ..], coefficient j at bit j%32 of word j/32) for every set bit
// i of g by Horner's rule.  Instance 0 is only read.  The step counters stay
// as seeded: g * 2^137 is 0 modulo 2^64.
__global__ __launch_bounds__(kBlock) void k_substreams_xs(uint8_t *st, uint64_t S, const uint32_t *polys,
                                                           uint32_t nbits) {
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t G = S / 32, g = t >> 4, lane = t & 15;
    if (g >= G || g == 0) return;  // whole 16-lane rows
    uint2 *W = reinterpret_cast<uint2 *>(st);
    const uint2 w = W[lane];
    uint32_t a = w.x, b = w.y;
    for (uint32_t i = 0; i < nbits; ++i)
        if ((g >> i) & 1) xs1024_apply_poly(polys + 32 * i, a, b);
    W[t] = make_uint2(a, b);
}

struct Aff { uint64_t a, c; };
Aff aff_after(Aff f, Aff g) { return {f.a * g.a, f.a * g.c + f.c}; }
Aff aff_pow(Aff f, uint64_t n) {
    Aff r{1, 0};
    while (n) { if (n & 1) r = aff_after(f, r); f = aff_after(f, f); n >>= 1; }
    return r;
}

uint64_t host_powmod_p(uint64_t a, uint64_t n) {
    unsigned __int128 r = 1, b = a;
    while (n) { if (n & 1) r = (r * b) % kMwcP; b = (b * b) % kMwcP; n >>= 1; }
    return static_cast<uint64_t>(r);
}

unsigned blocks_for(uint64_t threads) { return static_cast<unsigned>((threads + kBlock - 1) / kBlock); }

template <int NBITS>
void poly_table(const Poly &P, uint64_t step, uint64_t count, std::vector<uint32_t> *out) {
    constexpr int NW = NBITS / 32;
    out->assign(count * NW, 0);
    const Poly xs = x_pow_mod(step, P);
    Poly cur(P.size(), 0);
    cur[0] = 1;  // x^0
    for (uint64_t j = 0; j < count; ++j) {
        for (int i = 0; i < NBITS; ++i)
            if (poly_bit(cur, i)) (*out)[j * NW + i / 32] |= 1u << (i % 32);
        cur = poly_mulmod(cur, xs, P);
    }
}

}  // namespace

void jump_table(rngx_kind kind, uint64_t step, uint64_t count, std::vector<uint64_t> *u64s,
                std::vector<uint32_t> *u32s) {
    u64s->clear();
    u32s->clear();
    switch (kind) {
    case RNGX_LCG32:
    case RNGX_LCG64: {
        const Aff f = kind == RNGX_LCG32 ? Aff{kLcg32A, kLcg32C} : Aff{kLcg64A, kLcg64C};
        const Aff fs = aff_pow(f, step);
        Aff cur{1, 0};
        for (uint64_t j = 0; j < count; ++j) {
            u64s->push_back(cur.a);
            u64s->push_back(cur.c);
            cur = aff_after(fs, cur);
        }
        break;
    }
    case RNGX_MWC: {
        const unsigned __int128 as = host_powmod_p(kMwcA, step);
        unsigned __int128 cur = 1;
        for (uint64_t j = 0; j < count; ++j) {
            u64s->push_back(static_cast<uint64_t>(cur));
            cur = (cur * as) % kMwcP;
        }
        break;
    }
    case RNGX_XORWOW: poly_table<160>(xorwow_minpoly(), step, count, u32s); break;
    case RNGX_XS1024W: poly_table<1024>(xs1024_minpoly(), step, count, u32s); break;
    case RNGX_PHILOX4X32_7:
    case RNGX_PHILOX4X32_10:
    case RNGX_MWC_DIFF: break;  // counter; per-stream powers computed on the device
    default: break;
    }
}

void jump_table_gen(const Gen *g, uint64_t step, uint64_t count, std::vector<uint64_t> *u64s,
                    std::vector<uint32_t> *u32s) {
    if (!is_sub_lcg(g->kind)) { jump_table(g->kind, step, count, u64s, u32s); return; }
    // sub-stream LCGs: powers of the handle's S-step map
    u64s->clear();
    u32s->clear();
    const Aff fs = aff_pow(Aff{g->sub_a, g->sub_c}, step);
    Aff cur{1, 0};
    for (uint64_t j = 0; j < count; ++j) {
        u64s->push_back(cur.a);
        u64s->push_back(cur.c);
        cur = aff_after(fs, cur);
    }
}

hipError_t launch_skip(Gen *g, uint64_t n, hipStream_t st) {
    const uint64_t S = g->S;
    switch (g->kind) {
    case RNGX_LCG32_SUB: {
        const Aff f = aff_pow({g->sub_a, g->sub_c}, n);  // mod 2^64 reduces correctly mod 2^32
        hipLaunchKernelGGL(k_skip_affine32, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint32_t *>(g->d_state), S, static_cast<uint32_t>(f.a),
                           static_cast<uint32_t>(f.c));
        break;
    }
    case RNGX_LCG64_SUB: {
        const Aff f = aff_pow({g->sub_a, g->sub_c}, n);
        hipLaunchKernelGGL(k_skip_affine64, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint64_t *>(g->d_state), S, f.a, f.c);
        break;
    }
    case RNGX_LCG32: {
        const Aff f = aff_pow({kLcg32A, kLcg32C}, n);  // mod 2^64 reduces correctly mod 2^32
        hipLaunchKernelGGL(k_skip_affine32, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint32_t *>(g->d_state), S, static_cast<uint32_t>(f.a),
                           static_cast<uint32_t>(f.c));
        break;
    }
    case RNGX_LCG64: {
        const Aff f = aff_pow({kLcg64A, kLcg64C}, n);
        hipLaunchKernelGGL(k_skip_affine64, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint64_t *>(g->d_state), S, f.a, f.c);
        break;
    }
    case RNGX_MWC_DIFF: return launch_skip_mwc_diff(g, n, st);
    case RNGX_LFG521:
    case RNGX_LFG1279: return launch_skip_lfg(g, n, st);
    case RNGX_MWC:
        hipLaunchKernelGGL(k_skip_mwc, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint64_t *>(g->d_state), S, host_powmod_p(kMwcA, n));
        break;
    case RNGX_PHILOX4X32_7:
    case RNGX_PHILOX4X32_10:
        hipLaunchKernelGGL(k_skip_philox, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint64_t *>(g->d_state + 8 * S), S, n);
        break;
    case RNGX_XORWOW: {
        const Poly J = x_pow_mod(n, xorwow_minpoly());
        JumpPoly160 jp{};
        for (int i = 0; i < 160; ++i) if (poly_bit(J, i)) jp.c[i / 32] |= 1u << (i % 32);
        hipLaunchKernelGGL(k_skip_xorwow, dim3(blocks_for(S)), dim3(kBlock), 0, st,
                           reinterpret_cast<uint32_t *>(g->d_state), S, jp,
                           static_cast<uint32_t>(n) * kWeylC);
        break;
    }
    case RNGX_XS1024W: {
        const Poly J = x_pow_mod(n, xs1024_minpoly());
        JumpPoly1024 jp{};
        for (int i = 0; i < 1024; ++i) if (poly_bit(J, i)) jp.c[i / 32] |= 1u << (i % 32);
        hipLaunchKernelGGL(k_skip_xs, dim3(blocks_for(S / 2)), dim3(kBlock), 0, st, g->d_state, S, jp, n);
        break;
    }
    }
    return hipGetLastError();
}

hipError_t launch_substreams(Gen *g, hipStream_t st) {
    const uint64_t G = g->S / 32;
    if (g->kind != RNGX_XS1024W) return hipErrorInvalidValue;
    if (G < 2) return hipSuccess;
    uint32_t nbits = 0;
    while ((G - 1) >> nbits) ++nbits;
    // x^(2^137) mod P by 137 squarings, then one more squaring per bit
    const Poly &P = xs1024_minpoly();
    Poly J(P.size(), 0);
    J[0] = 2;  // x
    for (int k = 0; k < 137; ++k) J = poly_mod(poly_square(J), P);
    std::vector<uint32_t> words(32ull * nbits, 0);
    for (uint32_t i = 0; i < nbits; ++i) {
        for (int j = 0; j < 1024; ++j)
            if (poly_bit(J, j)) words[32ull * i + j / 32] |= 1u << (j % 32);
        J = poly_mod(poly_square(J), P);
    }
    uint32_t *d_polys = nullptr;
    hipError_t e = hipMalloc(&d_polys, 4 * words.size());
    if (e == hipSuccess) e = hipMemcpyAsync(d_polys, words.data(), 4 * words.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_substreams_xs, dim3(blocks_for(16 * G)), dim3(kBlock), 0, st, g->d_state, g->S, d_polys,
                           nbits);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_polys);
    return e;
}

}  // namespace rngx
