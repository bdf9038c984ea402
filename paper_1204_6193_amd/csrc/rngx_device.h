// Device-side definitions of the rngx generators: constants, the per-stream
// generator steps, the XS1024W lane-row step and jump helpers, and the fill
// pacing constants.  Shared by the HIP translation units; holds no handle types.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

// Fill pacing (see k_fill_xs).
constexpr uint32_t kBand = 8;         // rows per band
constexpr uint32_t kSlack = 3;        // bands a workgroup may run ahead of the slowest
constexpr uint32_t kRing = 32;        // band entries in the counter ring
constexpr uint32_t kPaceSlots = 256;  // counters per entry (a multiple of 64)
constexpr uint32_t kPollLimit = 4096; // polls before a workgroup stops waiting

enum { kOutU32 = 0, kOutF32 = 1, kOutXor = 2 };

// a ^ b ^ c as one gfx950 three-input bit operation (truth table 0x96 is
// the three-way xor); the compiler does not fuse chained xors by itself.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}


// Pacing of a fill's workgroups in bands of kBand rows (see k_fill_xs).
// before(b): wait (bounded) until every workgroup has finished band
// b - kSlack; after(b): count this workgroup's band b.  A workgroup whose wait
// times out stops waiting for the rest of the launch but keeps counting.
// Every thread of the workgroup must call both (they contain barriers).
struct Pacer {
    uint32_t *ring;  // null: not paced (before() and after() do nothing)
    bool waiting;    // false once a wait timed out, and always without a ring
    __device__ explicit Pacer(uint32_t *r) : ring(r), waiting(r != nullptr) {}
    __device__ void before(uint64_t band, uint32_t *s_free) {
        if (!ring || !waiting || band < kSlack) return;
        const uint32_t nblk = gridDim.x;
        if (threadIdx.x < 64) {
            const uint64_t prev = band - kSlack;
            const uint32_t *e = ring + (prev % kRing) * kPaceSlots;
            const uint32_t use = static_cast<uint32_t>(prev / kRing) + 1;
            uint32_t it = 0;
            for (; it < kPollLimit; ++it) {
                bool ok = true;
#pragma unroll
                for (uint32_t m = 0; m < kPaceSlots / 64; ++m) {
                    const uint32_t j = m * 64 + threadIdx.x;
                    const uint32_t want = (nblk / kPaceSlots + (j < nblk % kPaceSlots ? 1u : 0u)) * use;
                    ok &= __hip_atomic_load(e + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want;
                }
                if (__all(ok)) break;
                __builtin_amdgcn_s_sleep(1);
            }
            if (threadIdx.x == 0) *s_free = it == kPollLimit;
        }
        __syncthreads();
        if (*s_free) waiting = false;
    }
    __device__ void after(uint64_t band) {
        if (!ring) return;
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(ring + (band % kRing) * kPaceSlots + blockIdx.x % kPaceSlots, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
};


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

// n-step map of x -> a x + c modulo 2^64 (also right modulo 2^32 in its low
// words), by repeated squaring.
__host__ __device__ inline void affine_power(uint64_t a, uint64_t c, uint64_t n, uint64_t *A, uint64_t *C) {
    uint64_t ra = 1, rc = 0;
    for (; n; n >>= 1) {
        if (n & 1) { rc = a * rc + c; ra = a * ra; }
        c = a * c + c;
        a = a * a;
    }
    *A = ra;
    *C = rc;
}

// Sub-stream LCGs (eq. lcg_skipping with t = S): every stream steps S
// positions of one global sequence with the S-step map (A, C), kept after the
// S states in the image (u32 pair for LCG32, u64 pair for LCG64).
struct Lcg32Sub {
    uint32_t x, A, C;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t s) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        x = p[s]; A = p[S]; C = p[S + 1];
    }
    __device__ void store(uint8_t *st, uint64_t, uint64_t s) const { reinterpret_cast<uint32_t *>(st)[s] = x; }
    __device__ uint32_t next() { x = A * x + C; return x; }
};

struct Lcg64Sub {
    uint64_t x, A, C;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t s) {
        const uint64_t *p = reinterpret_cast<const uint64_t *>(st);
        x = p[s]; A = p[S]; C = p[S + 1];
    }
    __device__ void store(uint8_t *st, uint64_t, uint64_t s) const { reinterpret_cast<uint64_t *>(st)[s] = x; }
    __device__ uint32_t next() { x = A * x + C; return static_cast<uint32_t>(x >> 32); }
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

// Arithmetic modulo an odd n < 2^64 by Montgomery multiplication with
// R = 2^64: values are kept as x R mod n, and mul(a, b) = a b / R mod n for
// a, b < n.  Used where the modulus differs per stream (MWC_DIFF) and by the
// primality test of the multiplier search.
__device__ __forceinline__ uint64_t mul_hi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }
struct Mont64 {
    uint64_t n, ninv, one;  // ninv = -n^-1 mod 2^64; one = R mod n (the form of 1)
    __device__ explicit Mont64(uint64_t n_) : n(n_) {
        uint64_t x = n;                               // n^-1 mod 2^3 (n odd)
        for (int i = 0; i < 5; ++i) x *= 2 - n * x;  // Newton: 6, 12, 24, 48, 96 bits
        ninv = 0 - x;
        one = (0 - n) % n;                            // 2^64 mod n
    }
    // a b / R mod n (REDC of the 128-bit product)
    __device__ uint64_t mul(uint64_t a, uint64_t b) const {
        const uint64_t lo = a * b, hi = mul_hi64(a, b);
        const uint64_t m = lo * ninv;
        const uint64_t mlo = m * n, mhi = mul_hi64(m, n);
        const uint64_t c = (lo + mlo) < lo ? 1 : 0;  // the low word sums to 0 mod 2^64
        const uint64_t t1 = hi + mhi, t2 = t1 + c;
        const bool over = (t1 < hi) || (t2 < t1);     // the sum reached 2^64
        return (over || t2 >= n) ? t2 - n : t2;
    }
    __device__ uint64_t add(uint64_t a, uint64_t b) const {  // a + b mod n, a, b < n
        const uint64_t t = a + b;
        return (t < a || t >= n) ? t - n : t;
    }
    // Montgomery form of x < n: x R mod n, as x doubled 64 times modulo n
    __device__ uint64_t to(uint64_t x) const {
        for (int i = 0; i < 64; ++i) x = add(x, x);
        return x;
    }
    __device__ uint64_t from(uint64_t x) const { return mul(x, 1); }
    // b^e in Montgomery form, b in Montgomery form
    __device__ uint64_t pow(uint64_t b, uint64_t e) const {
        uint64_t r = one;
        for (; e; e >>= 1) {
            if (e & 1) r = mul(r, b);
            b = mul(b, b);
        }
        return r;
    }
};

// MWC with a multiplier a of its own per stream (image: u64 y[S], u32 a[S]).
struct MwcDiff {
    uint64_t y;  // carry << 32 | x
    uint32_t a;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t s) {
        y = reinterpret_cast<const uint64_t *>(st)[s];
        a = reinterpret_cast<const uint32_t *>(st + 8 * S)[s];
    }
    __device__ void store(uint8_t *st, uint64_t, uint64_t s) const { reinterpret_cast<uint64_t *>(st)[s] = y; }
    __device__ uint32_t next() {
        y = static_cast<uint64_t>(a) * static_cast<uint32_t>(y) + (y >> 32);
        return static_cast<uint32_t>(y);
    }
};

// y <- a^n y mod p with p = a 2^32 - 1: n steps of the MWC as the
// multiplicative congruential map it is (y = carry 2^32 + x, y' = a y mod p).
__device__ inline uint64_t mwc_jump_mod(uint64_t y, uint32_t a, uint64_t n) {
    const Mont64 M((static_cast<uint64_t>(a) << 32) - 1);
    const uint64_t an = M.pow(M.to(a), n);
    return M.from(M.mul(an, M.to(y)));
}

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
        v = xor3(v, v << 4, t ^ (t << 1));
        d += kWeylC;
        return d + v;
    }
};

// One Philox4x32 round on (x0, x1, x2, x3) with round key (k0, k1).
__device__ __forceinline__ void philox_round(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3, uint32_t k0,
                                             uint32_t k1) {
    const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * x0;
    const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * x2;
    const uint32_t n0 = xor3(static_cast<uint32_t>(p1 >> 32), x1, k0);
    const uint32_t n2 = xor3(static_cast<uint32_t>(p0 >> 32), x3, k1);
    x1 = static_cast<uint32_t>(p1);
    x3 = static_cast<uint32_t>(p0);
    x0 = n0; x2 = n2;
}

// Philox4x32-R block function on counter (lo, hi, 0, 0) with key (k0, k1);
// R = 10, or 7 for the faster variant of the counter-based section.
template <int ROUNDS = 10>
__device__ inline void philox_block(uint32_t k0, uint32_t k1, uint64_t blk, uint32_t &o0, uint32_t &o1,
                                    uint32_t &o2, uint32_t &o3) {
    uint32_t x0 = static_cast<uint32_t>(blk), x1 = static_cast<uint32_t>(blk >> 32), x2 = 0, x3 = 0;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        philox_round(x0, x1, x2, x3, k0, k1);
        k0 += kPhiloxW0; k1 += kPhiloxW1;
    }
    o0 = x0; o1 = x1; o2 = x2; o3 = x3;
}

// Blocks blk and blk + 1 of one key side by side, sharing the key schedule:
// o[0..3] and o[4..7] are the two blocks' words.
template <int ROUNDS = 10>
__device__ inline void philox_block2(uint32_t k0, uint32_t k1, uint64_t blk, uint32_t (&o)[8]) {
    const uint64_t nb = blk + 1;
    uint32_t x0 = static_cast<uint32_t>(blk), x1 = static_cast<uint32_t>(blk >> 32), x2 = 0, x3 = 0;
    uint32_t y0 = static_cast<uint32_t>(nb), y1 = static_cast<uint32_t>(nb >> 32), y2 = 0, y3 = 0;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        philox_round(x0, x1, x2, x3, k0, k1);
        philox_round(y0, y1, y2, y3, k0, k1);
        k0 += kPhiloxW0; k1 += kPhiloxW1;
    }
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
    o[4] = y0; o[5] = y1; o[6] = y2; o[7] = y3;
}

template <int ROUNDS>
struct PhiloxR {
    uint32_t k0, k1, b0, b1, b2, b3;
    uint64_t pos;
    __device__ void load(const uint8_t *st, uint64_t S, uint64_t s) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(st);
        k0 = p[s]; k1 = p[S + s];
        pos = reinterpret_cast<const uint64_t *>(st + 8 * S)[s];
        if (pos & 3) philox_block<ROUNDS>(k0, k1, pos >> 2, b0, b1, b2, b3);  // resume mid-block
    }
    __device__ void store(uint8_t *st, uint64_t S, uint64_t s) const {
        reinterpret_cast<uint64_t *>(st + 8 * S)[s] = pos;
    }
    __device__ uint32_t next() {
        const uint32_t j = static_cast<uint32_t>(pos) & 3;
        if (j == 0) philox_block<ROUNDS>(k0, k1, pos >> 2, b0, b1, b2, b3);
        ++pos;
        return j == 0 ? b0 : j == 1 ? b1 : j == 2 ? b2 : b3;
    }
    // The next 8 outputs.  From a block boundary these are two whole blocks,
    // made together; elsewhere they are 8 calls of next().
    __device__ void next8(uint32_t (&u)[8]) {
        if ((pos & 3) == 0) {
            philox_block2<ROUNDS>(k0, k1, pos >> 2, u);
            pos += 8;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) u[j] = next();
        }
    }
};
// Generators with next8() (outputs made 8 at a time).
template <class G> struct HasNext8 : std::false_type {};
template <int ROUNDS> struct HasNext8<PhiloxR<ROUNDS>> : std::true_type {};
using Philox = PhiloxR<10>;
using Philox7 = PhiloxR<7>;

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
// Each term a lane xors in is a funnel of two words of one other lane (5 to
// the right or left), so that lane's own funnel is made first and moved by a
// row shift: the shift then rides on the xor (a DPP operand of v_xor_b32)
// instead of being a separate move of each input word.
__device__ __forceinline__ void xs1024_step(uint32_t &a, uint32_t &b) {
    // << 329 = 10 words + 9 bits: W[i] ^= W[i+10] << 9 | W[i+11] >> 23
    uint32_t ta = funnel(a, b, 23), tb = funnel(b, from_lane_plus<1>(a), 23);
    a ^= from_lane_plus<5>(ta);
    b ^= from_lane_plus<5>(tb);
    // >> 347 = 10 words + 27 bits: W[i] ^= W[i-11] << 5 | W[i-10] >> 27
    ta = funnel(from_lane_minus<1>(b), a, 27);
    tb = funnel(a, b, 27);
    a ^= from_lane_minus<5>(ta);
    b ^= from_lane_minus<5>(tb);
    // << 344 = 10 words + 24 bits: W[i] ^= W[i+10] << 24 | W[i+11] >> 8
    ta = funnel(a, b, 8);
    tb = funnel(b, from_lane_plus<1>(a), 8);
    a ^= from_lane_plus<5>(ta);
    b ^= from_lane_plus<5>(tb);
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
        acc[4] = xor3(acc[4], acc[4] << 4, t ^ (t << 1));
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
template <int ROUNDS>
__device__ __forceinline__ void jump(PhiloxR<ROUNDS> &g, const uint64_t *, const uint32_t *, uint64_t j, uint64_t C) {
    g.pos += j * C;
    if (g.pos & 3) philox_block<ROUNDS>(g.k0, g.k1, g.pos >> 2, g.b0, g.b1, g.b2, g.b3);  // resume mid-block
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
