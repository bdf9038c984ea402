/*
 * CPU oracle: plain, serial definitions of the per-stream generators, their
 * seeding, jump-ahead and the checkerboard Metropolis update of the 2D Ising
 * ferromagnet.
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  The HIP library never links,
 * includes or calls anything here, and nothing here comes from the HIP
 * library: the two are written independently from the paper
 * (Manssen, Weigel, Hartmann, "Random number generators for massively
 * parallel simulations on GPU") and from the published definitions cited
 * below.
 *
 * Parity status of each function is stated in its comment; the pins live in
 * tests/test_oracle_*.py.  Philox4x32-10's round constants and XORWOW's
 * shift triple come from their original publications; they are pinned by
 * the published Philox known-answer vectors and by an independent
 * implementation (rocRAND's source headers, compiled for the host by the
 * tests).
 *
 * Conventions (project definitions where the paper is silent):
 *   - every recursive generator steps first and then outputs, so output #0
 *     is the value after one step;
 *   - a "stream" is one per-thread sequence of 32-bit outputs; for the
 *     XORShift-1024/Weyl generator a stream is one 32-bit word (one lane) of
 *     a 1024-bit instance, and the 32 lanes of an instance step together;
 *   - the canonical state image (orc_state_bytes) is structure-of-arrays:
 *       LCG32    u32 x[S]
 *       LCG64    u64 x[S]
 *       MWC      u64 y[S]            (y = carry << 32 | x)
 *       XORWOW   u32 x[S] y[S] z[S] w[S] v[S] d[S]
 *       PHILOX   u32 k0[S] k1[S]  u64 pos[S]   (pos = outputs consumed)
 *       XS1024W  u32 W[S]  u64 n[S/32]  u32 y0
 *     (XS1024W: W[32g+i] is word i of instance g, word 0 most significant;
 *      n[g] is the instance's step counter; y0 the shared Weyl seed.)
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_LCG32 = 1, ORC_LCG64, ORC_MWC, ORC_XORWOW, ORC_PHILOX, ORC_XS1024W, ORC_PHILOX7, ORC_LCG32S, ORC_LCG64S,
       ORC_LFG521, ORC_LFG1279, ORC_MWCD };
/* MWC with a different multiplier per stream (MWC section: multipliers found
 * by working downward from 4294967118, keeping every a for which a*2^32 - 1
 * and (a*2^32 - 2)/2 are both prime, tested with Rabin-Miller).  Stream s
 * uses a_s, the (s+1)-th largest such a below 2^32.  Image: u64 y[S] (carry
 * << 32 | x, as MWC), then u32 a[S]; seeding as MWC with the carry reduced
 * mod (a_s - 1).  At most 2^21 streams (all a_s stay above 2^31). */
#define MWCD_MAX_STREAMS (1ull << 21)
/* Additive lagged Fibonacci generators (Lagged Fibonacci section, eq.
 * used_fibonacci): u_n = u_{n-r} + u_{n-s} mod 1 with (r, s) = (521, 353) or
 * (1279, 861).  The values are u_n = x_n / 2^32 with 32-bit words x_n, so the
 * mod-1 addition is exact: x_n = x_{n-r} + x_{n-s} mod 2^32 (m = 2^32 in the
 * section's general form), output x_n.  An instance is one such sequence,
 * shared by the threads of a block; its LFG_W lanes are the streams: stream
 * s is lane s % LFG_W of instance s / LFG_W, and output k of lane i is
 * x_{k*LFG_W + i} of the instance's outputs (warp order, as for XS1024W).
 * Image: u32 X[G][r], X[g][j] = x_{n-r+j} of instance g (its last r values,
 * oldest first).  Seeding: X[g][j] = low32 (j even) / high32 (j odd) of
 * SM(1 + H*g + j/2), H = (r+1)/2; if every word is even, X[g][0] |= 1 (an
 * all-even start keeps the low bits zero forever). */
#define IS_LFG(kind) ((kind) == ORC_LFG521 || (kind) == ORC_LFG1279)
#define LFG_W 1024
#define LFG_R(kind) ((kind) == ORC_LFG521 ? 521 : 1279)
#define LFG_S(kind) ((kind) == ORC_LFG521 ? 353 : 861)
/* Sub-stream LCGs (LCG section, eq. lcg_skipping with t = S): the S streams
 * share one global sequence g_0 = the plain seeding's stream-0 value,
 * g_{n+1} = a g_n + c.  Stream s starts at g_s and steps S positions at a
 * time with the S-step map (A_S, C_S), so output k of stream s is
 * g_{s + (k+1) S}: an interleaved fill out[k S + s] is the global sequence
 * from position S on.  Image: x[S], then A_S and C_S (u32 for LCG32, u64 for
 * LCG64). */
/* Philox4x32 with 10 rounds (ORC_PHILOX) or 7 (ORC_PHILOX7); everything but the
 * round count is shared. */
#define IS_PHILOX(kind) ((kind) == ORC_PHILOX || (kind) == ORC_PHILOX7)
#define PHILOX_R(kind) ((kind) == ORC_PHILOX7 ? 7 : 10)
enum { ORC_OUT_U32 = 0, ORC_OUT_F32 = 1, ORC_OUT_XOR = 2 };

/* ------------------------------------------------------------------------ */
/* splitmix64 (Steele, Lea & Flood 2014): the paper only asks that instances
 * be seeded "with another RNG" (Sec. 2 and the XORShift section); this is
 * the seeding generator chosen for that.  SM(k) = mix64(seed + k*gamma) is
 * the k-th output of the sequential generator started at `seed`. */
#define SM_GAMMA 0x9E3779B97F4A7C15ull

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix(uint64_t seed, uint64_t k) { return orc_mix64(seed + k * SM_GAMMA); }

/* ------------------------------------------------------------------------ */
/* Generator constants. */
/* LCG32, Sec. 2: a = 1664525, c = 1013904223, m = 2^32. */
#define LCG32_A 1664525u
#define LCG32_C 1013904223u
/* LCG64, Sec. 2: a = 2862933555777941757, c = 1442695040888963407, m = 2^64;
 * only the 32 most significant bits are output. */
#define LCG64_A 2862933555777941757ull
#define LCG64_C 1442695040888963407ull
/* MWC, Sec. 3: lag 1, base 2^32, a = 4294967118. */
#define MWC_A 4294967118ull
/* Weyl increment, XORShift section (same as XORWOW's): c = 362437. */
#define WEYL_C 362437u
/* Philox4x32 (Salmon et al. 2011): multipliers and key increments. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u
/* XORShift-1024 shifts, XORShift section: a = 329 (left), b = 347 (right),
 * c = 344 (left) on a 1024-bit word. */
#define XS_A 329u
#define XS_B 347u
#define XS_C 344u
#define XS_WORDS 32

/* ------------------------------------------------------------------------ */
/* Canonical state image. */
size_t orc_state_bytes(int kind, uint64_t S)
{
    switch (kind) {
    case ORC_LCG32: return 4 * S;
    case ORC_LCG64: return 8 * S;
    case ORC_LCG32S: return 4 * S + 8;
    case ORC_LCG64S: return 8 * S + 16;
    case ORC_MWC: return 8 * S;
    case ORC_XORWOW: return 24 * S;
    case ORC_PHILOX:
    case ORC_PHILOX7: return 16 * S;
    case ORC_XS1024W: return 4 * S + 8 * (S / 32) + 4;
    case ORC_LFG521:
    case ORC_LFG1279: return 4 * (uint64_t)LFG_R(kind) * (S / LFG_W);
    case ORC_MWCD: return 12 * S;
    default: return 0;
    }
}

static int kind_ok(int kind, uint64_t S)
{
    if (kind < ORC_LCG32 || kind > ORC_MWCD) return 0;
    if (kind == ORC_MWCD && S > MWCD_MAX_STREAMS) return 0;
    if (kind == ORC_XS1024W && S % 32 != 0) return 0;
    if (IS_LFG(kind) && S % LFG_W != 0) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* XORShift-1024 on a 32-word big-endian word array: X = sum W[i]*2^(32(31-i)). */

/* out = X << b  (mod 2^1024) */
static void big_shl(const uint32_t *in, unsigned b, uint32_t *out)
{
    unsigned q = b / 32, r = b % 32;
    for (int i = 0; i < XS_WORDS; i++) {
        uint32_t hi = (i + q < XS_WORDS) ? in[i + q] : 0;
        uint32_t lo = (i + q + 1 < XS_WORDS) ? in[i + q + 1] : 0;
        out[i] = r ? (hi << r) | (lo >> (32 - r)) : hi;
    }
}

/* out = X >> b */
static void big_shr(const uint32_t *in, unsigned b, uint32_t *out)
{
    unsigned q = b / 32, r = b % 32;
    for (int i = 0; i < XS_WORDS; i++) {
        int j = i - (int)q;
        uint32_t lo = (j >= 0) ? in[j] : 0;       /* lands in word i unshifted by q */
        uint32_t hi = (j - 1 >= 0) ? in[j - 1] : 0; /* more significant neighbour */
        out[i] = r ? (lo >> r) | (hi << (32 - r)) : lo;
    }
}

/* One step x_n = x_{n-1} (I + L^a)(I + R^b)(I + L^c), eq. (threeshift) with
 * the row-vector convention of the paper, i.e. X ^= X<<a; X ^= X>>b; X ^= X<<c. */
static void xs1024_step(uint32_t *W)
{
    uint32_t t[XS_WORDS];
    big_shl(W, XS_A, t);
    for (int i = 0; i < XS_WORDS; i++) W[i] ^= t[i];
    big_shr(W, XS_B, t);
    for (int i = 0; i < XS_WORDS; i++) W[i] ^= t[i];
    big_shl(W, XS_C, t);
    for (int i = 0; i < XS_WORDS; i++) W[i] ^= t[i];
}

/* The four shift-direction choices sharing the characteristic polynomial of
 * eq. (threeshift) (Sec. XORShift generators, equidistribution paragraph):
 * 0 = L a, R b, L c (the generator above), 1 = R a, L b, R c,
 * 2 = L c, R b, L a, 3 = R c, L b, R a, with (a, b, c) = (329, 347, 344).
 * n steps of variant v on W in place; returns -1 for a bad variant. */
int orc_xs1024_variant_steps(int v, uint32_t *W, uint64_t n)
{
    if (v < 0 || v > 3) return -1;
    const unsigned sh[3] = {v < 2 ? XS_A : XS_C, XS_B, v < 2 ? XS_C : XS_A};
    const int left_first = (v % 2) == 0; /* L R L, else R L R */
    uint32_t t[XS_WORDS];
    for (uint64_t k = 0; k < n; k++)
        for (int j = 0; j < 3; j++) {
            if ((j % 2 == 0) == left_first) big_shl(W, sh[j], t);
            else big_shr(W, sh[j], t);
            for (int i = 0; i < XS_WORDS; i++) W[i] ^= t[i];
        }
    return 0;
}

/* Dimensions of equidistribution of the XORShift-1024 part (the paper tests
 * them as Panneton and L'Ecuyer do, Sec. XORShift generators).  For
 * resolution l (the l most significant bits of each 32-bit output) t_l is
 * the largest t such that the l-bit truncations of t successive outputs are
 * equidistributed: the t*l output bits, as GF(2)-linear functions of the
 * 1024-bit state, are linearly independent (t_l <= 1024/l).  Outputs:
 * lane 0..31 = that word after each step (single-thread order); lane = -1 =
 * the 32 words of each step in order (warp order).  The Weyl term is not
 * GF(2)-linear and is left out.  t_out[l-1] for l = 1..32.  Returns 0, -1 for
 * bad arguments, -3 if memory runs out. */
int orc_xs1024_equidistribution(int v, int lane, int32_t *t_out)
{
    if (v < 0 || v > 3 || lane < -1 || lane > 31) return -1;
    enum { K = 1024, T = 1024, NW64 = K / 64 };
    /* out[k*T + n]: output n of the run started from unit state e_k (bit k of X,
     * counted from the most significant end), so bit j of output n, as a linear
     * function of the start state, is the row (out[k*T + n] >> (31 - j) & 1)_k. */
    uint32_t *out = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K * T);
    uint64_t (*basis)[NW64] = malloc(sizeof(uint64_t) * K * NW64);
    unsigned char *have = malloc(K);
    if (!out || !basis || !have) { free(out); free(basis); free(have); return -3; }
    for (int k = 0; k < K; k++) {
        uint32_t W[XS_WORDS];
        memset(W, 0, sizeof W);
        W[k / 32] = 1u << (31 - k % 32);
        if (lane >= 0) {
            for (int n = 0; n < T; n++) { orc_xs1024_variant_steps(v, W, 1); out[(size_t)k * T + n] = W[lane]; }
        } else {
            for (int n = 0; n < T; n += XS_WORDS) {
                orc_xs1024_variant_steps(v, W, 1);
                for (int i = 0; i < XS_WORDS; i++) out[(size_t)k * T + n + i] = W[i];
            }
        }
    }
    for (int l = 1; l <= 32; l++) {
        memset(have, 0, K);
        int t = 0, dependent = 0;
        for (int n = 0; n < T && !dependent; n++) {
            for (int j = 0; j < l && !dependent; j++) {
                uint64_t row[NW64];
                memset(row, 0, sizeof row);
                for (int k = 0; k < K; k++)
                    if ((out[(size_t)k * T + n] >> (31 - j)) & 1u) row[k / 64] |= 1ull << (k % 64);
                for (;;) { /* reduce against the basis; a zero row is dependent */
                    int p = -1;
                    for (int w = NW64 - 1; w >= 0 && p < 0; w--)
                        if (row[w]) p = 64 * w + 63 - __builtin_clzll(row[w]);
                    if (p < 0) { dependent = 1; break; }
                    if (!have[p]) { memcpy(basis[p], row, sizeof row); have[p] = 1; break; }
                    for (int w = 0; w < NW64; w++) row[w] ^= basis[p][w];
                }
            }
            if (!dependent) t = n + 1;
        }
        t_out[l - 1] = t;
    }
    free(out); free(basis); free(have);
    return 0;
}

/* Weyl sequence, eq. (weylgen) and its closed form y_n = y_0 + n c mod 2^32;
 * combined output y_n (I + R^16) + x (mod 2^32), gamma = w/2 = 16. */
static uint32_t weyl_mix(uint32_t y0, uint64_t n)
{
    uint32_t y = y0 + (uint32_t)n * WEYL_C;
    return y ^ (y >> 16);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-r (Salmon et al. 2011; S-box as in the counter-based section:
 * L' = mullo(R,M), R' = mulhi(R,M) ^ k ^ L), on a full 128-bit counter
 * ctr[0..3] and key key[0..1]; the key is bumped by the Weyl constants
 * before every round but the first.  rounds = 10, or 7 for the faster
 * variant the section also measures.  Pinned by the published known-answer
 * vectors and by rocRAND's engine (tests). */
void orc_philox4x32_block(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < rounds; r++) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Block `block` of a stream with key (k0, k1): counter (block_lo, block_hi, 0, 0). */
static void philox4x32(uint32_t k0, uint32_t k1, uint64_t block, int rounds, uint32_t out[4])
{
    const uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32), 0, 0};
    const uint32_t key[2] = {k0, k1};
    orc_philox4x32_block(ctr, key, rounds, out);
}

/* ------------------------------------------------------------------------ */
/* Rabin-Miller with the first twelve primes as bases: for n < 3.3e24 (all
 * 64-bit n) a composite passes none of them all (Jaeschke 1993; Sorenson and
 * Webster 2015), so the test is exact here. */
static uint64_t mr_mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

static uint64_t mr_powmod(uint64_t b, uint64_t e, uint64_t m)
{
    uint64_t r = 1;
    b %= m;
    for (; e; e >>= 1) {
        if (e & 1) r = mr_mulmod(r, b, m);
        b = mr_mulmod(b, b, m);
    }
    return r;
}

int orc_is_prime_u64(uint64_t n)
{
    static const uint64_t base[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++)
        if (n % base[i] == 0) return n == base[i];
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = mr_powmod(base[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int witness = 1;
        for (int r = 1; r < s && witness; r++) {
            x = mr_mulmod(x, x, n);
            if (x == n - 1) witness = 0;
        }
        if (witness) return 0;
    }
    return 1;
}

/* The n largest multipliers a < 2^32 with a*2^32 - 1 and (a*2^32 - 2)/2
 * prime, in decreasing order (cached between calls); returns 0, or -3. */
static uint32_t *g_mult = NULL;
static uint64_t g_mult_n = 0, g_mult_cap = 0;
static uint64_t g_mult_next = 0xFFFFFFFFull; /* next candidate to test */

int orc_mwc_multipliers(uint64_t n, uint32_t *out)
{
    if (n > MWCD_MAX_STREAMS) return -1;
    if (g_mult_cap < n) {
        uint32_t *m = (uint32_t *)realloc(g_mult, 4 * n);
        if (!m) return -3;
        g_mult = m;
        g_mult_cap = n;
    }
    while (g_mult_n < n && g_mult_next > 1) {
        uint64_t a = g_mult_next--;
        uint64_t p = (a << 32) - 1;
        if (orc_is_prime_u64((p - 1) / 2) && orc_is_prime_u64(p)) g_mult[g_mult_n++] = (uint32_t)a;
    }
    if (g_mult_n < n) return -1;
    memcpy(out, g_mult, 4 * n);
    return 0;
}

/* flags[i] = 1 iff a = top - i (i < count, a > 1) qualifies: the same test
 * as above, one candidate at a time (orc_mwc_multipliers takes the
 * qualifying candidates in exactly this order). */
int orc_mwc_candidates(uint32_t top, uint64_t count, uint8_t *flags)
{
    if (count > top) return -1;
    for (uint64_t i = 0; i < count; i++) {
        uint64_t a = (uint64_t)top - i, p = (a << 32) - 1;
        flags[i] = (uint8_t)(a > 1 && orc_is_prime_u64((p - 1) / 2) && orc_is_prime_u64(p));
    }
    return 0;
}

/* MWC_DIFF states from a given multiplier list a[0..S): as MWC, with the
 * carry reduced mod (a_s - 1). */
static void seed_mwcd_from(uint64_t S, uint64_t seed, const uint32_t *a, uint8_t *b)
{
    uint64_t *y = (uint64_t *)b;
    uint32_t *ad = (uint32_t *)(b + 8 * S);
    for (uint64_t s = 0; s < S; s++) {
        uint64_t z = orc_splitmix(seed, 1 + s);
        uint64_t x = z & 0xFFFFFFFFull, c = (z >> 32) % ((uint64_t)a[s] - 1);
        if (x == 0 && c == 0) x = 1;
        y[s] = (c << 32) | x;
        ad[s] = a[s];
    }
}

int orc_seed_mwcd(uint64_t S, uint64_t seed, const uint32_t *a, void *st)
{
    if (!kind_ok(ORC_MWCD, S)) return -1;
    seed_mwcd_from(S, seed, a, (uint8_t *)st);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Seeding: every stream's initial state derives from SM(.) of the master
 * seed by fixed indices (project definition). */
int orc_seed(int kind, uint64_t S, uint64_t seed, void *st)
{
    if (!kind_ok(kind, S)) return -1;
    uint8_t *b = (uint8_t *)st;
    if (kind == ORC_LCG32) {
        uint32_t *x = (uint32_t *)b;
        for (uint64_t s = 0; s < S; s++) x[s] = (uint32_t)orc_splitmix(seed, 1 + s);
    } else if (kind == ORC_LCG64) {
        uint64_t *x = (uint64_t *)b;
        for (uint64_t s = 0; s < S; s++) x[s] = orc_splitmix(seed, 1 + s);
    } else if (kind == ORC_LCG32S) {
        uint32_t *x = (uint32_t *)b, g = (uint32_t)orc_splitmix(seed, 1), A = 1, C = 0;
        for (uint64_t s = 0; s < S; s++) { x[s] = g; g = LCG32_A * g + LCG32_C; }
        for (uint64_t s = 0; s < S; s++) { A = LCG32_A * A; C = LCG32_A * C + LCG32_C; } /* S steps composed */
        x[S] = A; x[S + 1] = C;
    } else if (kind == ORC_LCG64S) {
        uint64_t *x = (uint64_t *)b, g = orc_splitmix(seed, 1), A = 1, C = 0;
        for (uint64_t s = 0; s < S; s++) { x[s] = g; g = LCG64_A * g + LCG64_C; }
        for (uint64_t s = 0; s < S; s++) { A = LCG64_A * A; C = LCG64_A * C + LCG64_C; }
        x[S] = A; x[S + 1] = C;
    } else if (kind == ORC_MWC) {
        /* x = low word, carry = high word mod (a-1): then 0 <= y < p with
         * p = a*2^32 - 1; y = 0 is a fixed point and is replaced by x = 1. */
        uint64_t *y = (uint64_t *)b;
        for (uint64_t s = 0; s < S; s++) {
            uint64_t z = orc_splitmix(seed, 1 + s);
            uint64_t x = z & 0xFFFFFFFFull, c = (z >> 32) % (MWC_A - 1);
            if (x == 0 && c == 0) x = 1;
            y[s] = (c << 32) | x;
        }
    } else if (kind == ORC_XORWOW) {
        uint32_t *x = (uint32_t *)b, *y = x + S, *z = y + S, *w = z + S, *v = w + S, *d = v + S;
        for (uint64_t s = 0; s < S; s++) {
            uint64_t a = orc_splitmix(seed, 1 + 3 * s);
            uint64_t c = orc_splitmix(seed, 2 + 3 * s);
            uint64_t e = orc_splitmix(seed, 3 + 3 * s);
            x[s] = (uint32_t)a; y[s] = (uint32_t)(a >> 32);
            z[s] = (uint32_t)c; w[s] = (uint32_t)(c >> 32);
            v[s] = (uint32_t)e; d[s] = (uint32_t)(e >> 32);
            if ((x[s] | y[s] | z[s] | w[s] | v[s]) == 0) x[s] = 1;
        }
    } else if (IS_PHILOX(kind)) {
        uint32_t *k0 = (uint32_t *)b, *k1 = k0 + S;
        uint64_t *pos = (uint64_t *)(b + 8 * S);
        for (uint64_t s = 0; s < S; s++) {
            uint64_t z = orc_splitmix(seed, 1 + s);
            k0[s] = (uint32_t)z; k1[s] = (uint32_t)(z >> 32); pos[s] = 0;
        }
    } else if (kind == ORC_MWCD) {
        uint32_t *a = (uint32_t *)(b + 8 * S);
        if (orc_mwc_multipliers(S, a)) return -3;
        seed_mwcd_from(S, seed, a, b);
    } else if (IS_LFG(kind)) {
        const uint64_t r = LFG_R(kind), H = (r + 1) / 2;
        uint32_t *X = (uint32_t *)b;
        for (uint64_t g = 0; g < S / LFG_W; g++) {
            uint32_t odd = 0;
            for (uint64_t j = 0; j < r; j++) {
                uint64_t z = orc_splitmix(seed, 1 + H * g + j / 2);
                X[r * g + j] = (j % 2 == 0) ? (uint32_t)z : (uint32_t)(z >> 32);
                odd |= X[r * g + j] & 1u;
            }
            if (!odd) X[r * g] |= 1u;
        }
    } else { /* XS1024W */
        uint32_t *W = (uint32_t *)b;
        uint64_t *n = (uint64_t *)(b + 4 * S);
        uint32_t *y0 = (uint32_t *)(b + 4 * S + 8 * (S / 32));
        for (uint64_t g = 0; g < S / 32; g++) {
            uint32_t acc = 0;
            for (int i = 0; i < 32; i++) {
                uint64_t z = orc_splitmix(seed, 1 + 16 * g + (uint64_t)(i / 2));
                W[32 * g + i] = (i % 2 == 0) ? (uint32_t)z : (uint32_t)(z >> 32);
                acc |= W[32 * g + i];
            }
            if (acc == 0) return -2; /* the all-zero word is a fixed point */
            n[g] = 0;
        }
        *y0 = (uint32_t)(orc_splitmix(seed, 0) >> 32);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Output emission helper. */
static void emit(int mode, void *out, uint64_t k, uint64_t width, uint64_t col, uint32_t u)
{
    if (mode == ORC_OUT_U32) {
        ((uint32_t *)out)[k * width + col] = u;
    } else if (mode == ORC_OUT_F32) {
        /* (u >> 8) * 2^-24: exact in binary32, in [0, 1). */
        ((float *)out)[k * width + col] = (float)(u >> 8) * (1.0f / 16777216.0f);
    } else {
        ((uint32_t *)out)[col] ^= u;
    }
}

/* Generate `count` outputs of streams [lo, hi), advancing their state.
 * mode U32/F32: out[k*(hi-lo) + (s-lo)]; mode XOR: out[s-lo] ^= every output
 * (the caller zeroes it).  XS1024W needs lo, hi multiples of 32. */
int orc_generate(int kind, uint64_t S, void *st, uint64_t lo, uint64_t hi, uint64_t count, int mode,
                 void *out)
{
    if (!kind_ok(kind, S) || lo > hi || hi > S) return -1;
    if (kind == ORC_XS1024W && (lo % 32 || hi % 32)) return -1;
    if (IS_LFG(kind) && (lo % LFG_W || hi % LFG_W)) return -1;
    uint64_t width = hi - lo;
    uint8_t *b = (uint8_t *)st;
    if (IS_LFG(kind)) {
        /* the instance's sequence through a ring of its last r values:
         * buf[h] is x_{n-r}, buf[(h + r - s) % r] is x_{n-s} */
        const uint64_t r = LFG_R(kind), sl = LFG_S(kind);
        uint32_t *X = (uint32_t *)b;
        uint32_t *buf = (uint32_t *)malloc(4 * r);
        if (!buf) return -3;
        for (uint64_t g = lo / LFG_W; g < hi / LFG_W; g++) {
            memcpy(buf, &X[r * g], 4 * r);
            uint64_t h = 0;
            for (uint64_t k = 0; k < count; k++)
                for (uint64_t i = 0; i < LFG_W; i++) {
                    uint32_t x = buf[h] + buf[(h + r - sl) % r];
                    buf[h] = x;
                    h = (h + 1) % r;
                    emit(mode, out, k, width, LFG_W * g + i - lo, x);
                }
            for (uint64_t j = 0; j < r; j++) X[r * g + j] = buf[(h + j) % r];
        }
        free(buf);
        return 0;
    }
    if (kind == ORC_LCG32) {
        uint32_t *x = (uint32_t *)b;
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                x[s] = LCG32_A * x[s] + LCG32_C;
                emit(mode, out, k, width, s - lo, x[s]);
            }
    } else if (kind == ORC_LCG64) {
        uint64_t *x = (uint64_t *)b;
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                x[s] = LCG64_A * x[s] + LCG64_C;
                emit(mode, out, k, width, s - lo, (uint32_t)(x[s] >> 32));
            }
    } else if (kind == ORC_LCG32S) {
        uint32_t *x = (uint32_t *)b, A = x[S], C = x[S + 1];
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                x[s] = A * x[s] + C;
                emit(mode, out, k, width, s - lo, x[s]);
            }
    } else if (kind == ORC_LCG64S) {
        uint64_t *x = (uint64_t *)b, A = x[S], C = x[S + 1];
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                x[s] = A * x[s] + C;
                emit(mode, out, k, width, s - lo, (uint32_t)(x[s] >> 32));
            }
    } else if (kind == ORC_MWC) {
        uint64_t *y = (uint64_t *)b;
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                uint64_t x = y[s] & 0xFFFFFFFFull, c = y[s] >> 32;
                uint64_t t = MWC_A * x + c; /* < 2^64 since a < 2^32, c < a */
                y[s] = t;                   /* new carry t>>32, new x t mod 2^32 */
                emit(mode, out, k, width, s - lo, (uint32_t)t);
            }
    } else if (kind == ORC_MWCD) {
        uint64_t *y = (uint64_t *)b;
        const uint32_t *a = (const uint32_t *)(b + 8 * S);
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                uint64_t x = y[s] & 0xFFFFFFFFull, c = y[s] >> 32;
                uint64_t t = (uint64_t)a[s] * x + c; /* < 2^64: a < 2^32, c < a */
                y[s] = t;
                emit(mode, out, k, width, s - lo, (uint32_t)t);
            }
    } else if (kind == ORC_XORWOW) {
        uint32_t *X = (uint32_t *)b, *Y = X + S, *Z = Y + S, *Wd = Z + S, *V = Wd + S, *D = V + S;
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                /* Marsaglia 2003, "Xorshift RNGs", xorwow: shifts (2,1,4). */
                uint32_t t = X[s] ^ (X[s] >> 2);
                X[s] = Y[s]; Y[s] = Z[s]; Z[s] = Wd[s]; Wd[s] = V[s];
                V[s] = (V[s] ^ (V[s] << 4)) ^ (t ^ (t << 1));
                D[s] += WEYL_C;
                emit(mode, out, k, width, s - lo, D[s] + V[s]);
            }
    } else if (IS_PHILOX(kind)) {
        uint32_t *k0 = (uint32_t *)b, *k1 = k0 + S;
        uint64_t *pos = (uint64_t *)(b + 8 * S);
        for (uint64_t s = lo; s < hi; s++)
            for (uint64_t k = 0; k < count; k++) {
                uint32_t blk[4];
                philox4x32(k0[s], k1[s], pos[s] / 4, PHILOX_R(kind), blk);
                emit(mode, out, k, width, s - lo, blk[pos[s] % 4]);
                pos[s]++;
            }
    } else {
        uint32_t *W = (uint32_t *)b;
        uint64_t *n = (uint64_t *)(b + 4 * S);
        uint32_t y0 = *(uint32_t *)(b + 4 * S + 8 * (S / 32));
        for (uint64_t g = lo / 32; g < hi / 32; g++)
            for (uint64_t k = 0; k < count; k++) {
                xs1024_step(&W[32 * g]);
                n[g]++;
                uint32_t t = weyl_mix(y0, n[g]);
                for (int i = 0; i < 32; i++)
                    emit(mode, out, k, width, 32 * g + i - lo, W[32 * g + i] + t);
            }
    }
    return 0;
}

/* Advance streams [lo, hi) by n outputs by plain stepping (the definition
 * the jump-ahead below must reproduce). */
int orc_step_n(int kind, uint64_t S, void *st, uint64_t lo, uint64_t hi, uint64_t n)
{
    if (!kind_ok(kind, S) || lo > hi || hi > S) return -1;
    if (kind == ORC_XS1024W && (lo % 32 || hi % 32)) return -1;
    uint8_t *b = (uint8_t *)st;
    if (IS_PHILOX(kind)) { /* counter-based: stepping is counting */
        uint64_t *pos = (uint64_t *)(b + 8 * S);
        for (uint64_t s = lo; s < hi; s++) pos[s] += n;
        return 0;
    }
    if (IS_LFG(kind)) { /* n rows of each instance, outputs discarded */
        if (lo % LFG_W || hi % LFG_W) return -1;
        uint32_t *xs = (uint32_t *)calloc(LFG_W, 4);
        if (!xs) return -3;
        for (uint64_t g = lo / LFG_W; g < hi / LFG_W; g++)
            orc_generate(kind, S, st, LFG_W * g, LFG_W * g + LFG_W, n, ORC_OUT_XOR, xs);
        free(xs);
        return 0;
    }
    uint32_t sink[32];
    for (uint64_t k = 0; k < n; k++) {
        if (kind == ORC_XS1024W) {
            for (uint64_t g = lo / 32; g < hi / 32; g++) {
                memset(sink, 0, sizeof sink);
                orc_generate(kind, S, st, 32 * g, 32 * g + 32, 1, ORC_OUT_XOR, sink);
            }
        } else {
            for (uint64_t s = lo; s < hi; s++) {
                sink[0] = 0;
                orc_generate(kind, S, st, s, s + 1, 1, ORC_OUT_XOR, sink);
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Jump-ahead as powers of the one-step map.
 *
 * LCG (eq. lcg_skipping): the step is the affine map f(x) = a x + c mod m;
 * x_{k+n} = f^n(x_k), computed by repeated squaring of affine maps.  (The
 * paper prints c_t = sum_{i=1..t} a^i c, which gives a*c for t = 1; the
 * power of the map gives c * sum_{i=0..t-1} a^i, which is what stepping
 * produces.)
 *
 * MWC: with y = carry*2^32 + x and p = a*2^32 - 1 one step is y -> a*y mod p
 * (a*y = a*carry*2^32 + a*x = carry + a*x mod p since a*2^32 = 1 mod p), so
 * the n-step map is y -> a^n y mod p.
 *
 * XORWOW / XS1024W: the xorshift part is linear over GF(2); its n-step map is
 * the matrix power M^n of the one-step matrix M built column by column from
 * unit vectors.  The Weyl parts advance by n*c (XORWOW's d) or by n (the
 * XS1024W step counter).
 *
 * Philox: the position advances by n.
 *
 * n is given as n_words little-endian 64-bit words, so powers beyond 2^64
 * (periods) can be expressed. */

typedef struct { uint64_t a, c; } aff64;

static aff64 aff_compose(aff64 f, aff64 g) /* f after g */
{
    aff64 h = { f.a * g.a, f.a * g.c + f.c };
    return h;
}

static int exp_bit(const uint64_t *n_le, int n_words, int bit)
{
    if (bit >= 64 * n_words) return 0;
    return (int)((n_le[bit / 64] >> (bit % 64)) & 1u);
}

static aff64 aff_pow(aff64 f, const uint64_t *n_le, int n_words)
{
    aff64 r = { 1, 0 }, p = f;
    for (int bit = 0; bit < 64 * n_words; bit++) {
        if (exp_bit(n_le, n_words, bit)) r = aff_compose(p, r);
        p = aff_compose(p, p);
    }
    return r;
}

static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)a * b) % m);
}

/* GF(2) linear maps on nbits-bit vectors; a matrix is stored as nbits
 * columns of nw = ceil(nbits/64) words each; column j is the image of e_j. */
typedef struct { int nbits, nw; uint64_t *col; } gf2mat;

static gf2mat gf2_alloc(int nbits)
{
    gf2mat m; m.nbits = nbits; m.nw = (nbits + 63) / 64;
    m.col = (uint64_t *)calloc((size_t)nbits * m.nw, 8);
    return m;
}

static void gf2_apply(const gf2mat *m, const uint64_t *v, uint64_t *out)
{
    memset(out, 0, 8 * (size_t)m->nw);
    for (int j = 0; j < m->nbits; j++)
        if ((v[j / 64] >> (j % 64)) & 1u)
            for (int w = 0; w < m->nw; w++) out[w] ^= m->col[(size_t)j * m->nw + w];
}

static void gf2_mul(const gf2mat *a, const gf2mat *b, gf2mat *out) /* out = a*b */
{
    for (int j = 0; j < b->nbits; j++) gf2_apply(a, &b->col[(size_t)j * b->nw], &out->col[(size_t)j * out->nw]);
}

typedef void (*lin_step_fn)(uint64_t *v);

/* v_i <- M^n v_i for the nvec vectors v (nw words each), with M the matrix
 * of the linear map `step`. */
static void gf2_jump(int nbits, lin_step_fn step, uint64_t *v, uint64_t nvec, const uint64_t *n_le, int n_words)
{
    gf2mat P = gf2_alloc(nbits), T = gf2_alloc(nbits);
    int nw = P.nw;
    for (int j = 0; j < nbits; j++) { /* P = M */
        uint64_t *c = &P.col[(size_t)j * nw];
        c[j / 64] = 1ull << (j % 64);
        step(c);
    }
    uint64_t *tmp = (uint64_t *)calloc(nw, 8);
    int top = 64 * n_words - 1;
    while (top >= 0 && !exp_bit(n_le, n_words, top)) top--;
    for (int bit = 0; bit <= top; bit++) {
        if (exp_bit(n_le, n_words, bit))
            for (uint64_t i = 0; i < nvec; i++) {
                gf2_apply(&P, &v[i * nw], tmp);
                memcpy(&v[i * nw], tmp, 8 * (size_t)nw);
            }
        if (bit < top) { gf2_mul(&P, &P, &T); gf2mat x = P; P = T; T = x; }
    }
    free(tmp); free(P.col); free(T.col);
}

/* XORWOW xorshift part as a map on 160 bits: words x,y,z,w,v packed as
 * bits 32*i .. 32*i+31 for i = 0..4. */
static void xorwow_lin(uint64_t *v)
{
    uint32_t s[5];
    for (int i = 0; i < 5; i++) s[i] = (uint32_t)(v[(32 * i) / 64] >> ((32 * i) % 64));
    uint32_t t = s[0] ^ (s[0] >> 2);
    uint32_t nv = (s[4] ^ (s[4] << 4)) ^ (t ^ (t << 1));
    uint32_t r[5] = { s[1], s[2], s[3], s[4], nv };
    memset(v, 0, 24);
    for (int i = 0; i < 5; i++) v[(32 * i) / 64] |= (uint64_t)r[i] << ((32 * i) % 64);
}

/* XORShift-1024 as a map on 1024 bits: word i at bits 32*i .. 32*i+31. */
static void xs1024_lin(uint64_t *v)
{
    uint32_t W[32];
    for (int i = 0; i < 32; i++) W[i] = (uint32_t)(v[i / 2] >> (32 * (i % 2)));
    xs1024_step(W);
    for (int i = 0; i < 16; i++) v[i] = (uint64_t)W[2 * i] | ((uint64_t)W[2 * i + 1] << 32);
}

/* LFG: with P(x) = x^r - x^(r-s) - 1, the characteristic polynomial of
 * x_n = x_{n-s} + x_{n-r}, the shift by N outputs of an instance is
 * J(E) for J(x) = x^N mod P(x) over Z/2^32 (P is monic, so the division
 * needs no inverses): x_{m+N} = sum_i J_i x_{m+i}.  N = n rows = n*LFG_W
 * values, given as n_le; poly_mulmod is a plain O(r^2) product followed by
 * reduction from the top with x^r = x^(r-s) + 1. */
static void lfg_mulmod(const uint32_t *a, const uint32_t *b, uint32_t *out, uint32_t *tmp, int r, int sl)
{
    memset(tmp, 0, 4 * (size_t)(2 * r - 1));
    for (int i = 0; i < r; i++)
        if (a[i])
            for (int j = 0; j < r; j++) tmp[i + j] += a[i] * b[j];
    for (int d = 2 * r - 2; d >= r; d--) { /* x^d = x^(d-s) + x^(d-r) */
        tmp[d - sl] += tmp[d];
        tmp[d - r] += tmp[d];
        tmp[d] = 0;
    }
    memcpy(out, tmp, 4 * (size_t)r);
}

static int lfg_jump(int kind, uint64_t S, uint32_t *X, uint64_t lo, uint64_t hi, const uint64_t *n_le, int n_words)
{
    const int r = LFG_R(kind), sl = LFG_S(kind);
    uint32_t *J = calloc(r, 4), *P = calloc(r, 4), *T = calloc(r, 4), *tmp = calloc(2 * r, 4), *E = calloc(2 * r, 4);
    if (!J || !P || !T || !tmp || !E) { free(J); free(P); free(T); free(tmp); free(E); return -3; }
    (void)S;
    /* P = x^LFG_W mod P(x) (one row), J = P^n */
    J[0] = 1;
    P[0] = 0;
    {
        uint32_t *xp = calloc(r, 4);
        xp[0] = 1;
        for (int k = 0; k < LFG_W; k++) { /* multiply by x */
            uint32_t top = xp[r - 1];
            memmove(xp + 1, xp, 4 * (size_t)(r - 1));
            xp[0] = top;          /* x^r -> 1 */
            xp[r - sl] += top;    /*     + x^(r-s) */
        }
        memcpy(P, xp, 4 * (size_t)r);
        free(xp);
    }
    for (int bit = 0; bit < 64 * n_words; bit++) {
        if (exp_bit(n_le, n_words, bit)) { lfg_mulmod(J, P, T, tmp, r, sl); memcpy(J, T, 4 * (size_t)r); }
        lfg_mulmod(P, P, T, tmp, r, sl);
        memcpy(P, T, 4 * (size_t)r);
    }
    for (uint64_t g = lo / LFG_W; g < hi / LFG_W; g++) {
        /* E[k] = x_{n-r+k}, k < 2r - 1: the state, then r - 1 further values */
        memcpy(E, &X[(uint64_t)r * g], 4 * (size_t)r);
        for (int k = r; k < 2 * r - 1; k++) E[k] = E[k - r] + E[k - sl];
        for (int j = 0; j < r; j++) {
            uint32_t acc = 0;
            for (int i = 0; i < r; i++) acc += J[i] * E[j + i];
            X[(uint64_t)r * g + j] = acc;
        }
    }
    free(J); free(P); free(T); free(tmp); free(E);
    return 0;
}

int orc_jump(int kind, uint64_t S, void *st, uint64_t lo, uint64_t hi, const uint64_t *n_le, int n_words)
{
    if (!kind_ok(kind, S) || lo > hi || hi > S || n_words < 1) return -1;
    if (kind == ORC_XS1024W && (lo % 32 || hi % 32)) return -1;
    if (IS_LFG(kind)) {
        if (lo % LFG_W || hi % LFG_W) return -1;
        return lfg_jump(kind, S, (uint32_t *)st, lo, hi, n_le, n_words);
    }
    uint8_t *b = (uint8_t *)st;
    uint64_t n_lo = n_le[0]; /* n mod 2^64 */
    if (kind == ORC_LCG32) {
        aff64 f = { LCG32_A, LCG32_C }, fn = aff_pow(f, n_le, n_words);
        uint32_t *x = (uint32_t *)b;
        for (uint64_t s = lo; s < hi; s++) x[s] = (uint32_t)(fn.a * x[s] + fn.c);
    } else if (kind == ORC_LCG64) {
        aff64 f = { LCG64_A, LCG64_C }, fn = aff_pow(f, n_le, n_words);
        uint64_t *x = (uint64_t *)b;
        for (uint64_t s = lo; s < hi; s++) x[s] = fn.a * x[s] + fn.c;
    } else if (kind == ORC_LCG32S) {
        uint32_t *x = (uint32_t *)b;
        aff64 f = { x[S], x[S + 1] }, fn = aff_pow(f, n_le, n_words); /* mod 2^64, reduced below */
        for (uint64_t s = lo; s < hi; s++) x[s] = (uint32_t)(fn.a * x[s] + fn.c);
    } else if (kind == ORC_LCG64S) {
        uint64_t *x = (uint64_t *)b;
        aff64 f = { x[S], x[S + 1] }, fn = aff_pow(f, n_le, n_words);
        for (uint64_t s = lo; s < hi; s++) x[s] = fn.a * x[s] + fn.c;
    } else if (kind == ORC_MWC) {
        uint64_t p = (MWC_A << 32) - 1, an = 1, sq = MWC_A;
        for (int bit = 0; bit < 64 * n_words; bit++) {
            if (exp_bit(n_le, n_words, bit)) an = mulmod64(an, sq, p);
            sq = mulmod64(sq, sq, p);
        }
        uint64_t *y = (uint64_t *)b;
        for (uint64_t s = lo; s < hi; s++) y[s] = mulmod64(an, y[s], p);
    } else if (kind == ORC_MWCD) { /* y -> a_s^n y mod p_s, p_s = a_s 2^32 - 1, per stream */
        uint64_t *y = (uint64_t *)b;
        const uint32_t *a = (const uint32_t *)(b + 8 * S);
        for (uint64_t s = lo; s < hi; s++) {
            uint64_t p = ((uint64_t)a[s] << 32) - 1, an = 1, sq = a[s];
            for (int bit = 0; bit < 64 * n_words; bit++) {
                if (exp_bit(n_le, n_words, bit)) an = mulmod64(an, sq, p);
                sq = mulmod64(sq, sq, p);
            }
            y[s] = mulmod64(an, y[s], p);
        }
    } else if (kind == ORC_XORWOW) {
        uint32_t *X = (uint32_t *)b, *Y = X + S, *Z = Y + S, *Wd = Z + S, *V = Wd + S, *D = V + S;
        uint64_t m = hi - lo, *v = (uint64_t *)calloc(3 * (m ? m : 1), 8);
        if (!v) return -3;
        for (uint64_t s = lo; s < hi; s++) {
            uint32_t w5[5] = { X[s], Y[s], Z[s], Wd[s], V[s] };
            for (int i = 0; i < 5; i++) v[3 * (s - lo) + (32 * i) / 64] |= (uint64_t)w5[i] << ((32 * i) % 64);
        }
        gf2_jump(160, xorwow_lin, v, m, n_le, n_words);
        for (uint64_t s = lo; s < hi; s++) {
            uint32_t w5[5];
            for (int i = 0; i < 5; i++) w5[i] = (uint32_t)(v[3 * (s - lo) + (32 * i) / 64] >> ((32 * i) % 64));
            X[s] = w5[0]; Y[s] = w5[1]; Z[s] = w5[2]; Wd[s] = w5[3]; V[s] = w5[4];
            D[s] += (uint32_t)n_lo * WEYL_C;
        }
        free(v);
    } else if (IS_PHILOX(kind)) {
        uint64_t *pos = (uint64_t *)(b + 8 * S);
        for (uint64_t s = lo; s < hi; s++) pos[s] += n_lo;
    } else {
        uint32_t *W = (uint32_t *)b;
        uint64_t *n = (uint64_t *)(b + 4 * S);
        uint64_t m = (hi - lo) / 32, *v = (uint64_t *)calloc(16 * (m ? m : 1), 8);
        if (!v) return -3;
        for (uint64_t g = lo / 32; g < hi / 32; g++)
            for (int i = 0; i < 16; i++)
                v[16 * (g - lo / 32) + i] = (uint64_t)W[32 * g + 2 * i] | ((uint64_t)W[32 * g + 2 * i + 1] << 32);
        gf2_jump(1024, xs1024_lin, v, m, n_le, n_words);
        for (uint64_t g = lo / 32; g < hi / 32; g++) {
            for (int i = 0; i < 16; i++) {
                uint64_t q = v[16 * (g - lo / 32) + i];
                W[32 * g + 2 * i] = (uint32_t)q; W[32 * g + 2 * i + 1] = (uint32_t)(q >> 32);
            }
            n[g] += n_lo;
        }
        free(v);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Checkerboard Metropolis update of the 2D Ising ferromagnet (Sec. 2, the
 * application test): square L x L lattice, periodic, J = 1, h = 0, spins
 * int8 +-1 at index y*L + x.
 *
 * Project definitions (the paper fixes the method, not the bits):
 *   - S = L*L/4 streams; stream s = y*(L/4) + x/4 owns the 4 consecutive
 *     sites x0 .. x0+3 (x0 = 4*(x/4)) of row y;
 *   - a sweep is the pass over colour 0 (x+y even) followed by colour 1;
 *   - in pass c stream s updates site x0 + ((c+y)&1) with its next output,
 *     then site x0 + 2 + ((c+y)&1) with the one after; every update draws;
 *   - accept iff dE <= 0 or r < T_dE, T_dE = floor(exp(-beta*dE) * 2^32)
 *     evaluated in IEEE double on the host (dE in {4, 8});
 *   - E = -sum s(x,y)[s(x+1,y) + s(x,y+1)] is recorded after each sweep.
 * Sites of one colour only read the other colour, so a pass has one result
 * whatever the order of its updates. */

uint64_t orc_ising_threshold(double beta, int dE)
{
    double t = floor(exp(-beta * (double)dE) * 4294967296.0);
    return (uint64_t)t;
}

/* Hot start: spin i = +1 iff bit 63 of SM_{seed ^ 0xD1B54A32D192ED03}(i+1) is set. */
int orc_ising_hot_start(uint32_t L, uint64_t seed, int8_t *spins)
{
    if (L < 16 || L % 16) return -1;
    uint64_t ss = seed ^ 0xD1B54A32D192ED03ull;
    for (uint64_t i = 0; i < (uint64_t)L * L; i++) spins[i] = (orc_splitmix(ss, i + 1) >> 63) ? 1 : -1;
    return 0;
}

int32_t orc_ising_energy(uint32_t L, const int8_t *sp)
{
    int64_t e = 0;
    for (uint32_t y = 0; y < L; y++)
        for (uint32_t x = 0; x < L; x++) {
            int s = sp[(uint64_t)y * L + x];
            int right = sp[(uint64_t)y * L + (x + 1) % L];
            int down = sp[(uint64_t)((y + 1) % L) * L + x];
            e -= s * (right + down);
        }
    return (int32_t)e;
}

/* Multi-hit form (k = hits >= 1): every visited site gets `hits` Metropolis
 * updates in a row, its neighbours fixed, each drawing the stream's next
 * output; the stream's first site takes draws 0 .. hits-1 of the pass, its
 * second site draws hits .. 2*hits-1.  hits = 1 is the plain sweep above.
 * (The paper's k counts updates of a tile per load of the generator states:
 * k = 1 uses two numbers per state load and save, k = 100 two hundred.) */
int orc_ising_sweeps_hits(uint32_t L, int kind, double beta, void *st, int8_t *sp, uint64_t n_sweeps,
                          uint32_t hits, int32_t *e_trace)
{
    if (L < 16 || L % 16 || hits < 1) return -1;
    uint64_t S = (uint64_t)L * L / 4, spr = L / 4;
    if (!kind_ok(kind, S)) return -1;
    uint64_t T4 = orc_ising_threshold(beta, 4), T8 = orc_ising_threshold(beta, 8);
    uint32_t *r = (uint32_t *)malloc(2 * (uint64_t)hits * S * sizeof(uint32_t));
    if (!r) return -3;
    for (uint64_t t = 0; t < n_sweeps; t++) {
        for (int c = 0; c < 2; c++) {
            orc_generate(kind, S, st, 0, S, 2 * (uint64_t)hits, ORC_OUT_U32, r); /* r[j*S + s] */
            for (uint64_t s = 0; s < S; s++) {
                uint64_t y = s / spr, x0 = 4 * (s % spr);
                for (int h = 0; h < 2; h++) {
                    uint64_t x = x0 + 2 * h + ((c + y) & 1);
                    int nb = sp[y * L + (x + 1) % L] + sp[y * L + (x + L - 1) % L] +
                             sp[((y + 1) % L) * L + x] + sp[((y + L - 1) % L) * L + x];
                    for (uint32_t i = 0; i < hits; i++) {
                        int si = sp[y * L + x];
                        int dE = 2 * si * nb;
                        uint64_t u = r[((uint64_t)h * hits + i) * S + s];
                        int acc = (dE <= 0) || (dE == 4 && u < T4) || (dE == 8 && u < T8);
                        if (acc) sp[y * L + x] = (int8_t)(-si);
                    }
                }
            }
        }
        if (e_trace) e_trace[t] = orc_ising_energy(L, sp);
    }
    free(r);
    return 0;
}

int orc_ising_sweeps(uint32_t L, int kind, double beta, void *st, int8_t *sp, uint64_t n_sweeps, int32_t *e_trace)
{
    return orc_ising_sweeps_hits(L, kind, beta, st, sp, n_sweeps, 1, e_trace);
}
