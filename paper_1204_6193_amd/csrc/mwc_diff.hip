// MWC with a different multiplier per stream (MWC section): the multipliers
// a are those below 2^32 for which p = a 2^32 - 1 and (p - 1)/2 = a 2^31 - 1
// are both prime, taken in decreasing order starting from the largest,
// 4294967118.  Stream s uses the (s+1)-th of them.
//
// The search runs on the device: one thread per candidate a, trial division
// of both numbers by the odd primes below 256, then a strong-probable-prime
// test to the first twelve prime bases (which decides primality exactly for
// every n < 2^64) with Montgomery arithmetic.  A wave writes one 64-bit word
// of the result bitmap (lane i: candidate top - 64 w - i); the host collects
// the multipliers in order from it.  Near 2^32 about one candidate in 730
// qualifies, so 2^20 streams take about 7.6e8 candidates.  The list is found
// once per process and grows on demand.
#include <mutex>
#include <vector>

#include "rngx_internal.h"

namespace rngx {

namespace {

constexpr int kBlock = 256;

constexpr uint32_t kSmallPrimes[] = {3,   5,   7,   11,  13,  17,  19,  23,  29,  31,  37,  41,  43,  47,  53,
                                     59,  61,  67,  71,  73,  79,  83,  89,  97,  101, 103, 107, 109, 113, 127,
                                     131, 137, 139, 149, 151, 157, 163, 167, 173, 179, 181, 191, 193, 197, 199,
                                     211, 223, 227, 229, 233, 239, 241, 251};
constexpr int kNumSmallPrimes = sizeof(kSmallPrimes) / sizeof(kSmallPrimes[0]);
constexpr uint32_t kMrBases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};

// Strong probable prime to base b (b < n): with n - 1 = d 2^s, d odd,
// b^d = 1 or b^(d 2^r) = n - 1 for some r < s.
__device__ bool sprp(const Mont64 &M, uint64_t d, int s, uint64_t b) {
    const uint64_t mone = M.n - M.one;  // Montgomery form of n - 1
    uint64_t x = M.pow(M.to(b), d);
    if (x == M.one || x == mone) return true;
    for (int r = 1; r < s; ++r) {
        x = M.mul(x, x);
        if (x == mone) return true;
    }
    return false;
}

// n odd, n > 37: exact primality for 64-bit n.
__device__ bool is_prime_big(uint64_t n) {
    const Mont64 M(n);
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (int i = 0; i < 12; ++i)
        if (!sprp(M, d, s, kMrBases[i])) return false;
    return true;
}

// a 2^32 - 1 and a 2^31 - 1 both prime (a > 2^31, so both exceed every
// trial divisor and every base).
__device__ bool multiplier_ok(uint32_t a) {
    for (int i = 0; i < kNumSmallPrimes; ++i) {
        const uint32_t r = kSmallPrimes[i];
        const uint32_t ar = a % r, t31 = (1u << 31) % r;
        const uint32_t q = (ar * t31 + r - 1) % r;  // (a 2^31 - 1) mod r
        const uint32_t p = (2 * q + 1) % r;         // (a 2^32 - 1) mod r
        if (q == 0 || p == 0) return false;
    }
    const uint64_t p = (static_cast<uint64_t>(a) << 32) - 1;
    return is_prime_big(p >> 1) && is_prime_big(p);  // (p - 1)/2 = p >> 1 for odd p
}

// count candidates top, top - 1, ..., top - count + 1 (count a multiple of
// 64, every block of whole waves): bit i of bits[w] is candidate top - 64 w - i.
__global__ __launch_bounds__(kBlock) void k_mwc_search(uint32_t top, uint64_t count, uint64_t *bits) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool ok = i < count && multiplier_ok(top - static_cast<uint32_t>(i));
    const uint64_t mask = __ballot(ok);
    if ((threadIdx.x & 63) == 0 && i < count) bits[i / 64] = mask;
}

// y <- a_s^n y mod p_s for every stream.
__global__ __launch_bounds__(kBlock) void k_skip_mwc_diff(uint8_t *st, uint64_t S, uint64_t n) {
    const uint64_t s = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint64_t *y = reinterpret_cast<uint64_t *>(st);
    const uint32_t a = reinterpret_cast<const uint32_t *>(st + 8 * S)[s];
    y[s] = mwc_jump_mod(y[s], a, n);
}

std::mutex g_mu;
std::vector<uint32_t> g_mults;          // found so far, decreasing
uint64_t g_next = 0xFFFFFFFFull;        // next candidate to test
constexpr uint64_t kFloor = 1ull << 31;  // candidates stay above 2^31
constexpr uint64_t kSearchBlock = 1ull << 26;

// Extends the list to at least n multipliers (caller holds g_mu).
hipError_t grow(uint64_t n, hipStream_t st) {
    if (g_mults.size() >= n) return hipSuccess;
    uint64_t *d_bits = nullptr;
    hipError_t e = hipMalloc(&d_bits, kSearchBlock / 8);
    if (e != hipSuccess) return e;
    std::vector<uint64_t> bits(kSearchBlock / 64);
    while (e == hipSuccess && g_mults.size() < n) {
        if (g_next <= kFloor) { e = hipErrorInvalidValue; break; }
        const uint64_t count = std::min(kSearchBlock, (g_next - kFloor) / 64 * 64);
        if (count == 0) { e = hipErrorInvalidValue; break; }
        const uint32_t top = static_cast<uint32_t>(g_next);
        hipLaunchKernelGGL(k_mwc_search, dim3(static_cast<unsigned>(count / kBlock + (count % kBlock != 0))),
                           dim3(kBlock), 0, st, top, count, d_bits);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(bits.data(), d_bits, count / 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        for (uint64_t w = 0; w < count / 64; ++w)
            for (uint64_t m = bits[w]; m; m &= m - 1)
                g_mults.push_back(top - static_cast<uint32_t>(64 * w + __builtin_ctzll(m)));
        g_next -= count;
    }
    (void)hipFree(d_bits);
    return e;
}

}  // namespace

hipError_t mwc_diff_multipliers(uint64_t n, uint32_t *d_dst, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipError_t e = grow(n, st);
    if (e != hipSuccess) return e;
    if (!d_dst) return hipSuccess;
    e = hipMemcpyAsync(d_dst, g_mults.data(), 4 * n, hipMemcpyHostToDevice, st);
    // the list may grow (and move) once the lock is released
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
}

bool mwc_diff_multipliers_match(const uint32_t *a, uint64_t n) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_mults.size() < n) return false;
    for (uint64_t i = 0; i < n; ++i)
        if (a[i] != g_mults[i]) return false;
    return true;
}

hipError_t launch_skip_mwc_diff(Gen *g, uint64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_skip_mwc_diff, dim3(static_cast<unsigned>((g->S + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, g->d_state, g->S, n);
    return hipGetLastError();
}

}  // namespace rngx
