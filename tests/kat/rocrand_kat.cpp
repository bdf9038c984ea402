// Known-answer source for the oracle's Philox4x32-10 and XORWOW: drives
// rocRAND's host-callable engines (its source headers, an implementation
// independent of this repository) and prints their outputs in hex, one per
// line.  Built for the host only; nothing here runs on a GPU.
//
//   philox KEY BLOCK COUNT   -> COUNT outputs of the engine seeded with the
//                               64-bit KEY (low word = key word 0), started
//                               at output 4*BLOCK, i.e. blocks BLOCK, ... of
//                               counter (block_lo, block_hi, 0, 0)
//   block C0 C1 C2 C3 K0 K1  -> the 4 words of the ten-round block function
//                               on the 128-bit counter (C0..C3) and key
//                               (K0, K1), set directly in the engine
//   xorwow X Y Z W V D COUNT -> COUNT outputs from the state (x, y, z, w, v)
//                               with Weyl word d (the engine's own seeding
//                               is bypassed)
#include <rocrand/rocrand_philox4x32_10.h>
#include <rocrand/rocrand_xorwow.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {
struct XorwowFromState : rocrand_device::xorwow_engine {
    XorwowFromState(const unsigned s[5], unsigned d) {
        for (int i = 0; i < 5; ++i) m_state.x[i] = s[i];
        m_state.d = d;
    }
};
struct PhiloxBlock : rocrand_device::philox4x32_10_engine {
    uint4 run(const unsigned c[4], const unsigned k[2]) {
        m_state.counter = uint4{c[0], c[1], c[2], c[3]};
        m_state.key = uint2{k[0], k[1]};
        return ten_rounds(m_state.counter, m_state.key);
    }
};
unsigned long long arg(const char *s) { return std::strtoull(s, nullptr, 0); }
}  // namespace

int main(int argc, char **argv) {
    if (argc == 5 && !std::strcmp(argv[1], "philox")) {
        const unsigned long long key = arg(argv[2]), block = arg(argv[3]), count = arg(argv[4]);
        rocrand_device::philox4x32_10_engine e(key, 0, 4 * block);
        for (unsigned long long i = 0; i < count; ++i) std::printf("%08x\n", e.next());
        return 0;
    }
    if (argc == 8 && !std::strcmp(argv[1], "block")) {
        unsigned c[4], k[2];
        for (int i = 0; i < 4; ++i) c[i] = static_cast<unsigned>(arg(argv[2 + i]));
        for (int i = 0; i < 2; ++i) k[i] = static_cast<unsigned>(arg(argv[6 + i]));
        const uint4 o = PhiloxBlock().run(c, k);
        std::printf("%08x\n%08x\n%08x\n%08x\n", o.x, o.y, o.z, o.w);
        return 0;
    }
    if (argc == 9 && !std::strcmp(argv[1], "xorwow")) {
        unsigned s[5];
        for (int i = 0; i < 5; ++i) s[i] = static_cast<unsigned>(arg(argv[2 + i]));
        XorwowFromState e(s, static_cast<unsigned>(arg(argv[7])));
        const unsigned long long count = arg(argv[8]);
        for (unsigned long long i = 0; i < count; ++i) std::printf("%08x\n", e.next());
        return 0;
    }
    std::fprintf(stderr, "usage: philox KEY BLOCK COUNT | block C0 C1 C2 C3 K0 K1 | xorwow X Y Z W V D COUNT\n");
    return 2;
}
