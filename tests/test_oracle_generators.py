"""Pins of the oracle's small-state generators against what the paper fixes.

LCG32 / LCG64 (LCG section): constants, full period, output word.
MWC (multiply-with-carry section): a = 4294967118 is the largest a < 2^32 with
a*2^32 - 1 a safe prime; MWC equals the multiplicative LCG y -> a y mod p.
XORWOW (XORShift section; recurrence from Marsaglia 2003): the xorshift part
has a primitive degree-160 minimal polynomial, so with the Weyl term the
period is 2^192 - 2^32 as the paper states.
Philox4x32-10 and -7 (counter-based section): structural checks here; the
published known-answer vectors and rocRAND's engine pin the block function
(test_oracle_kat.py).  The seven-round variant is also tied to the ten-round
one: three further rounds (written out here from the section's S-box) turn
its block into the ten-round block.
"""
import numpy as np
import pytest
import sympy

import gf2poly

M32 = (1 << 32) - 1
M64 = (1 << 64) - 1


def _u32(img, S, i):
    return img.view(np.uint32)[i * S:(i + 1) * S]


def test_lcg32_constants_and_step(orc):
    S = 4
    st = orc.seed("lcg32", S, 1)
    x0 = st.view(np.uint32).copy()
    out = orc.generate("lcg32", S, st, 3)
    x = [int(v) for v in x0]
    for k in range(3):
        x = [(1664525 * v + 1013904223) & M32 for v in x]
        assert [int(v) for v in out[k]] == x


@pytest.mark.slow
def test_lcg32_full_period_by_stepping(orc):
    # The state returns after exactly 2^32 steps and not after 2^31 (the
    # period divides 2^32, so 2^31 is the only divisor left to exclude).
    S = 1
    st = orc.seed("lcg32", S, 1)
    x0 = st.copy()
    orc.generate("lcg32", S, st, 1 << 31, mode=orc.OUT_XOR)
    assert not np.array_equal(st, x0)
    orc.generate("lcg32", S, st, 1 << 31, mode=orc.OUT_XOR)
    assert np.array_equal(st, x0)


def test_lcg64_output_is_top_word_and_full_period(orc):
    S = 8
    st = orc.seed("lcg64", S, 3)
    for _ in range(5):
        out = orc.generate("lcg64", S, st, 1)
        assert np.array_equal(out[0], (st.view(np.uint64) >> np.uint64(32)).astype(np.uint32))
    # Period exactly 2^64: the 2^63-step map is not the identity, its square is.
    a = st.copy()
    orc.jump("lcg64", S, a, 1 << 63)
    assert not np.array_equal(a, st)
    orc.jump("lcg64", S, a, 1 << 63)
    assert np.array_equal(a, st)


MWC_A = 4294967118
MWC_P = MWC_A * (1 << 32) - 1


def _mwc_multiplier_from_oracle(orc):
    # Recover a from one step: t = a*x + c, so a = (t - c) / x.
    st = orc.seed("mwc", 1, 5)
    y = int(st.view(np.uint64)[0])
    orc.generate("mwc", 1, st, 1)
    t = int(st.view(np.uint64)[0])
    x, c = y & M32, y >> 32
    assert (t - c) % x == 0
    return (t - c) // x


def test_mwc_multiplier_is_largest_safe_prime_multiplier(orc):
    a = _mwc_multiplier_from_oracle(orc)
    assert a == MWC_A
    assert sympy.isprime(a * 2**32 - 1) and sympy.isprime((a * 2**32 - 2) // 2)
    for b in range(a + 1, 2**32):
        assert not (sympy.isprime(b * 2**32 - 1) and sympy.isprime((b * 2**32 - 2) // 2))


def test_mwc_is_multiplicative_lcg_mod_p(orc):
    S = 16
    st = orc.seed("mwc", S, 9)
    y = [int(v) for v in st.view(np.uint64)]
    assert all(0 < v < MWC_P for v in y)
    for _ in range(1000):
        out = orc.generate("mwc", S, st, 1)
        y = [(MWC_A * v) % MWC_P for v in y]
        assert [int(v) for v in st.view(np.uint64)] == y
        assert [int(v) for v in out[0]] == [v & M32 for v in y]


def test_mwc_period_is_half_of_p_minus_1(orc):
    q = (MWC_P - 1) // 2
    assert sympy.isprime(q) and pow(MWC_A, q, MWC_P) == 1
    S = 4
    st = orc.seed("mwc", S, 2)
    a = st.copy()
    orc.jump("mwc", S, a, q)
    assert np.array_equal(a, st)


def _xorwow_v_bits(orc, nsteps, bit):
    """Bit `bit` of the xorshift word v after each step, from the state image."""
    S = 1
    st = orc.seed("xorwow", S, 11)
    seq = []
    for _ in range(nsteps):
        orc.generate("xorwow", S, st, 1)
        v = int(_u32(st, S, 4)[0])
        seq.append((v >> bit) & 1)
    return seq


def test_xorwow_xorshift_part_is_primitive_degree_160(orc):
    p = gf2poly.berlekamp_massey(_xorwow_v_bits(orc, 400, 7))
    assert gf2poly.deg(p) == 160
    factors = list(sympy.factorint(2**160 - 1).keys())
    assert gf2poly.is_irreducible(p, [2, 5])
    assert gf2poly.is_primitive(p, factors)


def test_xorwow_weyl_part_and_output(orc):
    S = 3
    st = orc.seed("xorwow", S, 4)
    d0 = _u32(st, S, 5).copy().astype(np.uint64)
    for k in range(1, 50):
        out = orc.generate("xorwow", S, st, 1)
        d = _u32(st, S, 5).astype(np.uint64)
        assert np.array_equal(d, (d0 + np.uint64(k * 362437)) & np.uint64(M32))
        v = _u32(st, S, 4).astype(np.uint64)
        assert np.array_equal(out[0].astype(np.uint64), (d + v) & np.uint64(M32))


@pytest.mark.parametrize("kind", ["philox4x32_10", "philox4x32_7"])
def test_philox_counter_and_key_semantics(orc, kind):
    # Output k of a stream is word k%4 of block k/4; the position jump is exact;
    # blocks of one key are distinct (the rounds are a bijection of the counter).
    S = 4
    st = orc.seed(kind, S, 1)
    full = orc.generate(kind, S, st.copy(), 64)
    for n in (0, 1, 3, 4, 5, 31):
        a = st.copy()
        orc.jump(kind, S, a, n)
        part = orc.generate(kind, S, a, 64 - n)
        assert np.array_equal(part, full[n:])
    blocks = {tuple(full[4 * b:4 * b + 4, 0]) for b in range(16)}
    assert len(blocks) == 16
    # distinct keys per stream
    k0 = st.view(np.uint32)[:S]
    assert len(set(k0.tolist())) == S


@pytest.mark.parametrize("kind", ["philox4x32_10", "philox4x32_7"])
def test_philox_output_balance(orc, kind):
    # Coarse sanity (not a pin of the constants): bits are balanced.
    S = 64
    st = orc.seed(kind, S, 1)
    out = orc.generate(kind, S, st, 256)
    bits = np.unpackbits(out.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.005


def _philox_round(x, k0, k1):
    # one round: products of words 0 and 2 with the multipliers; the high
    # halves are mixed with the other words and the round key
    p0 = 0xD2511F53 * x[0]
    p1 = 0xCD9E8D57 * x[2]
    return [((p1 >> 32) ^ x[1] ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ x[3] ^ k1) & M32, p0 & M32]


def test_philox7_is_the_first_seven_rounds(orc):
    S = 8
    st = orc.seed("philox4x32_7", S, 3)
    assert np.array_equal(st, orc.seed("philox4x32_10", S, 3))  # same keys, same positions
    b7 = orc.generate("philox4x32_7", S, st.copy(), 8)
    b10 = orc.generate("philox4x32_10", S, st.copy(), 8)
    k0s, k1s = st.view(np.uint32)[:S], st.view(np.uint32)[S:2 * S]
    for s in range(S):
        for blk in range(2):
            x = [int(v) for v in b7[4 * blk:4 * blk + 4, s]]
            for r in (7, 8, 9):
                x = _philox_round(x, (int(k0s[s]) + r * 0x9E3779B9) & M32, (int(k1s[s]) + r * 0xBB67AE85) & M32)
            assert x == [int(v) for v in b10[4 * blk:4 * blk + 4, s]], (s, blk)
    assert not np.array_equal(b7, b10)


def _S(kind, S):
    return orc_lfg_streams(S) if kind.startswith("lfg") else S


def orc_lfg_streams(S):
    return max(1024, S // 1024 * 1024)  # lagged Fibonacci kinds: whole 1024-lane instances


def test_f32_conversion_exact(orc):
    for kind in orc.KINDS:
        S = _S(kind, 32)
        st = orc.seed(kind, S, 1)
        u = orc.generate(kind, S, st.copy(), 16)
        f = orc.generate(kind, S, st.copy(), 16, mode=orc.OUT_F32)
        assert f.dtype == np.float32
        assert np.all(f >= 0) and np.all(f < 1)
        # exact: f * 2^24 is the integer u >> 8
        assert np.array_equal((f.astype(np.float64) * 2**24).astype(np.uint32), u >> np.uint32(8))


def test_consume_is_xor_of_outputs(orc):
    for kind in orc.KINDS:
        S = _S(kind, 64)
        st = orc.seed(kind, S, 3)
        u = orc.generate(kind, S, st.copy(), 33)
        x = orc.generate(kind, S, st.copy(), 33, mode=orc.OUT_XOR)
        assert np.array_equal(np.bitwise_xor.reduce(u, axis=0), x)


def test_seeding_distinct_and_deterministic(orc):
    for kind in orc.KINDS:
        S = _S(kind, 256)
        a = orc.seed(kind, S, 1)
        b = orc.seed(kind, S, 1)
        c = orc.seed(kind, S, 2)
        assert np.array_equal(a, b) and not np.array_equal(a, c)
        out = orc.generate(kind, S, a, 4)
        assert len(set(out[0].tolist())) > S - 4  # streams do not coincide


@pytest.mark.parametrize("kind,S", [("lcg32_sub", 37), ("lcg32_sub", 64), ("lcg64_sub", 37)])
def test_substream_lcg_is_the_global_sequence(orc, kind, S):
    # eq. lcg_skipping with t = S: an interleaved fill of the S streams is the
    # one global sequence from position S on (serial LCG written out here)
    bits = 32 if kind == "lcg32_sub" else 64
    a, c = (1664525, 1013904223) if bits == 32 else (2862933555777941757, 1442695040888963407)
    m = (1 << bits) - 1
    plain = orc.seed(kind.replace("_sub", ""), S, 7)
    g = int(plain.view(np.uint32 if bits == 32 else np.uint64)[0])  # g_0: the plain stream-0 value
    seq = []
    for _ in range(S * 9):
        seq.append(g)
        g = (a * g + c) & m
    st = orc.seed(kind, S, 7)
    words = st.view(np.uint32 if bits == 32 else np.uint64)
    assert [int(v) for v in words[:S]] == seq[:S]
    A, C = int(words[S]), int(words[S + 1])
    assert A == pow(a, S, 1 << bits) and C == sum(c * pow(a, i, 1 << bits) for i in range(S)) & m
    out = orc.generate(kind, S, st, 8).ravel()
    want = np.array([v if bits == 32 else v >> 32 for v in seq[S:9 * S]], dtype=np.uint64)
    assert np.array_equal(out.astype(np.uint64), want)
