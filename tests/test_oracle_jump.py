"""Pins of the oracle's jump-ahead: it must equal plain stepping, compose, and
return to the start after each generator's period.

LCG (eq. lcg_skipping, with the affine-map power c_t = c * sum_{i<t} a^i that
stepping produces; the printed sum over i = 1..t is off by one power of a),
MWC (a^n mod p), the GF(2) matrix powers of XORWOW's and XS1024W's xorshift
parts, and Philox's counter.
"""
import numpy as np
import pytest

KIND_S = {"lcg32": 5, "lcg64": 5, "mwc": 5, "xorwow": 5, "philox4x32_10": 5, "xs1024w": 64, "philox4x32_7": 5,
          "lcg32_sub": 5, "lcg64_sub": 5}


@pytest.mark.parametrize("kind", list(KIND_S))
def test_jump_equals_stepping(orc, kind):
    S = KIND_S[kind]
    st = orc.seed(kind, S, 17)
    for n in (0, 1, 2, 3, 31, 32, 1000, 4097):
        a, b = st.copy(), st.copy()
        orc.jump(kind, S, a, n)
        orc.step_n(kind, S, b, n)
        assert np.array_equal(a, b), (kind, n)
        # and the outputs after the jump are the outputs of the stepped stream
        assert np.array_equal(orc.generate(kind, S, a, 9), orc.generate(kind, S, b, 9))


@pytest.mark.parametrize("kind", list(KIND_S))
def test_jump_equals_stepping_long(orc, kind):
    S = KIND_S[kind]
    st = orc.seed(kind, S, 2)
    n = 99991
    a, b = st.copy(), st.copy()
    orc.jump(kind, S, a, n)
    orc.step_n(kind, S, b, n)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", list(KIND_S))
def test_jump_composes(orc, kind):
    S = KIND_S[kind]
    st = orc.seed(kind, S, 8)
    p, q = (1 << 40) + 3, (1 << 45) + 12345
    a, b = st.copy(), st.copy()
    orc.jump(kind, S, a, p)
    orc.jump(kind, S, a, q)
    orc.jump(kind, S, b, p + q)
    assert np.array_equal(a, b)


def test_lcg32_period(orc):
    st = orc.seed("lcg32", 7, 1)
    a = st.copy()
    orc.jump("lcg32", 7, a, 1 << 31)
    assert not np.array_equal(a, st)
    orc.jump("lcg32", 7, a, 1 << 31)
    assert np.array_equal(a, st)


def test_xorwow_period(orc):
    S = 3
    st = orc.seed("xorwow", S, 1)
    a = st.copy()
    n = (1 << 160) - 1
    orc.jump("xorwow", S, a, n)
    u = st.view(np.uint32)
    v = a.view(np.uint32)
    assert np.array_equal(v[:5 * S], u[:5 * S])  # xorshift words back
    # Weyl word advanced by n*c mod 2^32 = -c
    assert np.array_equal(v[5 * S:], (u[5 * S:].astype(np.int64) - 362437) % (1 << 32))


@pytest.mark.slow
def test_xs1024w_period(orc):
    S = 32
    st = orc.seed("xs1024w", S, 1)
    a = st.copy()
    orc.jump("xs1024w", S, a, (1 << 1024) - 1)
    assert np.array_equal(a[:128], st[:128])
    # step counter advanced by (2^1024 - 1) mod 2^64
    assert int(a[128:136].view(np.uint64)[0]) == (1 << 64) - 1


def test_substream_seeding_composes(orc):
    # instance 0 is the plain seeding's; instance g+1 is instance g skipped
    # 2^137 steps (jumps of 2^137 compose); counters stay 0 (2^137 g mod 2^64)
    S = 32 * 3
    st = orc.seed_substreams("xs1024w", S, 9)
    plain = orc.seed("xs1024w", S, 9)
    W, P = st.view(np.uint32), plain.view(np.uint32)
    assert np.array_equal(W[:32], P[:32])
    nxt = st.copy()
    orc.jump("xs1024w", S, nxt, 1 << 137, lo=32, hi=64)
    assert np.array_equal(nxt.view(np.uint32)[32:64], W[64:96])
    assert not np.array_equal(W[32:64], W[64:96])
    assert np.all(st[4 * S: 4 * S + 8 * 3].view(np.uint64) == 0)
    assert np.array_equal(st[-4:], plain[-4:])  # shared Weyl seed
