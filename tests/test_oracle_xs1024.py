"""Pins of the oracle's XORShift-1024/Weyl generator (the paper's XORShift section).

- The word-array recurrence equals eq. (threeshift) on a 1024-bit integer with
  (a, b, c) = (329, 347, 344), written here independently with Python ints.
- Its minimal polynomial has degree 1024 and weight 475, the weight the paper
  states for its primitive characteristic polynomial; the polynomial is
  irreducible (Rabin), so the state returns after 2^1024 - 1 steps.
- The output is y_n (I + R^16) + x with the Weyl closed form y_n = y_0 + n c,
  c = 362437, shared by all lanes (eq. weylgen and its closed form).
"""
import numpy as np
import pytest

import gf2poly

S = 32  # one instance
MASK = (1 << 1024) - 1
M32 = (1 << 32) - 1


def _words(st):
    return [int(v) for v in st.view(np.uint32)[:32]]


def _n(st):
    return int(st[128:136].view(np.uint64)[0])


def _y0(st):
    return int(st[136:140].view(np.uint32)[0])


def _to_int(words):
    x = 0
    for w in words:  # word 0 most significant
        x = (x << 32) | w
    return x


def _from_int(x):
    return [(x >> (32 * (31 - i))) & M32 for i in range(32)]


def test_word_recurrence_equals_1024_bit_threeshift(orc):
    st = orc.seed("xs1024w", S, 1)
    X = _to_int(_words(st))
    for _ in range(64):
        orc.generate("xs1024w", S, st, 1)
        X ^= (X << 329) & MASK
        X ^= X >> 347
        X ^= (X << 344) & MASK
        assert _words(st) == _from_int(X)


def test_weyl_combination(orc):
    st = orc.seed("xs1024w", 64, 5)
    y0 = int(st[256 + 16:256 + 20].view(np.uint32)[0])
    for n in range(1, 40):
        out = orc.generate("xs1024w", 64, st, 1)[0]
        W = st.view(np.uint32)[:64].astype(np.int64)
        y = (y0 + n * 362437) & M32
        t = y ^ (y >> 16)
        assert np.array_equal(out.astype(np.int64), (W + t) & M32)
        assert [int(v) for v in st[256:272].view(np.uint64)] == [n, n]


def _state_bit_sequence(orc, nsteps, word, bit):
    st = orc.seed("xs1024w", S, 3)
    seq = []
    for _ in range(nsteps):
        orc.generate("xs1024w", S, st, 1)
        seq.append((_words(st)[word] >> bit) & 1)
    return seq


@pytest.fixture(scope="module")
def minpoly(orc):
    return gf2poly.berlekamp_massey(_state_bit_sequence(orc, 2200, 31, 0))


def test_minimal_polynomial_degree_and_weight(minpoly):
    assert gf2poly.deg(minpoly) == 1024
    assert gf2poly.weight(minpoly) == 475


def test_minimal_polynomial_irreducible(minpoly):
    assert gf2poly.is_irreducible(minpoly, [2])


def test_other_bit_positions_share_the_polynomial(orc, minpoly):
    p2 = gf2poly.berlekamp_massey(_state_bit_sequence(orc, 2200, 7, 19))
    assert p2 == minpoly


def test_lanes_step_together_and_instances_are_independent(orc):
    st = orc.seed("xs1024w", 96, 1)
    a = st.copy()
    full = orc.generate("xs1024w", 96, a, 5)
    b = st.copy()
    part = orc.generate("xs1024w", 96, b, 5, lo=32, hi=64)
    assert np.array_equal(full[:, 32:64], part)
    assert np.array_equal(a[128:256], b[128:256])
