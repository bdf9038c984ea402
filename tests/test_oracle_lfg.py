"""Pins of the oracle's additive lagged Fibonacci generators (Lagged
Fibonacci section, eq. used_fibonacci; lags (521, 353) and (1279, 861)).

- The low bit of an instance's sequence obeys the GF(2) recurrence of the
  lags: its minimal polynomial (Berlekamp-Massey) is exactly the trinomial
  x^r + x^(r-s) + 1, of degree r, irreducible (Rabin's test); with 2^r - 1 a
  Mersenne prime it is primitive, so the low bit has period 2^r - 1.
- The operation is addition mod 2^32: the map from start state to outputs
  is additive (outputs of A + B = outputs of A + outputs of B), and not
  XOR-linear (which a shift-register form would be).
- In the section's floating-point notation, u_n = x_n / 2^32 satisfies
  u_n = u_{n-r} + u_{n-s} mod 1 exactly (checked in float64, exact here).
- The layout: output k of lane i is value k*1024 + i of the instance's
  sequence (its rows, concatenated, form the sequence above).
- Jump-ahead equals stepping; composition; the full period 2^31 (2^r - 1)
  the section cites for m = 2^32 (Brent) returns every state, half of it
  does not.
"""
import numpy as np
import pytest
import sympy

import gf2poly

W = 1024
LAGS = {"lfg521": (521, 353), "lfg1279": (1279, 861)}
M32 = (1 << 32) - 1


def _sequence(orc, kind, img, rows):
    """The instance's values (one instance image), in order."""
    st = img.copy()
    return orc.generate(kind, W, st, rows).reshape(-1)


@pytest.mark.parametrize("kind", list(LAGS))
def test_low_bit_minimal_polynomial_is_the_lag_trinomial(orc, kind):
    r, s = LAGS[kind]
    img = orc.seed(kind, W, 5)
    seq = _sequence(orc, kind, img, -(-3 * r // W))
    low = [int(v) & 1 for v in seq[: 3 * r]]
    p = gf2poly.berlekamp_massey(low)
    assert p == (1 << r) | (1 << (r - s)) | 1
    assert gf2poly.is_irreducible(p, [r])
    assert sympy.isprime(2**r - 1)  # so every irreducible of degree r is primitive


@pytest.mark.parametrize("kind", list(LAGS))
def test_additive_mod_2_32_not_xor(orc, kind):
    a = orc.seed(kind, W, 1)
    b = orc.seed(kind, W, 2)
    ab = (a.view(np.uint32).astype(np.uint64) + b.view(np.uint32)).astype(np.uint32).view(np.uint8).copy()
    xa, xb, xab = (_sequence(orc, kind, v, 3) for v in (a, b, ab))
    assert np.array_equal(xab, (xa.astype(np.uint64) + xb).astype(np.uint32))
    x_xor = (a.view(np.uint32) ^ b.view(np.uint32)).view(np.uint8).copy()
    assert not np.array_equal(_sequence(orc, kind, x_xor, 3), xa ^ xb)


@pytest.mark.parametrize("kind", list(LAGS))
def test_mod_one_addition_in_float(orc, kind):
    r, s = LAGS[kind]
    img = orc.seed(kind, W, 9)
    start = img.view(np.uint32).astype(np.float64) / 2**32
    u = np.concatenate([start, _sequence(orc, kind, img, 4).astype(np.float64) / 2**32])
    n = np.arange(r, len(u))
    assert np.array_equal(u[n], np.mod(u[n - r] + u[n - s], 1.0))
    assert np.all((u >= 0) & (u < 1))


@pytest.mark.parametrize("kind", list(LAGS))
def test_lanes_are_consecutive_values_of_the_instance(orc, kind):
    # two instances, interleaved layout out[k*S + s]: lane i of instance g in
    # row k is value k*W + i of instance g's own sequence
    S = 2 * W
    st = orc.seed(kind, S, 3)
    out = orc.generate(kind, S, st.copy(), 3)
    r = LAGS[kind][0]
    for g in range(2):
        one = st[4 * r * g: 4 * r * (g + 1)].copy()
        assert np.array_equal(out[:, W * g: W * (g + 1)].reshape(-1), _sequence(orc, kind, one, 3))


@pytest.mark.parametrize("kind", list(LAGS))
def test_seeding_has_an_odd_word_and_is_deterministic(orc, kind):
    r = LAGS[kind][0]
    S = 8 * W
    a = orc.seed(kind, S, 1)
    assert np.array_equal(a, orc.seed(kind, S, 1)) and not np.array_equal(a, orc.seed(kind, S, 2))
    X = a.view(np.uint32).reshape(S // W, r)
    assert np.all((X & 1).max(axis=1) == 1)
    # word j of instance g is a half of SM(1 + H g + j/2)
    H = (r + 1) // 2
    z = orc.splitmix(1, 1 + H * 3 + 7)
    assert int(X[3, 14]) == z & M32 and int(X[3, 15]) == z >> 32


@pytest.mark.parametrize("kind", list(LAGS))
def test_jump_equals_stepping_and_composes(orc, kind):
    S = 2 * W
    st = orc.seed(kind, S, 4)
    for n in (1, 2, 5):
        a, b = st.copy(), st.copy()
        orc.jump(kind, S, a, n)
        orc.step_n(kind, S, b, n)
        assert np.array_equal(a, b), n
    a, b = st.copy(), st.copy()
    orc.jump(kind, S, a, 3)
    orc.jump(kind, S, a, 1 << 40)
    orc.jump(kind, S, b, (1 << 40) + 3)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", list(LAGS))
def test_full_period(orc, kind):
    # period 2^31 (2^r - 1) values = 2^21 (2^r - 1) rows of 1024
    r = LAGS[kind][0]
    st = orc.seed(kind, W, 6)
    a = st.copy()
    orc.jump(kind, W, a, (1 << 21) * (2**r - 1))
    assert np.array_equal(a, st)
    b = st.copy()
    orc.jump(kind, W, b, (1 << 20) * (2**r - 1))
    assert not np.array_equal(b, st)
