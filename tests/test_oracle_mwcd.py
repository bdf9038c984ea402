"""Pins of the oracle's MWC with a different multiplier per stream (MWC
section: multipliers found downward from 4294967118, each with a*2^32 - 1
and (a*2^32 - 2)/2 prime, checked by Rabin-Miller).

- The primality routine agrees with sympy's on random 64-bit numbers, on
  primes near 2^64, and rejects the published strong pseudoprimes to the
  first several prime bases (Jaeschke).
- The multiplier list equals an independent scan with sympy.isprime over
  the top of the range; its first entry is the section's 4294967118; sampled
  later entries are safe-prime multipliers.
- Each stream is the multiplicative LCG y -> a_s y mod p_s (1000 steps), and
  its jump by the order (p_s - 1)/2 returns it.
"""
import numpy as np
import pytest
import sympy

M32 = (1 << 32) - 1


def test_rabin_miller_agrees_with_sympy(orc):
    rng = np.random.default_rng(3)
    for n in rng.integers(0, 2**63, size=3000, dtype=np.uint64):
        n = int(n) | 1
        assert orc.is_prime_u64(n) == sympy.isprime(n), n
    for n in (2, 3, 5, 37, 41, (1 << 61) - 1, 18446744073709551557, 18446744073709551533):
        assert orc.is_prime_u64(n) == sympy.isprime(n) == True, n  # noqa: E712
    # strong pseudoprimes to the bases 2..7, 2..11, 2..13, 2..17, 2..23 (Jaeschke 1993)
    for n in (3215031751, 2152302898747, 3474749660383, 341550071728321, 3825123056546413051):
        assert not orc.is_prime_u64(n) and not sympy.isprime(n), n
    for n in (0, 1, 4, 9, 1 << 63, M32 * M32):
        assert not orc.is_prime_u64(n)


def _scan(count):
    """The first `count` safe-prime multipliers by a plain scan with sympy."""
    out, a = [], M32
    while len(out) < count:
        p = (a << 32) - 1
        q = (p - 1) // 2
        if all(p % d and q % d for d in (3, 5, 7, 11, 13)) and sympy.isprime(q) and sympy.isprime(p):
            out.append(a)
        a -= 1
    return out


def test_multiplier_list_matches_an_independent_scan(orc):
    m = orc.mwc_multipliers(150)
    assert int(m[0]) == 4294967118
    assert [int(v) for v in m] == _scan(150)
    assert np.all(np.diff(m.astype(np.int64)) < 0)


def test_sampled_multipliers_are_safe_prime_multipliers(orc):
    m = orc.mwc_multipliers(4096)
    for a in m[::97]:
        p = (int(a) << 32) - 1
        assert sympy.isprime(p) and sympy.isprime((p - 1) // 2), int(a)


def test_streams_are_multiplicative_lcgs_mod_their_own_safe_prime(orc):
    S = 64
    st = orc.seed("mwc_diff", S, 7)
    y = [int(v) for v in st[: 8 * S].view(np.uint64)]
    a = [int(v) for v in st[8 * S:].view(np.uint32)]
    assert a == [int(v) for v in orc.mwc_multipliers(S)]
    p = [(v << 32) - 1 for v in a]
    assert all(0 < yy < pp and (yy >> 32) < aa - 1 for yy, pp, aa in zip(y, p, a))
    for _ in range(1000):
        out = orc.generate("mwc_diff", S, st, 1)
        y = [(aa * yy) % pp for aa, yy, pp in zip(a, y, p)]
        assert [int(v) for v in st[: 8 * S].view(np.uint64)] == y
        assert [int(v) for v in out[0]] == [v & M32 for v in y]
    assert np.array_equal(st[8 * S:].view(np.uint32), np.array(a, dtype=np.uint32))  # multipliers stay


@pytest.mark.parametrize("s", [0, 5, 63])
def test_period_and_jump(orc, s):
    S = 64
    st = orc.seed("mwc_diff", S, 2)
    a = int(st[8 * S:].view(np.uint32)[s])
    q = (((a << 32) - 1) - 1) // 2
    assert pow(a, q, (a << 32) - 1) == 1
    b = st.copy()
    orc.jump("mwc_diff", S, b, q, lo=s, hi=s + 1)
    assert np.array_equal(b, st)
    c, d = st.copy(), st.copy()
    orc.jump("mwc_diff", S, c, 777)
    orc.step_n("mwc_diff", S, d, 777)
    assert np.array_equal(c, d)


def test_threaded_enumeration_equals_the_downward_search(orc, monkeypatch):
    """The per-candidate test over blocks on several threads gives the same
    list as the sequential downward search (small blocks, so that the list
    spans many blocks and threads)."""
    monkeypatch.setattr(orc, "_MULT_CACHE", np.zeros(0, dtype=np.uint32))
    monkeypatch.setattr(orc, "_MULT_BLOCK", 4096)
    assert np.array_equal(orc.mwc_multipliers(3000, threads=4), orc.mwc_multipliers(3000))
    flags = np.zeros(1000, dtype=np.uint8)
    assert orc.lib().orc_mwc_candidates(4294967118, 1000, flags.ctypes.data) == 0
    assert flags[0] == 1 and int(flags.sum()) == int(np.sum(orc.mwc_multipliers(40) > 4294967118 - 1000))


def test_seeding_from_a_given_list(orc):
    S = 300
    a = orc.mwc_multipliers(S)
    st = np.zeros(orc.state_bytes("mwc_diff", S), dtype=np.uint8)
    assert orc.lib().orc_seed_mwcd(S, 5, a.ctypes.data, st.ctypes.data) == 0
    assert np.array_equal(st, orc.seed("mwc_diff", S, 5))
