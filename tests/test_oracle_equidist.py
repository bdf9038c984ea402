"""Equidistribution of the XORShift-1024 part (Sec. XORShift generators).

The paper tests the generator for equidistribution as Panneton and L'Ecuyer
do and reports that, of the four shift-direction choices that share the
characteristic polynomial of eq. (threeshift), one is clearly worse and its
own choice is the best.  The oracle computes the dimensions t_l (l = 1..32)
by GF(2) ranks; these tests pin that computation and check the paper's
statement in warp order (the 32 words of a step fed in sequence, the order
the paper runs its tests in).

- Variant 0 is the generator's own step; all four variants share one minimal
  polynomial (degree 1024, weight 475).
- t_l never exceeds 1024 / l, and a step's 32 words determine the state.
- The rank computation agrees with an independent Python elimination over
  outputs produced by the oracle's XS1024W stepping.
- Warp order: variant 0 has the smallest total gap; the worst is at least
  twice it.
"""
import numpy as np
import pytest

import gf2poly

K = 1024


def _gap(t):
    return int(sum(K // l - int(t[l - 1]) for l in range(1, 33)))


def test_variant_zero_is_the_generator(orc):
    st = orc.seed("xs1024w", 32, 3)
    for _ in range(20):
        w = st.view(np.uint32)[:32].copy()
        orc.generate("xs1024w", 32, st, 1)
        assert np.array_equal(orc.xs1024_variant_steps(0, w, 1), st.view(np.uint32)[:32])


def test_variants_share_the_minimal_polynomial(orc):
    rng = np.random.default_rng(1)
    w0 = rng.integers(0, 1 << 32, size=32, dtype=np.uint64).astype(np.uint32)
    polys = []
    for v in range(4):
        w, bits = w0.copy(), []
        for _ in range(2200):
            w = orc.xs1024_variant_steps(v, w, 1)
            bits.append(int(w[7] >> 19) & 1)
        polys.append(gf2poly.berlekamp_massey(bits))
    assert all(p == polys[0] for p in polys)
    assert gf2poly.deg(polys[0]) == 1024 and gf2poly.weight(polys[0]) == 475


@pytest.fixture(scope="module")
def warp(orc):
    return [orc.xs1024_equidistribution(v, -1) for v in range(4)]


def test_bounds(orc, warp):
    for t in warp + [orc.xs1024_equidistribution(0, 0)]:
        assert all(0 < t[l - 1] <= K // l for l in range(1, 33))
    assert all(t[31] == 32 for t in warp)  # one step's 32 words: a bijective image of the state


def _unit_runs(orc, steps):
    """Words of `steps` steps from each of the 1024 unit states, by the
    oracle's XS1024W stepping: words[n][k] = the 32 words after step n+1
    from e_k (bit k counted from the most significant end)."""
    n_inst = K
    st = orc.seed("xs1024w", 32 * n_inst, 1)
    W = st.view(np.uint32)
    W[: 32 * n_inst] = 0
    for k in range(K):
        W[32 * k + k // 32] = np.uint32(1 << (31 - k % 32))
    out = []
    for _ in range(steps):
        orc.step_n("xs1024w", 32 * n_inst, st, 1)
        out.append(W[: 32 * n_inst].reshape(n_inst, 32).copy())
    return out


def _t_by_elimination(words, l, lane):
    """Largest t with independent l-bit truncations of t successive outputs,
    by Gaussian elimination on Python ints (one bit per start state)."""
    seq = []  # outputs as [k] arrays, in order
    for w in words:
        if lane >= 0:
            seq.append(w[:, lane])
        else:
            seq.extend(w[:, i] for i in range(32))
    basis = {}
    t = 0
    for out in seq:
        for j in range(l):
            bits = (out >> np.uint32(31 - j)) & np.uint32(1)
            row = int("".join("1" if b else "0" for b in bits[::-1]), 2)
            while row:
                p = row.bit_length() - 1
                if p not in basis:
                    basis[p] = row
                    break
                row ^= basis[p]
            if row == 0:
                return t
        t += 1
    return t


def test_rank_computation_cross_check(orc, warp):
    words = _unit_runs(orc, 3)
    for l in (11, 12, 16, 32):
        assert _t_by_elimination(words, l, -1) == min(int(warp[0][l - 1]), 96), l
    lane0 = orc.xs1024_equidistribution(0, 0)
    words = _unit_runs(orc, 40)
    for l in (26, 29, 32):
        assert _t_by_elimination(words, l, 0) == lane0[l - 1], l


def test_paper_ranking_in_warp_order(orc, warp):
    gaps = [_gap(t) for t in warp]
    print("total dimension gaps (warp order):", dict(zip(orc.XS1024_VARIANTS, gaps)))
    assert gaps[0] == min(gaps) and gaps.count(gaps[0]) == 1
    assert max(gaps) >= 2 * gaps[0]
