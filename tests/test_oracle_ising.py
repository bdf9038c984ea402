"""Pins of the oracle's checkerboard Metropolis update (Sec. 2, the Ising
application test).

- The energy function equals an independent numpy evaluation.
- beta = 0 accepts every proposal: each sweep flips every spin.
- beta -> infinity accepts only dE <= 0: the result does not depend on the
  generator and the energy never rises.
- At L = 16 the measured e and C_V agree with the exact finite-lattice values
  (Ferdinand-Fisher) within 4 standard errors for good generators.
"""
import json
import os

import numpy as np
import pytest

import isingstats
from oracle import exact_ising as ex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _np_energy(sp, L):
    s = sp.reshape(L, L).astype(np.int64)
    return int(-(s * (np.roll(s, -1, axis=1) + np.roll(s, -1, axis=0))).sum())


def test_hot_start_is_random_and_deterministic(orc):
    a = orc.ising_hot_start(64, 1)
    b = orc.ising_hot_start(64, 1)
    c = orc.ising_hot_start(64, 2)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert set(np.unique(a).tolist()) == {-1, 1}
    assert abs(a.mean()) < 0.05


@pytest.mark.parametrize("L", [16, 32, 48])
def test_energy_matches_numpy(orc, L):
    sp = orc.ising_hot_start(L, 3)
    assert orc.ising_energy(L, sp) == _np_energy(sp, L)


def test_thresholds(orc):
    assert orc.ising_threshold(0.0, 4) == 1 << 32
    assert orc.ising_threshold(1e9, 8) == 0
    for beta in (0.1, 0.4, ex.BETA_C, 1.0):
        t4, t8 = orc.ising_threshold(beta, 4), orc.ising_threshold(beta, 8)
        assert 0 < t8 < t4 < 1 << 32
        assert abs(t4 / 2**32 - np.exp(-4 * beta)) < 2**-32


@pytest.mark.parametrize("kind", ["lcg32", "xs1024w", "philox4x32_10"])
def test_infinite_temperature_flips_everything(orc, kind):
    L = 16
    sp, st = orc.ising_create(L, kind, 5)
    sp0 = sp.copy()
    tr = orc.ising_sweeps(L, kind, 0.0, st, sp, 3)
    assert np.array_equal(sp, -sp0)  # odd number of sweeps
    assert np.all(tr == orc.ising_energy(L, sp0))


def test_zero_temperature_ignores_the_generator(orc):
    L = 64  # every kind, the lagged Fibonacci ones included (L % 64 == 0)
    ref = None
    for kind in orc.KINDS:
        sp, st = orc.ising_create(L, kind, 9)
        tr = orc.ising_sweeps(L, kind, 1e9, st, sp, 6)
        assert np.all(np.diff(tr) <= 0)
        if ref is None:
            ref = sp.copy()
        assert np.array_equal(sp, ref), kind


def test_trace_is_energy_after_each_sweep(orc):
    L = 16
    sp, st = orc.ising_create(L, "mwc", 2)
    a_sp, a_st = sp.copy(), st.copy()
    tr = orc.ising_sweeps(L, "mwc", 0.4, st, sp, 5)
    for t in range(5):
        orc.ising_sweeps(L, "mwc", 0.4, a_st, a_sp, 1, trace=False)
        assert tr[t] == _np_energy(a_sp, L)


def test_streams_draw_two_per_pass(orc):
    # After t sweeps every stream has produced exactly 4 t outputs.
    L, kind = 16, "lcg64"
    sp, st = orc.ising_create(L, kind, 4)
    st2 = st.copy()
    orc.ising_sweeps(L, kind, 0.4, st, sp, 3, trace=False)
    orc.step_n(kind, L * L // 4, st2, 12)
    assert np.array_equal(st, st2)


def _exact(L, beta):
    with open(os.path.join(GOLDEN, "exact_ising.json")) as f:
        for rec in json.load(f)["values"]:
            if rec["L"] == L and abs(rec["beta"] - beta) < 1e-15:
                return rec["e"], rec["C_V"]
    raise KeyError((L, beta))


@pytest.mark.parametrize("kind", ["xs1024w", "philox4x32_10", "mwc"])
@pytest.mark.parametrize("beta", [0.4, ex.BETA_C])
def test_statistics_match_exact_L16(orc, kind, beta):
    L, n_eq, n_meas = 16, 2000, 40000
    sp, st = orc.ising_create(L, kind, 1)
    orc.ising_sweeps(L, kind, beta, st, sp, n_eq, trace=False)
    tr = orc.ising_sweeps(L, kind, beta, st, sp, n_meas)
    e, se, c, sc = isingstats.estimates(tr, L * L, beta)
    ee, ce = _exact(L, beta)
    assert abs(e - ee) < 4 * se, (e, se, ee)
    assert abs(c - ce) < 4 * sc, (c, sc, ce)


def test_colour_zero_goes_first(orc):
    # Neel state s = (-1)^(x+y): colour 0 (x+y even) holds +1.  At zero
    # temperature the first pass flips its whole sublattice (dE = -8) and the
    # second pass then sees dE = +8 everywhere, so one sweep ends uniform with
    # the sign colour 1 had: all -1 iff colour 0 is updated first.
    L = 16
    y, x = np.mgrid[0:L, 0:L]
    sp = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8).ravel()
    st = orc.seed("lcg32", L * L // 4, 1)
    orc.ising_sweeps(L, "lcg32", 1e9, st, sp, 1, trace=False)
    assert np.all(sp == -1)


# ---------------------------------------------------------------- multi-hit
# k Metropolis updates per visited site, neighbours fixed (the paper's k of
# updates per load of the generator states, read as single-site hits).

@pytest.mark.parametrize("hits", [2, 3])
def test_multihit_infinite_temperature(orc, hits):
    # every hit is taken: a sweep flips every spin `hits` times
    L, kind = 16, "xs1024w"
    sp, st = orc.ising_create(L, kind, 5)
    sp0 = sp.copy()
    tr = orc.ising_sweeps(L, kind, 0.0, st, sp, 3, hits=hits)
    assert np.array_equal(sp, sp0 if hits % 2 == 0 else -sp0)
    assert np.all(tr == orc.ising_energy(L, sp0))


@pytest.mark.parametrize("hits", [2, 5])
def test_multihit_draw_count(orc, hits):
    # after t sweeps every stream has produced 4 k t outputs
    L, kind = 16, "lcg64"
    sp, st = orc.ising_create(L, kind, 4)
    st2 = st.copy()
    orc.ising_sweeps(L, kind, 0.4, st, sp, 3, trace=False, hits=hits)
    orc.step_n(kind, L * L // 4, st2, 12 * hits)
    assert np.array_equal(st, st2)


@pytest.mark.parametrize("hits", [1, 2, 3])
def test_multihit_neel_zero_temperature(orc, hits):
    # Neel state: a colour-0 site has dE = -8, flips on its first hit and then
    # sees dE = +8, so it flips exactly once whatever k is; colour 1 then sees
    # dE = +8.  One sweep ends all -1 for every k (a hit loop that kept the
    # first hit's dE would flip colour 0 k times).
    L = 16
    y, x = np.mgrid[0:L, 0:L]
    sp = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8).ravel()
    st = orc.seed("mwc", L * L // 4, 1)
    orc.ising_sweeps(L, "mwc", 1e9, st, sp, 1, trace=False, hits=hits)
    assert np.all(sp == -1)


def test_multihit_zero_temperature_ignores_the_generator(orc):
    L = 64
    for hits in (2, 3):
        ref = None
        for kind in orc.KINDS:
            sp, st = orc.ising_create(L, kind, 9)
            tr = orc.ising_sweeps(L, kind, 1e9, st, sp, 6, hits=hits)
            assert np.all(np.diff(tr) <= 0)
            if ref is None:
                ref = sp.copy()
            assert np.array_equal(sp, ref), (kind, hits)


@pytest.mark.parametrize("beta", [0.4, ex.BETA_C])
def test_multihit_statistics_match_exact_L16(orc, beta):
    # every hit is a Metropolis step with the environment fixed, so the
    # equilibrium is unchanged
    L, n_eq, n_meas, kind = 16, 2000, 40000, "xs1024w"
    sp, st = orc.ising_create(L, kind, 1)
    orc.ising_sweeps(L, kind, beta, st, sp, n_eq, trace=False, hits=2)
    tr = orc.ising_sweeps(L, kind, beta, st, sp, n_meas, hits=2)
    e, se, c, sc = isingstats.estimates(tr, L * L, beta)
    ee, ce = _exact(L, beta)
    assert abs(e - ee) < 4 * se, (e, se, ee)
    assert abs(c - ce) < 4 * sc, (c, sc, ce)
