"""Pins of the exact finite-lattice Ising values used as the statistical target.

- Brute-force enumeration of every configuration at L = 2, 3, 4.
- L = 1024 equals Onsager's infinite-lattice limit (to ~1e-10).
- The paper's Table 2 "exact" row (L = 1024, beta = 0.4) within 5e-9: the
  printed values are ~3e-9 away from a high-precision evaluation.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import exact_ising as ex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _brute(L, beta):
    N = L * L
    confs = np.array(list(itertools.product((-1, 1), repeat=N)), dtype=np.float64).reshape(-1, L, L)
    E = -(confs * (np.roll(confs, -1, axis=2) + np.roll(confs, -1, axis=1))).sum(axis=(1, 2))
    w = np.exp(-beta * (E - E.min()))
    Z = w.sum()
    m1 = (w * E).sum() / Z
    m2 = (w * E * E).sum() / Z
    return -m1 / N, beta * beta * (m2 - m1 * m1) / N


@pytest.mark.parametrize("L", [2, 3, 4])
@pytest.mark.parametrize("beta", [0.2, 0.4, ex.BETA_C, 0.7])
def test_exact_equals_brute_force(L, beta):
    e, c = ex.exact(L, beta)
    eb, cb = _brute(L, beta)
    assert abs(e - eb) < 1e-11 * max(1, abs(eb))
    assert abs(c - cb) < 1e-10 * max(1, abs(cb))


@pytest.mark.parametrize("beta", [0.3, 0.4, 0.5])
def test_large_lattice_reaches_onsager(beta):
    e, c = ex.exact(1024, beta)
    eo, co = ex.onsager(beta)
    assert abs(e - eo) < 1e-10
    assert abs(c - co) < 1e-9


def _paper_row():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_table2_exact.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_paper_exact_row():
    row = _paper_row()
    e, c = ex.exact(int(row["L"]), row["beta"])
    assert abs(e - row["e"]) < 5e-9
    assert abs(c - row["C_V"]) < 5e-9


def test_golden_exact_table_matches():
    import json
    with open(os.path.join(GOLDEN, "exact_ising.json")) as f:
        table = json.load(f)
    for rec in table["values"][:3]:
        e, c = ex.exact(rec["L"], rec["beta"])
        assert abs(e - rec["e"]) < 1e-12 and abs(c - rec["C_V"]) < 1e-11
