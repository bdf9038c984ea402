"""GPU <-> oracle parity of the checkerboard Metropolis update: spins, energy
trace and generator state bit-exact after every call; statistics against the
exact finite-lattice values."""
import json
import os

import numpy as np
import pytest
import torch

import isingstats
from oracle import exact_ising as ex

pytestmark = pytest.mark.gpu

KINDS = ["lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "xs1024w"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run_both(rx, orc, L, kind, beta, sweeps, seed=1, chunks=(None,)):
    lat = rx.ising_create(L, kind, seed)
    sp, st = orc.ising_create(L, kind, seed)
    assert np.array_equal(rx.ising_get_spins(lat).ravel(), sp)
    for n in chunks:
        n = sweeps if n is None else n
        tr = torch.zeros(n, dtype=torch.int32, device="cuda")
        rx.ising_sweep(lat, beta, n, tr)
        want_tr = orc.ising_sweeps(L, kind, beta, st, sp, n)
        assert np.array_equal(tr.cpu().numpy(), want_tr), (L, kind, beta)
        assert np.array_equal(rx.ising_get_spins(lat).ravel(), sp), (L, kind, beta)
        assert np.array_equal(rx.rng_get_state(rx.ising_rng(lat)), st), (L, kind, beta)
    return lat


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("L", [16, 32, 48, 80])
def test_sweep_parity(rngx, orc, kind, L):
    print(f"case ising {kind} L={L}", flush=True)
    for beta in (0.4, ex.BETA_C):
        _run_both(rngx, orc, L, kind, beta, 25, chunks=(10, 1, 14))


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32"])
def test_extreme_temperatures(rngx, orc, kind):
    for beta in (0.0, 1e9, 0.05, 3.0):
        _run_both(rngx, orc, 32, kind, beta, 6)


def test_colour_order_neel(rngx):
    L = 16
    lat = rngx.ising_create(L, "lcg32", 1)
    y, x = np.mgrid[0:L, 0:L]
    rngx.ising_set_spins(lat, np.where((x + y) % 2 == 0, 1, -1))
    rngx.ising_sweep(lat, 1e9, 1)
    assert np.all(rngx.ising_get_spins(lat) == -1)


def test_sweep_without_trace_and_argument_errors(rngx, orc):
    L, kind = 32, "mwc"
    lat = rngx.ising_create(L, kind, 4)
    sp, st = orc.ising_create(L, kind, 4)
    rngx.ising_sweep(lat, 0.4, 7)
    orc.ising_sweeps(L, kind, 0.4, st, sp, 7, trace=False)
    assert np.array_equal(rngx.ising_get_spins(lat).ravel(), sp)
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(rngx.RngxError):
            rngx.ising_sweep(lat, bad, 1)
    with pytest.raises(rngx.RngxError):
        rngx.ising_set_spins(lat, np.zeros(L * L))
    assert np.array_equal(rngx.ising_get_spins(lat).ravel(), sp)
    # the lattice's generator cannot be destroyed on its own
    assert rngx.load().rng_destroy(rngx.ising_rng(lat).handle) == -1


def test_checkpoint_resume(rngx):
    L, kind = 64, "xs1024w"
    a = rngx.ising_create(L, kind, 8)
    rngx.ising_sweep(a, 0.42, 10)
    spins = rngx.ising_get_spins(a)
    image = rngx.rng_get_state(rngx.ising_rng(a))
    tra = torch.zeros(10, dtype=torch.int32, device="cuda")
    rngx.ising_sweep(a, 0.42, 10, tra)
    b = rngx.ising_create(L, kind, 999)
    rngx.ising_set_spins(b, spins)
    rngx.rng_set_state(rngx.ising_rng(b), image)
    trb = torch.zeros(10, dtype=torch.int32, device="cuda")
    rngx.ising_sweep(b, 0.42, 10, trb)
    assert torch.equal(tra, trb)
    assert np.array_equal(rngx.ising_get_spins(a), rngx.ising_get_spins(b))


@pytest.mark.parametrize("kind", ["xs1024w", "philox4x32_10", "lcg32", "xorwow"])
def test_large_lattice_parity(rngx, orc, kind):
    """L = 4096 (the throughput workload) for 3 sweeps in two calls, bit-exact."""
    print(f"case ising L=4096 {kind}", flush=True)
    lat = _run_both(rngx, orc, 4096, kind, 0.4, 3, chunks=(2, 1))
    assert rngx.ising_info(lat)["strips"] == 256


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("L", [368, 512, 1024, 2064])
def test_multi_strip_parity(rngx, orc, kind, L):
    """Lattices held as several on-chip strips that exchange halo rows."""
    print(f"case ising strips {kind} L={L}", flush=True)
    lat = _run_both(rngx, orc, L, kind, ex.BETA_C, 7, chunks=(4, 3))
    assert rngx.ising_info(lat)["strips"] > 1


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "philox4x32_10"])
def test_per_pass_path_parity(rngx, orc, kind):
    """L = 8192 does not fit on chip: one launch per colour pass."""
    print(f"case ising per-pass {kind} L=8192", flush=True)
    lat = _run_both(rngx, orc, 8192, kind, 0.4, 1)
    assert rngx.ising_info(lat)["strips"] == 0


def test_small_lattices_use_one_workgroup(rngx):
    for L in (16, 64, 128, 256):
        for kind in ("lcg32", "xs1024w"):
            assert rngx.ising_info(rngx.ising_create(L, kind, 1))["strips"] == 1


def _exact(L, beta):
    with open(os.path.join(GOLDEN, "exact_ising.json")) as f:
        for rec in json.load(f)["values"]:
            if rec["L"] == L and abs(rec["beta"] - beta) < 1e-15:
                return rec["e"], rec["C_V"]
    raise KeyError((L, beta))


@pytest.mark.parametrize("kind", ["xs1024w", "philox4x32_10"])
@pytest.mark.parametrize("beta", [0.4, ex.BETA_C])
def test_statistics_L32(rngx, kind, beta):
    """e and C_V within 3 standard errors of the exact L = 32 values."""
    L, n_eq, n_meas = 32, 20000, 200000
    lat = rngx.ising_create(L, kind, 1)
    rngx.ising_sweep(lat, beta, n_eq)
    tr = torch.zeros(n_meas, dtype=torch.int32, device="cuda")
    rngx.ising_sweep(lat, beta, n_meas, tr)
    e, se, c, sc = isingstats.estimates(tr.cpu().numpy(), L * L, beta)
    ee, ce = _exact(L, beta)
    print(f"L={L} {kind} beta={beta:.5f} e={e:.6f}+-{se:.6f} (exact {ee:.6f}) "
          f"C={c:.5f}+-{sc:.5f} (exact {ce:.5f})", flush=True)
    assert abs(e - ee) < 3 * se
    assert abs(c - ce) < 3 * sc
