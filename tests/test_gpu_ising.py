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

KINDS = ["lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "xs1024w", "philox4x32_7", "lcg32_sub", "lcg64_sub",
         "mwc_diff"]
# MWC_DIFF allows at most 2^21 streams, i.e. L <= 2896
KINDS_L4096 = [k for k in KINDS if k != "mwc_diff"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run_both(rx, orc, L, kind, beta, sweeps, seed=1, chunks=(None,), plan=None):
    lat = rx.ising_create(L, kind, seed)
    if plan is not None:
        rx.ising_set_plan(lat, plan)
        assert rx.ising_info(lat)["strips"] == plan
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
@pytest.mark.parametrize("L", [16, 32, 48, 80, 160])
def test_sweep_parity(rngx, orc, kind, L):
    print(f"case ising {kind} L={L}", flush=True)
    for beta in (0.4, ex.BETA_C):
        _run_both(rngx, orc, L, kind, beta, 25, chunks=(10, 1, 14))


@pytest.mark.parametrize("kind", KINDS)
def test_long_parity_L32(rngx, orc, kind):
    """10^4 sweeps at beta_c, energy trace, spins and states bit-exact."""
    print(f"case ising long {kind}", flush=True)
    _run_both(rngx, orc, 32, kind, ex.BETA_C, 10_000)


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


@pytest.mark.parametrize("kind", KINDS_L4096)
def test_large_lattice_parity(rngx, orc, kind):
    """L = 4096 (the throughput workload) for 10 sweeps in two calls, bit-exact."""
    print(f"case ising L=4096 {kind}", flush=True)
    lat = _run_both(rngx, orc, 4096, kind, 0.4, 10, chunks=(6, 4))
    assert rngx.ising_info(lat)["strips"] == 256


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("L", [368, 512, 1024, 2048, 2064])
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


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "philox4x32_10"])
@pytest.mark.parametrize("L", [512, 2048])
def test_every_plan_gives_the_same_lattice(rngx, orc, kind, L):
    """Each autotuner candidate (every strip count that fits, and the
    per-pass path) gives the oracle's spins, energies and streams."""
    plans = rngx.ising_plans(rngx.ising_create(L, kind, 1))
    assert plans[-1] == 0 and len(plans) >= 2 and plans[:-1] == sorted(plans[:-1], reverse=True)
    for strips in plans:
        print(f"case ising plan {kind} L={L} strips={strips}", flush=True)
        _run_both(rngx, orc, L, kind, 0.4, 3, chunks=(2, 1), plan=strips)


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32"])
def test_plans_with_several_strips_per_cu(rngx, orc, kind):
    """At L = 4096 the tuner's candidates include more strips than CUs (8
    rows each), made resident by more units and fewer threads per strip (for
    the kinds whose strips then fit two to a CU's LDS); they give the
    oracle's lattice too."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    plans = rngx.ising_plans(rngx.ising_create(4096, kind, 1))
    many = [p for p in plans if p > n_cu]
    assert many, plans
    for strips in many:
        print(f"case ising plan {kind} L=4096 strips={strips}", flush=True)
        _run_both(rngx, orc, 4096, kind, 0.4, 2, chunks=(2,), plan=strips)


def test_autotune_restores_the_lattice(rngx, orc):
    L, kind = 1024, "xs1024w"
    print("case ising autotune", flush=True)
    lat = rngx.ising_create(L, kind, 4)
    rngx.ising_sweep(lat, 0.4, 2)
    spins = rngx.ising_get_spins(lat)
    state = rngx.rng_get_state(rngx.ising_rng(lat))
    ms = rngx.ising_autotune(lat, 0.4, 3, reps=1)
    plans = rngx.ising_plans(lat)
    assert len(ms) == len(plans) and all(m > 0 for m in ms)
    assert rngx.ising_info(lat)["strips"] == plans[int(np.argmin(ms))]
    assert np.array_equal(rngx.ising_get_spins(lat), spins)
    assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lat)), state)
    # and it still computes the oracle's lattice
    sp, st = orc.ising_create(L, kind, 4)
    orc.ising_sweeps(L, kind, 0.4, st, sp, 2)
    tr = torch.zeros(3, dtype=torch.int32, device="cuda")
    rngx.ising_sweep(lat, 0.4, 3, tr)
    want = orc.ising_sweeps(L, kind, 0.4, st, sp, 3)
    assert np.array_equal(tr.cpu().numpy(), want)
    assert np.array_equal(rngx.ising_get_spins(lat).ravel(), sp.ravel())
    with pytest.raises(rngx.RngxError):
        rngx.ising_set_plan(lat, 7)


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


GATED = ("xs1024w", "philox4x32_10", "philox4x32_7", "mwc", "lcg64", "mwc_diff")  # LCG32, XORWOW: reported only


def test_statistics_all_kinds(rngx):
    """e and C_V against the exact finite-lattice values for every kind at
    L = 32 and 64, beta = 0.4 and beta_c: 10^5 equilibration sweeps, 10^6
    measured, 20 bins, jackknife errors.  Gate |z| <= 3 for XS1024W, Philox,
    MWC and LCG64 (fixed seeds); LCG32 and XORWOW are printed, not gated (the
    paper reports both deviating).  One batch per kind, all six on their own
    streams at once."""
    n_eq, n_meas = 100_000, 1_000_000
    cases = [(32, 0.4), (32, ex.BETA_C), (64, 0.4), (64, ex.BETA_C)]
    runs = []
    for kind in KINDS:
        lats = [rngx.ising_create(L, kind, 1) for L, _ in cases]
        trs = [torch.zeros(n_eq + n_meas, dtype=torch.int32, device="cuda") for _ in cases]
        b = rngx.ising_batch_create(lats, [beta for _, beta in cases], [n_eq + n_meas] * len(cases), trs)
        s = torch.cuda.Stream()
        rngx.ising_batch_run(b, stream=s)
        runs.append((kind, b, trs, s))
    torch.cuda.synchronize()
    bad = []
    for kind, b, trs, _ in runs:
        for (L, beta), tr in zip(cases, trs):
            e, se, c, sc = isingstats.estimates(tr[n_eq:].cpu().numpy(), L * L, beta)
            ee, ce = _exact(L, beta)
            ze, zc = (e - ee) / se, (c - ce) / sc
            print(f"stat {kind:14s} L={L} beta={beta:.5f} e={e:.6f}+-{se:.6f} z={ze:+.2f} "
                  f"C={c:.5f}+-{sc:.5f} z={zc:+.2f}", flush=True)
            if kind in GATED and (abs(ze) > 3 or abs(zc) > 3):
                bad.append((kind, L, beta, round(ze, 2), round(zc, 2)))
        b.destroy()
    assert not bad, bad


# ---------------------------------------------------------------- batches
def _batch_case(rngx, kind, seed, n=24, max_L=512, big=(400, 512)):
    rng = np.random.default_rng(seed)
    Ls = list(rng.choice(np.arange(16, max_L + 1, 16), size=n - len(big))) + list(big)
    betas = list(rng.uniform(0.3, 0.6, size=n))
    sweeps = list(rng.integers(1, 12, size=n))
    return [int(L) for L in Ls], betas, [int(x) for x in sweeps]


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "philox4x32_10", "xorwow"])
def test_batch_equals_individual_sweeps(rngx, kind):
    """One launch over replicas of uneven L and beta (on-chip and streamed)
    gives every replica exactly what ising_sweep gives it alone."""
    print(f"case batch {kind}", flush=True)
    Ls, betas, sweeps = _batch_case(rngx, kind, 5)
    lats = [rngx.ising_create(L, kind, 100 + i) for i, L in enumerate(Ls)]
    twins = [rngx.ising_create(L, kind, 100 + i) for i, L in enumerate(Ls)]
    traces = [torch.full((s,), 7, dtype=torch.int32, device="cuda") for s in sweeps]
    batch = rngx.ising_batch_create(lats, betas, sweeps, traces)
    for rep in range(2):
        rngx.ising_batch_run(batch)
        for i, tw in enumerate(twins):
            tt = torch.zeros(sweeps[i], dtype=torch.int32, device="cuda")
            rngx.ising_sweep(tw, betas[i], sweeps[i], tt)
            assert torch.equal(traces[i], tt), (rep, i, Ls[i])
            assert np.array_equal(rngx.ising_get_spins(lats[i]), rngx.ising_get_spins(tw)), (rep, i, Ls[i])
            assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[i])),
                                  rngx.rng_get_state(rngx.ising_rng(tw))), (rep, i)


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32"])
def test_batch_gangs_and_memory_replicas(rngx, orc, kind):
    """Large replicas run as gangs of strip workgroups or, beyond the largest
    gang, in memory (L = 4096); each equals ising_sweep on the lattice alone.
    XS1024W gangs: 1024 = 16 x 64 rows; 1008 = 15 x 64 + 48; 976 = 15 x 64
    + 16 (a last strip of one XS1024W row of instances); 784 = 9 x 80 + 64;
    272 = 2 x 136; 2048 = 64 x 32, the largest gang.  LCG32: 1008 = 16 x 63
    (odd rows), 976 = 14 x 66 + 52, 784 = 9 x 79 + 73."""
    print(f"case batch gangs {kind}", flush=True)
    Ls = [1024, 1008, 784, 272, 2048, 976, 4096, 48]
    betas, sweeps = [0.4, 0.35, 0.5, 0.44, 0.41, 0.45, 0.38, 0.3], [3, 2, 4, 3, 2, 3, 2, 5]
    lats = [rngx.ising_create(L, kind, 300 + i) for i, L in enumerate(Ls)]
    twins = [rngx.ising_create(L, kind, 300 + i) for i, L in enumerate(Ls)]
    refs = [orc.ising_create(L, kind, 300 + i) for i, L in enumerate(Ls)]
    traces = [torch.full((s,), 7, dtype=torch.int32, device="cuda") for s in sweeps]
    batch = rngx.ising_batch_create(lats, betas, sweeps, traces)
    for rep in range(2):
        rngx.ising_batch_run(batch)
        assert rngx.ising_batch_status(batch) == 0
        # the oracle directly: every gang (uneven last strips) and the
        # replica streamed through memory (L = 4096)
        for i, (sp, st) in enumerate(refs):
            want = orc.ising_sweeps(Ls[i], kind, betas[i], st, sp, sweeps[i])
            assert np.array_equal(traces[i].cpu().numpy(), want), (rep, i, Ls[i])
            assert np.array_equal(rngx.ising_get_spins(lats[i]).ravel(), sp), (rep, i, Ls[i])
            assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[i])), st), (rep, i, Ls[i])
        for i, tw in enumerate(twins):
            tt = torch.zeros(sweeps[i], dtype=torch.int32, device="cuda")
            rngx.ising_sweep(tw, betas[i], sweeps[i], tt)
            assert torch.equal(traces[i], tt), (rep, i, Ls[i])
            assert np.array_equal(rngx.ising_get_spins(lats[i]), rngx.ising_get_spins(tw)), (rep, i, Ls[i])
            assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[i])),
                                  rngx.rng_get_state(rngx.ising_rng(tw))), (rep, i)


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32"])
def test_batch_every_size_to_1040(rngx, kind):
    """One batch of every L = 16, 32, ..., 1040: on-chip replicas and gangs
    with every last-strip height the strip rule produces, more items than
    resident workgroups (gangs start while others run); each replica equals
    ising_sweep on the lattice alone."""
    print(f"case batch every size {kind}", flush=True)
    Ls = list(range(16, 1041, 16))
    rng = np.random.default_rng(17)
    betas = [float(b) for b in rng.uniform(0.3, 0.6, size=len(Ls))]
    sweeps = [int(x) for x in rng.integers(1, 4, size=len(Ls))]
    lats = [rngx.ising_create(L, kind, 500 + i) for i, L in enumerate(Ls)]
    twins = [rngx.ising_create(L, kind, 500 + i) for i, L in enumerate(Ls)]
    traces = [torch.full((s,), 7, dtype=torch.int32, device="cuda") for s in sweeps]
    batch = rngx.ising_batch_create(lats, betas, sweeps, traces)
    rngx.ising_batch_run(batch)
    for i, tw in enumerate(twins):
        tt = torch.zeros(sweeps[i], dtype=torch.int32, device="cuda")
        rngx.ising_sweep(tw, betas[i], sweeps[i], tt)
        assert torch.equal(traces[i], tt), Ls[i]
        assert np.array_equal(rngx.ising_get_spins(lats[i]), rngx.ising_get_spins(tw)), Ls[i]
        assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[i])),
                              rngx.rng_get_state(rngx.ising_rng(tw))), Ls[i]


def test_batch_gang_behind_long_replicas(rngx, orc):
    """A gang whose first strip is claimed while every other workgroup runs a
    long on-chip replica: its remaining strips start only when those finish
    (about a second later), so its members must wait to start together
    rather than give up.  Regression test for gang members that timed out
    waiting for strips not yet started; the gang is compared with the
    oracle and every replica must be valid."""
    kind = "xs1024w"
    probe = rngx.ising_batch_create([rngx.ising_create(64, kind, 1)], [0.4], [1])
    grid = rngx.ising_batch_info(probe)["resident"]
    probe.destroy()
    gang_L, gang_sweeps = 1024, 3
    n_long = max(grid, 2) - 2  # leaves two workgroups for the gang's first strips
    Ls = [64] * n_long + [gang_L]
    betas = [0.4] * n_long + [0.44]
    sweeps = [400_000] * n_long + [gang_sweeps]
    print(f"case batch gang behind {n_long} long replicas (grid {grid})", flush=True)
    lats = [rngx.ising_create(L, kind, 900 + i) for i, L in enumerate(Ls)]
    tr = torch.zeros(gang_sweeps, dtype=torch.int32, device="cuda")
    batch = rngx.ising_batch_create(lats, betas, sweeps, [None] * n_long + [tr])
    info = rngx.ising_batch_info(batch)
    assert info["items"] > info["grid"]  # the gang cannot start in the first wave
    rngx.ising_batch_run(batch)
    assert rngx.ising_batch_status(batch) == 0
    sp, st = orc.ising_create(gang_L, kind, 900 + n_long)
    want = orc.ising_sweeps(gang_L, kind, 0.44, st, sp, gang_sweeps)
    assert np.array_equal(tr.cpu().numpy(), want)
    assert np.array_equal(rngx.ising_get_spins(lats[-1]).ravel(), sp)
    assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[-1])), st)


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "philox4x32_10", "xorwow"])
def test_batch_every_shape_matches_oracle(rngx, orc, kind):
    """Every batch launch shape (threads per workgroup, sites per thread,
    strip LDS) tiles the replicas differently -- one workgroup, gangs of
    strips or streaming through memory -- and every one gives the oracle's
    spins, energies and stream states.  The runs follow each other, the
    oracle advanced in step."""
    Ls = [16, 48, 128, 256, 400, 1008, 2048, 64]
    betas = [0.3, 0.41, 0.44, 0.5, 0.38, 0.45, 0.42, 0.6]
    sweeps = [3, 2, 2, 3, 2, 2, 2, 4]
    lats = [rngx.ising_create(L, kind, 800 + i) for i, L in enumerate(Ls)]
    refs = [orc.ising_create(L, kind, 800 + i) for i, L in enumerate(Ls)]
    traces = [torch.full((s,), 7, dtype=torch.int32, device="cuda") for s in sweeps]
    batch = rngx.ising_batch_create(lats, betas, sweeps, traces)
    for shape in range(len(rngx.ising_batch_shapes())):
        print(f"case batch shape {kind} {shape}", flush=True)
        rngx.ising_batch_set_shape(batch, shape)
        assert rngx.ising_batch_get_shape(batch) == shape
        rngx.ising_batch_run(batch)
        assert rngx.ising_batch_status(batch) == 0
        for i, (sp, st) in enumerate(refs):
            want = orc.ising_sweeps(Ls[i], kind, betas[i], st, sp, sweeps[i])
            assert np.array_equal(traces[i].cpu().numpy(), want), (shape, i, Ls[i])
            assert np.array_equal(rngx.ising_get_spins(lats[i]).ravel(), sp), (shape, i, Ls[i])
            assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[i])), st), (shape, i, Ls[i])


def test_batch_autotune_restores_replicas(rngx):
    """The batch autotuner times every shape, keeps one, and leaves every
    replica's spins and streams as they were; runs afterwards still equal
    ising_sweep on each lattice alone."""
    kind = "xs1024w"
    Ls, betas, sweeps = _batch_case(rngx, kind, 21, n=16, max_L=512, big=(1024,))
    sweeps = [s * 40 for s in sweeps]  # tuned at most 50 sweeps: scaled down
    lats = [rngx.ising_create(L, kind, 900 + i) for i, L in enumerate(Ls)]
    twins = [rngx.ising_create(L, kind, 900 + i) for i, L in enumerate(Ls)]
    traces = [torch.full((s,), 7, dtype=torch.int32, device="cuda") for s in sweeps]
    batch = rngx.ising_batch_create(lats, betas, sweeps, traces)
    spins0 = [rngx.ising_get_spins(x) for x in lats]
    states0 = [rngx.rng_get_state(rngx.ising_rng(x)) for x in lats]
    ms = rngx.ising_batch_autotune(batch, max_sweeps=50, reps=1)
    print(f"case batch autotune ms={ms}", flush=True)
    assert len(ms) == len(rngx.ising_batch_shapes()) and all(m > 0 for m in ms)
    assert ms[rngx.ising_batch_get_shape(batch)] == min(ms)
    for i, x in enumerate(lats):
        assert np.array_equal(rngx.ising_get_spins(x), spins0[i]), i
        assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(x)), states0[i]), i
        assert int(traces[i][0]) == 7  # tuning runs write no trace
    assert rngx.ising_batch_status(batch) == 0
    rngx.ising_batch_run(batch)
    for i, tw in enumerate(twins):
        tt = torch.zeros(sweeps[i], dtype=torch.int32, device="cuda")
        rngx.ising_sweep(tw, betas[i], sweeps[i], tt)
        assert torch.equal(traces[i], tt), (i, Ls[i])
        assert np.array_equal(rngx.ising_get_spins(lats[i]), rngx.ising_get_spins(tw)), (i, Ls[i])
        assert np.array_equal(rngx.rng_get_state(rngx.ising_rng(lats[i])),
                              rngx.rng_get_state(rngx.ising_rng(tw))), i


def test_batch_small_replicas_match_oracle(rngx, orc):
    kind = "xs1024w"
    Ls, betas, sweeps = [16, 48, 96], [0.31, 0.44, 0.58], [3, 5, 2]
    lats = [rngx.ising_create(L, kind, 7 + i) for i, L in enumerate(Ls)]
    traces = [torch.zeros(s, dtype=torch.int32, device="cuda") for s in sweeps]
    batch = rngx.ising_batch_create(lats, betas, sweeps, traces)
    rngx.ising_batch_run(batch)
    for i, L in enumerate(Ls):
        sp, st = orc.ising_create(L, kind, 7 + i)
        tr = orc.ising_sweeps(L, kind, betas[i], st, sp, sweeps[i])
        assert np.array_equal(traces[i].cpu().numpy(), tr)
        assert np.array_equal(rngx.ising_get_spins(lats[i]).ravel(), sp)


@pytest.mark.parametrize("shape", [0, 4])
def test_batch_graph_replay(rngx, shape):
    """The batch run captured in a HIP graph (under the default launch shape
    and the 256-thread one): every replay equals an eager run of a batch
    left at the default shape."""
    kind = "xs1024w"
    Ls, betas, sweeps = _batch_case(rngx, kind, 9, n=10, max_L=256, big=(320,))
    a = [rngx.ising_create(L, kind, 50 + i) for i, L in enumerate(Ls)]
    b = [rngx.ising_create(L, kind, 50 + i) for i, L in enumerate(Ls)]
    ta = [torch.zeros(s, dtype=torch.int32, device="cuda") for s in sweeps]
    tb = [torch.zeros(s, dtype=torch.int32, device="cuda") for s in sweeps]
    ba = rngx.ising_batch_create(a, betas, sweeps, ta)
    bb = rngx.ising_batch_create(b, betas, sweeps, tb)
    rngx.ising_batch_set_shape(ba, shape)
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        rngx.ising_batch_run(ba, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        rngx.ising_batch_run(bb)
        torch.cuda.synchronize()
        for i in range(len(Ls)):
            assert torch.equal(ta[i], tb[i]), (rep, i)
            assert np.array_equal(rngx.ising_get_spins(a[i]), rngx.ising_get_spins(b[i])), (rep, i)


def test_batch_argument_errors(rngx):
    x = rngx.ising_create(32, "lcg32", 1)
    y = rngx.ising_create(32, "mwc", 1)
    with pytest.raises(rngx.RngxError):
        rngx.ising_batch_create([x, x], [0.4, 0.4], [1, 1])
    with pytest.raises(rngx.RngxError):
        rngx.ising_batch_create([x, y], [0.4, 0.4], [1, 1])
    with pytest.raises(rngx.RngxError):
        rngx.ising_batch_create([x], [float("nan")], [1])
    b = rngx.ising_batch_create([x], [0.4], [1])
    assert rngx.load().ising_destroy(x.handle) == -7  # held by the batch
    b.destroy()


# ---------------------------------------------------------------- multi-hit
def _run_hits(rx, orc, L, kind, beta, sweeps, hits, plan=None, chunks=(None,)):
    lat = rx.ising_create(L, kind, 3)
    if plan is not None:
        rx.ising_set_plan(lat, plan)
    sp, st = orc.ising_create(L, kind, 3)
    for n in chunks:
        n = sweeps if n is None else n
        tr = torch.zeros(n, dtype=torch.int32, device="cuda")
        rx.ising_sweep_hits(lat, beta, n, hits, tr)
        want_tr = orc.ising_sweeps(L, kind, beta, st, sp, n, hits=hits)
        assert np.array_equal(tr.cpu().numpy(), want_tr), (L, kind, beta, hits)
        assert np.array_equal(rx.ising_get_spins(lat).ravel(), sp), (L, kind, beta, hits)
        assert np.array_equal(rx.rng_get_state(rx.ising_rng(lat)), st), (L, kind, beta, hits)
    return lat


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("hits", [2, 3])
def test_multihit_parity(rngx, orc, kind, hits):
    """One workgroup (L = 32) and several strips (L = 512), bit-exact."""
    print(f"case ising multihit {kind} hits={hits}", flush=True)
    for beta in (0.4, ex.BETA_C):
        _run_hits(rngx, orc, 32, kind, beta, 12, hits, chunks=(5, 7))
    lat = _run_hits(rngx, orc, 512, kind, 0.4, 3, hits)
    assert rngx.ising_info(lat)["strips"] > 1


@pytest.mark.parametrize("kind", KINDS)
def test_multihit_per_pass_path_and_many_hits(rngx, orc, kind):
    """The per-pass kernels (plan 0) with 2 hits, and 100 hits on chip."""
    print(f"case ising multihit passes {kind}", flush=True)
    _run_hits(rngx, orc, 64, kind, 0.4, 3, 2, plan=0)
    _run_hits(rngx, orc, 32, kind, ex.BETA_C, 2, 100)


def test_multihit_extremes_and_errors(rngx, orc):
    for beta in (0.0, 1e9):
        _run_hits(rngx, orc, 48, "lcg32", beta, 3, 2)
        _run_hits(rngx, orc, 48, "xs1024w", beta, 3, 3)
    lat = rngx.ising_create(32, "lcg32", 1)
    for bad in (0, (1 << 20) + 1):
        with pytest.raises(rngx.RngxError):
            rngx.ising_sweep_hits(lat, 0.4, 1, bad)


def test_multihit_statistics(rngx):
    """k = 2 leaves the equilibrium unchanged: XS1024W at L = 32, beta_c."""
    L, beta, n_eq, n_meas = 32, ex.BETA_C, 50_000, 500_000
    lat = rngx.ising_create(L, "xs1024w", 7)
    rngx.ising_sweep_hits(lat, beta, n_eq, 2)
    tr = torch.zeros(n_meas, dtype=torch.int32, device="cuda")
    rngx.ising_sweep_hits(lat, beta, n_meas, 2, tr)
    e, se, c, sc = isingstats.estimates(tr.cpu().numpy(), L * L, beta)
    ee, ce = _exact(L, beta)
    print(f"stat multihit k=2 xs1024w L={L} e={e:.6f}+-{se:.6f} z={(e - ee) / se:+.2f} "
          f"C={c:.5f}+-{sc:.5f} z={(c - ce) / sc:+.2f}", flush=True)
    assert abs(e - ee) < 3 * se
    assert abs(c - ce) < 3 * sc


def test_substream_lcg32_fails_the_ising_test(rngx):
    """Table 2's checkerboard rows at L = 1024, beta = 0.4: LCG32 drawn as
    sub-streams of one sequence (eq. lcg_skipping with t = S) misses the exact
    energy by many standard errors, LCG32 with per-stream seeds does not."""
    L, beta, n_eq, n_meas = 1024, 0.4, 2000, 20000
    ee, ce = _exact(L, beta)
    z = {}
    for kind in ("lcg32_sub", "lcg32", "lcg64_sub"):
        lat = rngx.ising_create(L, kind, 1)
        rngx.ising_sweep(lat, beta, n_eq)
        tr = torch.zeros(n_meas, dtype=torch.int32, device="cuda")
        rngx.ising_sweep(lat, beta, n_meas, tr)
        e, se, c, sc = isingstats.estimates(tr.cpu().numpy(), L * L, beta)
        z[kind] = ((e - ee) / se, (c - ce) / sc)
        print(f"stat table2 {kind:10s} L={L} e={e:.7f}+-{se:.7f} z={z[kind][0]:+.1f} "
              f"C={c:.5f}+-{sc:.5f} z={z[kind][1]:+.1f}", flush=True)
    assert abs(z["lcg32_sub"][0]) > 20
    assert abs(z["lcg32"][0]) < 4 and abs(z["lcg32"][1]) < 4


@pytest.mark.parametrize("L", [512, 1008])
def test_xs1024w_strips_with_uneven_step_counts(rngx, orc, L):
    """The strip kernel derives the XS1024W Weyl word of a pass from the
    call's start when every instance of a strip has taken the same number of
    steps, and holds and steps it per unit otherwise: step counts that
    differ in the lower half of the lattice only (its strips take the
    per-unit form, the others the shared one), then all equal again at a
    count past 2^32 -- bit-exact with the oracle every time.  At L = 1008
    (126 units of 8 sites per row, every strip plan in turn) instances
    straddle rows and, for strips whose height is not a multiple of 8, strips."""
    print(f"case xs1024w step counts L={L}", flush=True)
    probe = rngx.ising_create(L, "xs1024w", 4)
    plans = [p for p in rngx.ising_plans(probe) if p > 1] if L == 1008 else [rngx.ising_info(probe)["strips"]]
    assert plans and plans[0] > 1
    for strips in plans:
        print(f"case xs1024w step counts L={L} strips={strips}", flush=True)
        lat = rngx.ising_create(L, "xs1024w", 4)
        rngx.ising_set_plan(lat, strips)
        g = rngx.ising_rng(lat)
        sp, st = orc.ising_create(L, "xs1024w", 4)
        S = L * L // 4
        G = S // 32
        n = st[4 * S:4 * S + 8 * G].view(np.uint64)
        for rep in range(3):
            if rep == 1:  # uneven in the lower half
                n[G // 2:] += np.arange(G - G // 2, dtype=np.uint64) % np.uint64(5)
                rngx.rng_set_state(g, st)
            if rep == 2:
                n[:] = np.uint64((1 << 32) + 12345)  # equal again
                rngx.rng_set_state(g, st)
            tr = torch.zeros(3, dtype=torch.int32, device="cuda")
            rngx.ising_sweep(lat, 0.42, 3, tr)
            want = orc.ising_sweeps(L, "xs1024w", 0.42, st, sp, 3)
            assert np.array_equal(tr.cpu().numpy(), want), (strips, rep)
            assert np.array_equal(rngx.ising_get_spins(lat).ravel(), sp), (strips, rep)
            assert np.array_equal(rngx.rng_get_state(g), st), (strips, rep)


@pytest.mark.parametrize("kind", ["philox4x32_10", "philox4x32_7"])
def test_philox_strips_with_uneven_positions(rngx, orc, kind):
    """The strip kernel makes each Philox block once per sweep when all
    streams of a strip stand at one block boundary, and falls back to the
    per-stream form otherwise: positions that are equal but not a multiple of
    4, positions that differ in the lower half of the lattice only (its
    strips take the fallback, the others the sweep form), and all equal
    again -- bit-exact with the oracle every time."""
    L = 512
    print(f"case philox positions {kind}", flush=True)
    lat = rngx.ising_create(L, kind, 4)
    assert rngx.ising_info(lat)["strips"] > 1
    g = rngx.ising_rng(lat)
    sp, st = orc.ising_create(L, kind, 4)
    S = L * L // 4
    rngx.rng_skip(g, 1)  # every stream at position 1
    orc.jump(kind, S, st, 1)
    pos = st[8 * S:].view(np.uint64)
    for rep in range(3):
        if rep == 1:  # uneven in the lower half
            pos[S // 2:] += np.arange(S - S // 2, dtype=np.uint64) % np.uint64(7)
            rngx.rng_set_state(g, st)
        if rep == 2:
            pos[:] = np.uint64(4 * 1000)  # even and aligned again
            rngx.rng_set_state(g, st)
        tr = torch.zeros(3, dtype=torch.int32, device="cuda")
        rngx.ising_sweep(lat, 0.42, 3, tr)
        want = orc.ising_sweeps(L, kind, 0.42, st, sp, 3)
        assert np.array_equal(tr.cpu().numpy(), want), rep
        assert np.array_equal(rngx.ising_get_spins(lat).ravel(), sp), rep
        assert np.array_equal(rngx.rng_get_state(g), st), rep
