"""Benchmark of the per-stream generator hot path on one MI355X.

Headline (one JSON line): bulk fill with the paper's XORShift-1024/Weyl
generator, 2^20 streams x 4096 uint32 outputs per step (16 GiB written per
step), inputs (generator state) resident in HBM, in Gsamples/s.  One step is
one rng_fill_u32 call = one kernel launch; it is timed with HIP events on the
stream the kernel runs on.

The same line carries, under "parts", every generator's u32 fill, FP32 fill,
consume-only rate and jump-ahead time at the same size, a plain write
kernel's ceiling, and checkerboard-Ising throughput at L = 4096 in flips/ns;
"roofline" for the dominant kernel and "cpu_baseline" for the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
S_FULL, COUNT_FULL = 1 << 20, 4096
KINDS = ["xs1024w", "lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "philox4x32_7", "mwc_diff", "lfg521",
         "lfg1279"]
# kinds whose L = 4096 lattice fits their stream count (MWC_DIFF: at most 2^21 streams)
ISING_KINDS = [k for k in KINDS if k != "mwc_diff"]
RAGGED_KINDS = [k for k in KINDS if not k.startswith("lfg")]  # ragged fills take no LFG kind
# state bytes read + written once per launch, per stream (MWC_DIFF: y read and
# written, the multiplier read only; LFG: r words per 1024-stream instance)
STATE_BYTES = {"lcg32": 4, "lcg64": 8, "mwc": 8, "xorwow": 24, "philox4x32_10": 16, "philox4x32_7": 16,
               "xs1024w": 4 + 8 / 32, "mwc_diff": 10, "lfg521": 4 * 521 / 1024, "lfg1279": 4 * 1279 / 1024}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "xs1024w_fill_u32_2p20x4096_hbm_traffic.md")
PROFILE_ISING_VALU = os.path.join(ROOT, "profiles", "ising_valu_L4096_all_kinds.md")
KERNEL_SOURCES = ["paper_1204_6193_amd/csrc/gen.hip", "paper_1204_6193_amd/csrc/rngx_device.h"]
ISING_SOURCES = ["paper_1204_6193_amd/csrc/ising.hip", "paper_1204_6193_amd/csrc/rngx_device.h"]
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 instruction
# occupies a SIMD for 4 cycles)
VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_json(path):
    """The json block of a committed profile summary, or None."""
    try:
        with open(path) as f:
            return json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None


def ising_valu_per_site():
    """VALU lane-instructions per site update for each kind's L = 4096
    kernel, from the committed counter summary, while the Ising sources are
    the ones it was taken from."""
    rec = profile_json(PROFILE_ISING_VALU)
    if not rec or rec.get("kernel_hash") != kernel_hash(ISING_SOURCES):
        return {}
    return {k: v["valu_lane_instr_per_site"] for k, v in rec.get("kinds", {}).items()}


def time_launches(fn, steps, warmup):
    """Per-launch durations (ms) from HIP events on torch's current stream,
    which is the stream every call below launches on."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [a.elapsed_time(b) for a, b in evs], wall


def bench_fill(rx, kind, mode, out, steps, warmup, tune=True):
    """Timed fills of one handle; with `tune` the fill autotuner first picks
    the handle's configuration (untimed; it leaves the streams unchanged)."""
    import torch
    g = rx.rng_create(kind, S_FULL, 1)
    tuned = None
    if tune and mode != "consume":
        tune_ms = rx.rng_autotune_fill(g, out, COUNT_FULL, reps=4)
        cfg = rx.rng_fill_configs(kind)[rx.rng_get_fill_config(g)]
        tuned = {"config": {"paced": cfg[0], "streams_per_thread": cfg[1], "block": cfg[2]},
                 "candidates_ms": [round(m, 4) for m in tune_ms]}
    if mode == "u32":
        fn = lambda: rx.rng_fill_u32(g, out, COUNT_FULL)
    elif mode == "f32":
        fo = out.view(torch.float32)
        fn = lambda: rx.rng_fill_f32(g, fo, COUNT_FULL)
    else:
        acc = torch.empty(S_FULL, dtype=torch.int32, device="cuda")
        fn = lambda: rx.rng_consume(g, acc, COUNT_FULL)
    durs, _ = time_launches(fn, steps, warmup)
    ms = sum(durs) / len(durs)
    samples = S_FULL * COUNT_FULL
    out_bytes = samples * 4 if mode != "consume" else S_FULL * 4
    alg_bytes = out_bytes + 2 * STATE_BYTES[kind] * S_FULL
    rec = {"ms": round(ms, 4), "gsamples_s": round(samples / ms / 1e6, 2),
           "gbs": round(alg_bytes / ms / 1e6, 1), "hbm_frac": round(alg_bytes / ms / 1e6 / HBM_PEAK_GBS, 4),
           "ms_min": round(min(durs), 4)}
    if tuned:
        rec["autotune"] = tuned
    return rec


def bench_write_ceiling(out, steps, warmup):
    durs, _ = time_launches(lambda: out.fill_(7), steps, warmup)
    ms = sum(durs) / len(durs)
    return {"ms": round(ms, 4), "gbs": round(out.numel() * 4 / ms / 1e6, 1)}


def bench_skip(rx, kind, reps=5):
    g = rx.rng_create(kind, S_FULL, 1)
    durs, _ = time_launches(lambda: rx.rng_skip(g, (1 << 40) + 12345), reps, 1)
    return round(sum(durs) / len(durs), 4)


def bench_ising(rx, kind, L, sweeps, beta=0.4, hits=1):
    """One call of `sweeps` sweeps (energy trace on), after the plan
    autotuner (untimed; it restores spins and streams) and 5 warm-up sweeps.
    With hits > 1 every visited site gets `hits` updates; flips_per_ns counts
    attempted updates."""
    import torch
    lat = rx.ising_create(L, kind, 1)
    plans = rx.ising_plans(lat)
    tune_ms = rx.ising_autotune(lat, beta, 20, reps=1)
    rx.ising_sweep_hits(lat, beta, 5, hits)
    tr = torch.zeros(sweeps, dtype=torch.int32, device="cuda")
    durs, _ = time_launches(lambda: rx.ising_sweep_hits(lat, beta, sweeps, hits, tr), 1, 0)
    ms = durs[0]
    if rx.ising_status(lat):
        raise RuntimeError(f"Ising {kind} L={L}: a strip gave up waiting; the timed lattice is invalid")
    rec = {"sweeps": sweeps, "ms": round(ms, 3), "flips_per_ns": round(L * L * sweeps * hits / (ms * 1e6), 2),
           "strips": rx.ising_info(lat)["strips"],
           "autotune": {"plans": plans, "ms_per_20_sweeps": [round(m, 3) for m in tune_ms]}}
    per_site = ising_valu_per_site().get(kind) if (L == 4096 and hits == 1) else None
    if per_site:  # VALU roofline: lane-instructions issued per second over the issue peak
        rec["valu_lane_instr_per_site"] = per_site
        rec["valu_frac"] = round(rec["flips_per_ns"] * 1e9 * per_site / VALU_PEAK_LANE_INSTR, 4)
    if hits > 1:
        rec["hits"] = hits
        rec["ns_per_attempted_flip"] = round(ms * 1e6 / (L * L * sweeps * hits), 5)
    return rec


def run_tuned_batch(rx, lats, betas, sweeps, tune_sweeps):
    """Create the batch, autotune its launch shape on runs of at most
    tune_sweeps sweeps (replicas restored afterwards), time one run, check
    every replica's status; returns (ms, shape index, per-shape tuning ms)."""
    batch = rx.ising_batch_create(lats, betas, sweeps)
    tune_ms = rx.ising_batch_autotune(batch, max_sweeps=tune_sweeps, reps=1)
    shape = rx.ising_batch_get_shape(batch)
    durs, _ = time_launches(lambda: rx.ising_batch_run(batch), 1, 0)
    bad = rx.ising_batch_status(batch)
    batch.destroy()
    if bad:
        raise RuntimeError(f"Ising batch: {bad} replicas are invalid after the timed run")
    return durs[0], shape, [round(m, 3) for m in tune_ms]


def bench_ising_batch(rx, n=512, sweeps=10000, seed=1):
    """512 XS1024W replicas, L uniform over {16, 32, ..., 1024}, beta uniform in
    [0.3, 0.6], drawn with numpy default_rng(seed): one batched launch for
    `sweeps` sweeps (launch shape autotuned first on runs of 500 sweeps),
    then the same replicas from the same start one ising_sweep call each for
    the same `sweeps` (the per-launch form), both timed with HIP events on
    the stream they run on.  Every replica's status is checked after each
    form, so an invalid lattice fails the bench.  A second batch of 2048
    small replicas (L uniform over {16, ..., 128}, 2000 sweeps) is timed
    batched only."""
    import numpy as np
    rng = np.random.default_rng(seed)
    Ls = [int(x) for x in rng.choice(np.arange(16, 1025, 16), size=n)]
    betas = [float(b) for b in rng.uniform(0.3, 0.6, size=n)]
    lats = [rx.ising_create(L, "xs1024w", 1000 + i) for i, L in enumerate(Ls)]
    sites = sum(L * L for L in Ls)
    batched_ms, shape, tune_ms = run_tuned_batch(rx, lats, betas, [sweeps] * n, 500)
    for lat in lats:
        lat.destroy()
    small_n, small_sweeps = 2048, 2000
    sLs = [int(x) for x in rng.choice(np.arange(16, 129, 16), size=small_n)]
    sbetas = [float(b) for b in rng.uniform(0.3, 0.6, size=small_n)]
    slats = [rx.ising_create(L, "xs1024w", 5000 + i) for i, L in enumerate(sLs)]
    ssites = sum(L * L for L in sLs)
    small_ms, small_shape, small_tune = run_tuned_batch(rx, slats, sbetas, [small_sweeps] * small_n, 200)
    for lat in slats:
        lat.destroy()
    small = {"replicas": small_n, "sites": ssites, "sweeps": small_sweeps, "batched_ms": round(small_ms, 2),
             "batched_flips_per_ns": round(ssites * small_sweeps / (small_ms * 1e6), 2),
             "shape": rx.ising_batch_shapes()[small_shape], "tune_ms": small_tune}
    lats = [rx.ising_create(L, "xs1024w", 1000 + i) for i, L in enumerate(Ls)]

    def per_launch():
        for lat, b in zip(lats, betas):
            rx.ising_sweep(lat, b, sweeps)

    durs, _ = time_launches(per_launch, 1, 0)
    single_ms = durs[0]
    bad = sum(rx.ising_status(lat) for lat in lats)
    for lat in lats:
        lat.destroy()
    if bad:
        raise RuntimeError(f"Ising per-launch leg: {bad} lattices are invalid after the timed run")
    rate = sites * sweeps / (batched_ms * 1e6)
    per_site = ising_valu_per_site().get("batch_xs1024w")
    extra = {}
    if per_site:
        extra = {"valu_lane_instr_per_site": per_site,
                 "valu_frac": round(rate * 1e9 * per_site / VALU_PEAK_LANE_INSTR, 4)}
    return {"replicas": n, "sites": sites, "sweeps": sweeps, "batched_ms": round(batched_ms, 2),
            "batched_flips_per_ns": round(rate, 2), **extra,
            "shape": rx.ising_batch_shapes()[shape], "tune_ms": tune_ms,
            "per_launch_sweeps": sweeps, "per_launch_ms": round(single_ms, 2),
            "per_launch_flips_per_ns": round(sites * sweeps / (single_ms * 1e6), 2), "small": small}


def bench_ragged(rx, kind="xs1024w", n=10000, seed=1, baseline_requests=256):
    """10^4 requests with lengths log-uniform in [2^10, 2^22] (numpy
    default_rng(seed)); XS1024W requests are per instance.  One ragged call
    (3 timed after 1 warm-up, the plan's shape autotuned first) vs the plain
    form, one launch per request: a
    generator of one stream (XS1024W: one instance) per request, created
    before the timed region, fills its request at its offset.  The plain form
    is timed over `baseline_requests` requests drawn at random without
    replacement (numpy default_rng(seed + 1)); rates are values per second."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    lens = np.floor(2.0 ** (10 + 12 * rng.random(n))).astype(np.uint64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    S = 32 * n if kind == "xs1024w" else n
    g = rx.rng_create(kind, S, 1)
    plan = rx.rng_ragged_create(g, off)
    out = torch.empty(int(off[-1]) + 32, dtype=torch.int32, device="cuda")
    tune_ms = rx.rng_ragged_autotune(plan, out, reps=1)
    shape = rx.rng_ragged_shapes(kind)[rx.rng_ragged_get_shape(plan)]
    durs, _ = time_launches(lambda: rx.rng_fill_ragged_u32(plan, out), 3, 1)
    ms = sum(durs) / len(durs)
    total = int(off[-1])
    plan.destroy()
    g.destroy()
    width = 32 if kind == "xs1024w" else 1
    pick = np.sort(np.random.default_rng(seed + 1).choice(n, size=min(baseline_requests, n), replace=False))
    gens = [rx.rng_create(kind, width, 1 + int(u)) for u in pick]
    # a request's values start at its offset; XS1024W instances write whole
    # 32-value rows, so each view starts at a 16-byte aligned position
    views = []
    for u in pick:
        o = int(off[u]) // 4 * 4
        cnt = -(-int(lens[u]) // width)
        views.append((out[o:o + cnt * width], cnt))

    def per_request():
        for gu, (v, cnt) in zip(gens, views):
            rx.rng_fill_u32(gu, v, cnt)

    durs, _ = time_launches(per_request, 1, 0)
    sub = int(sum(int(lens[u]) for u in pick))
    for gu in gens:
        gu.destroy()
    return {"kind": kind, "requests": n, "values": total, "ms": round(ms, 3),
            "gsamples_s": round(total / ms / 1e6, 2), "gbs": round(total * 4 / ms / 1e6, 1),
            "hbm_frac": round(total * 4 / ms / 1e6 / HBM_PEAK_GBS, 4),
            "shape": shape, "tune_ms": [round(m, 3) for m in tune_ms],
            "per_launch_requests": len(pick), "per_launch_values": sub, "per_launch_ms": round(durs[0], 2),
            "per_launch_gsamples_s": round(sub / durs[0] / 1e6, 3)}


def bench_serve(rx, n_req=20000, rate=2000.0, clients=64, slots=8, inflight=32, seed=1, budget=64 << 30):
    """Poisson arrivals (numpy default_rng(seed)); 90% fills (kind uniform over
    every kind, count = floor(2^(10 + 18 u)), u32/f32 half each), 10% Ising jobs
    (L in {64, ..., 2048} powers of two, 100 sweeps, beta uniform in
    [0.3, 0.6], kind uniform).  Latency = submission to completion."""
    import threading
    import numpy as np
    rng = np.random.default_rng(seed)
    # kinds the server takes (not the sub-stream, per-stream-multiplier or lagged Fibonacci ones)
    kinds = [k for k in rx.KINDS if not k.endswith("_sub") and k != "mwc_diff" and not k.startswith("lfg")]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    reqs = []
    for i in range(n_req):
        c = int(rng.integers(clients))
        k = kinds[int(rng.integers(len(kinds)))]
        if rng.random() < 0.9:
            reqs.append(("fill", c, k, int(2 ** (10 + 18 * rng.random())), bool(rng.random() < 0.5)))
        else:
            reqs.append(("ising", c, k, int(2 ** rng.integers(6, 12)), float(rng.uniform(0.3, 0.6))))
    srv = rx.Server(slots=slots, max_inflight=inflight, memory_budget=budget, seed=seed)
    tickets = [None] * n_req
    ising_tickets = set()

    failed = []

    def submitter():
        t0 = time.perf_counter()
        try:
            for i, r in enumerate(reqs):
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                if r[0] == "fill":
                    tickets[i] = srv.submit_fill(r[1], r[2], r[3], r[4])
                else:
                    tickets[i] = srv.submit_ising(r[1], r[2], r[3], r[4], 100)
                    ising_tickets.add(tickets[i])
        except Exception as exc:  # reported by the consuming loop
            failed.append(exc)

    t0 = time.perf_counter()
    th = threading.Thread(target=submitter)
    th.start()
    lat, done = [], []
    # results are consumed in completion order, as independent clients would
    while len(done) < n_req:
        try:
            ticket, res = srv.wait_any(timeout_s=1.0)
        except rx.RngxError as exc:
            if failed:
                th.join()
                srv.destroy()
                raise RuntimeError(f"served trace: submission failed: {failed[0]}") from exc
            if exc.status == -7:  # RNGX_E_BUSY: nothing finished within the second
                continue
            raise
        lat.append(res.latency_s)
        done.append((ticket, res.n_values))
        srv.release(ticket)
    th.join()
    wall = time.perf_counter() - t0
    flips = sum(n * 100 for t, n in done if t in ising_tickets)
    samples = sum(n for t, n in done if t not in ising_tickets)
    srv.destroy()
    lat = np.array(lat)
    return {"requests": n_req, "rate_per_s": rate, "slots": slots, "max_inflight": inflight,
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "wall_s": round(wall, 2),
            "gsamples_s": round(samples / wall / 1e9, 3), "flips_per_ns": round(flips / wall / 1e9, 3)}


def traffic_from_profile():
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    only while the kernel sources are the ones it was taken from."""
    rec = profile_json(PROFILE_TRAFFIC)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def host_threads() -> int:
    """Host threads for the CPU oracle: every core this process may run on,
    capped at 16, the CPU share a one-GPU job gets on the GPU hosts."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(target_s: float = 10.0):
    """The CPU oracle (never tuned) on a bounded sample of the same workload:
    XS1024W u32 fill of all 2^20 streams, the first n outputs of each (n sized
    for about target_s seconds of wall time), streams split over the host
    threads, each thread producing its block 64 outputs per oracle call; the
    one-thread rate of the same call beside it.  Then the oracle's Ising
    sweep, which is serial: one independent lattice per host thread, at L = 64
    (2000 sweeps) and at L = 4096 (3 sweeps; the 10^4-sweep run is
    extrapolated from that rate)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    threads = host_threads()
    S = S_FULL
    st = oracle.seed("xs1024w", S, 1)
    probe = st.copy()
    oracle.generate("xs1024w", S, probe, 64, lo=0, hi=32 * 1024)  # warm-up
    t = time.perf_counter()
    oracle.generate("xs1024w", S, probe, 64, lo=0, hi=32 * 1024)
    rate1 = 32 * 1024 * 64 / (time.perf_counter() - t)  # values/s on one thread
    del probe
    n = max(64, int(rate1 * threads * target_s / S) // 64 * 64)
    chunk = S // threads

    def work(i):
        lo, hi = i * chunk, (i + 1) * chunk
        for _ in range(n // 64):
            oracle.generate("xs1024w", S, st, 64, lo=lo, hi=hi)

    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, range(threads)))
    dt = time.perf_counter() - t

    def ising_rate(L, sweeps):
        lats = [oracle.ising_create(L, "xs1024w", 1 + i) for i in range(threads)]

        def run(i):
            sp, stt = lats[i]
            oracle.ising_sweeps(L, "xs1024w", 0.4, stt, sp, sweeps, trace=True)

        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, range(threads)))
        w = time.perf_counter() - t0
        return {"L": L, "sweeps": sweeps, "lattices": threads, "wall_s": round(w, 2),
                "flips_per_ns": round(threads * L * L * sweeps / w / 1e9, 5)}

    ising = [ising_rate(64, 2000), ising_rate(4096, 3)]
    ising[1]["note"] = "rate at L=4096 from 3 sweeps; 10^4 sweeps extrapolated at that rate"
    ising[1]["extrapolated_1e4_sweeps_s"] = round(4096 * 4096 * 1e4 / (ising[1]["flips_per_ns"] * 1e9), 1)
    return {"value": round(S * n / dt / 1e9, 4), "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "sample": f"xs1024w u32 fill of {S} streams x first {n} outputs ({S * n} values, {dt:.1f} s wall, "
                      f"{threads} threads over stream blocks)",
            "single_thread_gsamples_s": round(rate1 / 1e9, 4), "host_cpus_visible": os.cpu_count(),
            "ising_xs1024w_beta0.4": ising}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--parts", default="all", help="all | none: per-kind parts and Ising")
    ap.add_argument("--ising-sweeps", type=int, default=10000)
    ap.add_argument("--kinds", default=None, help="comma-separated kinds for the parts (default: all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="time the headline kernel only (for profiling)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="for rocprofv3: the headline fill `steps` times, then a plain 4 GiB device-to-device "
                         "copy `steps` times as the reference for scaling HBM byte counters; prints no JSON")
    ap.add_argument("--profile-ising", action="store_true",
                    help="for rocprofv3: `steps` Ising calls of 200 sweeps each at L=4096, beta=0.4 "
                         "(energy trace on) of --profile-kind (default xs1024w); prints no JSON")
    ap.add_argument("--profile-fill", action="store_true",
                    help="for rocprofv3: the fill autotuner, then `steps` u32 fills of 2^20 x 4096 of "
                         "--profile-kind, then `steps` consume calls of the same size; prints no JSON")
    ap.add_argument("--profile-kind", default="xs1024w")
    ap.add_argument("--profile-batch", action="store_true",
                    help="for rocprofv3: `steps` runs of the 512-replica XS1024W batch (L in 16..1024, "
                         "numpy default_rng(1)) at 1000 sweeps each; prints no JSON")
    ap.add_argument("--profile-ragged", action="store_true",
                    help="for rocprofv3: `steps` ragged fills of the 10^4-request plan (lengths log-uniform in "
                         "[2^10, 2^22], numpy default_rng(1)) for XS1024W, then LCG32; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent streams shard by index range with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1204_6193_amd as rx
    rx.load()
    torch.cuda.set_device(0)
    if args.profile_fill:
        kind = args.profile_kind
        g = rx.rng_create(kind, S_FULL, 1)
        out = torch.empty(S_FULL * COUNT_FULL, dtype=torch.int32, device="cuda")
        rx.rng_autotune_fill(g, out, COUNT_FULL, reps=1)  # the configuration the bench times
        for _ in range(args.steps):
            rx.rng_fill_u32(g, out, COUNT_FULL)
        acc = torch.empty(S_FULL, dtype=torch.int32, device="cuda")
        for _ in range(args.steps):
            rx.rng_consume(g, acc, COUNT_FULL)
        torch.cuda.synchronize()
        g.destroy()
        print(f"profile pass done: {args.steps} fills and consumes of {S_FULL}x{COUNT_FULL}, {kind}", flush=True)
        return
    if args.profile_ising:
        lat = rx.ising_create(4096, args.profile_kind, 1)
        tr = torch.zeros(200, dtype=torch.int32, device="cuda")
        for _ in range(args.steps):
            rx.ising_sweep(lat, 0.4, 200, tr)
        torch.cuda.synchronize()
        if rx.ising_status(lat):
            raise RuntimeError("profile pass: the lattice is invalid")
        lat.destroy()
        del tr
        torch.cuda.synchronize()
        print(f"profile pass done: {args.steps} calls of 200 sweeps at L=4096, {args.profile_kind}", flush=True)
        return
    if args.profile_ragged:
        import numpy as np
        rng = np.random.default_rng(1)
        lens = np.floor(2.0 ** (10 + 12 * rng.random(10000))).astype(np.uint64)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
        out = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
        for kind in ("xs1024w", "lcg32"):
            g = rx.rng_create(kind, 32 * 10000 if kind == "xs1024w" else 10000, 1)
            plan = rx.rng_ragged_create(g, off)
            for _ in range(args.steps):
                rx.rng_fill_ragged_u32(plan, out)
            torch.cuda.synchronize()
            plan.destroy()
        print(f"profile pass done: {args.steps} ragged fills of {int(off[-1])} values, xs1024w and lcg32",
              flush=True)
        return
    if args.profile_batch:
        import numpy as np
        rng = np.random.default_rng(1)
        Ls = [int(x) for x in rng.choice(np.arange(16, 1025, 16), size=512)]
        betas = [float(b) for b in rng.uniform(0.3, 0.6, size=512)]
        lats = [rx.ising_create(L, "xs1024w", 1000 + i) for i, L in enumerate(Ls)]
        batch = rx.ising_batch_create(lats, betas, [1000] * 512)
        for _ in range(args.steps):
            rx.ising_batch_run(batch)
        torch.cuda.synchronize()
        if rx.ising_batch_status(batch):
            raise RuntimeError("profile pass: invalid replicas")
        batch.destroy()
        for lat in lats:
            lat.destroy()
        torch.cuda.synchronize()
        print(f"profile pass done: {args.steps} batch runs of 512 replicas x 1000 sweeps", flush=True)
        return
    out = torch.empty(S_FULL * COUNT_FULL, dtype=torch.int32, device="cuda")
    if args.profile_pass:
        g = rx.rng_create("xs1024w", S_FULL, 1)
        for _ in range(args.steps):
            rx.rng_fill_u32(g, out, COUNT_FULL)
        torch.cuda.synchronize()
        src = out[: 1 << 30]
        dst = torch.empty(1 << 30, dtype=torch.int32, device="cuda")
        for _ in range(args.steps):
            dst.copy_(src)  # reads 4 GiB, writes 4 GiB
        torch.cuda.synchronize()
        print(f"profile pass done: {args.steps} fills of {S_FULL}x{COUNT_FULL}, {args.steps} copies of 4 GiB",
              flush=True)
        return

    kinds = args.kinds.split(",") if args.kinds else KINDS
    ising_kinds = [k for k in kinds if k in ISING_KINDS]
    head = bench_fill(rx, "xs1024w", "u32", out, args.steps, args.warmup)
    print(f"# headline xs1024w u32 fill: {head}", file=sys.stderr, flush=True)
    parts = {}
    if not args.only_headline and args.parts == "all":
        parts["write_ceiling"] = bench_write_ceiling(out, max(5, args.steps // 2), 2)
        ceiling = parts["write_ceiling"]["gbs"]
        head["ceiling_frac"] = round(head["gbs"] / ceiling, 4)
        print(f"# write ceiling {parts['write_ceiling']}", file=sys.stderr, flush=True)
        for kind in kinds:
            rec = {}
            for mode in ("u32", "f32", "consume"):
                rec[mode] = bench_fill(rx, kind, mode, out, max(5, args.steps // 2), 2)
                if mode != "consume":
                    rec[mode]["ceiling_frac"] = round(rec[mode]["gbs"] / ceiling, 4)
            rec["skip_2p40_ms"] = bench_skip(rx, kind)
            parts[kind] = rec
            print(f"# {kind}: {rec}", file=sys.stderr, flush=True)
        del out
        torch.cuda.empty_cache()
        ising = {}
        for kind in ising_kinds:
            sweeps = args.ising_sweeps if kind == "xs1024w" else max(100, args.ising_sweeps // 10)
            ising[kind] = bench_ising(rx, kind, 4096, sweeps)
            print(f"# ising L=4096 {kind}: {ising[kind]}", file=sys.stderr, flush=True)
        parts["ising_L4096_beta0.4"] = ising
        beta_c = math.log(1 + math.sqrt(2)) / 2
        parts["ising_L4096_betac"] = {
            kind: bench_ising(rx, kind, 4096, args.ising_sweeps if kind == "xs1024w" else max(100, args.ising_sweeps // 10),
                              beta_c) for kind in ising_kinds}
        print(f"# ising L=4096 xs1024w beta_c: {parts['ising_L4096_betac']}", file=sys.stderr, flush=True)
        mh = {"k2": {k: bench_ising(rx, k, 4096, 200, hits=2) for k in ising_kinds},
              "k100": {k: bench_ising(rx, k, 4096, 10, hits=100) for k in ising_kinds}}
        parts["ising_L4096_multihit"] = mh
        print(f"# ising L=4096 multi-hit: " + json.dumps({h: {k: v["flips_per_ns"] for k, v in r.items()}
                                                         for h, r in mh.items()}), file=sys.stderr, flush=True)
        if not args.skip_batched:
            parts["ising_batch"] = bench_ising_batch(rx)
            print(f"# ising batch: {parts['ising_batch']}", file=sys.stderr, flush=True)
            parts["ragged"] = [bench_ragged(rx, k) for k in kinds if k in RAGGED_KINDS]
            print(f"# ragged: {parts['ragged']}", file=sys.stderr, flush=True)
        if not args.skip_serve:
            parts["serve"] = {"continuous": bench_serve(rx), "fifo_one_at_a_time": bench_serve(rx, slots=1, inflight=1)}
            print(f"# serve: {parts['serve']}", file=sys.stderr, flush=True)

    samples = S_FULL * COUNT_FULL
    alg_bytes = samples * 4 + 2 * STATE_BYTES["xs1024w"] * S_FULL
    achieved = alg_bytes / head["ms"] / 1e6
    line = {
        "metric": "RNG Gsamples/s (% HBM peak) per generator; Ising Metropolis flips/ns at L=4096",
        "value": head["gsamples_s"],
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "xs1024w bulk fill, uint32, interleaved out[k*S+s]", "n_streams": S_FULL,
                   "outputs_per_stream": COUNT_FULL, "seed": 1, "generator": "XORShift-1024 + Weyl (paper's)",
                   "fill_config": head.get("autotune", {}).get("config")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile()},
        "kernel_hash": kernel_hash(),
    }
    if parts:
        line["parts"] = parts
    if not args.no_cpu and not args.only_headline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
