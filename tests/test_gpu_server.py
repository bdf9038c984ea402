"""The served form: results equal the plain calls, and a client's results are
the same alone and in a mix of other clients' requests."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

SEED = 12345


def _unit(kind):
    return 32 if kind == "xs1024w" else 1


def _result_bytes(rx, srv, ticket, nbytes):
    r = srv.wait(ticket, 60.0)
    assert r.status == 0
    host = rx.copy_to_host(r.d_output, nbytes)
    srv.release(ticket)
    return host, r


def test_server_fills_equal_direct_fills(rngx, orc):
    """A served fill is the next `count` values of the client's stream: equal
    to filling stream 0 (instance 0) of rng_create(kind, 1 or 32, seed')."""
    srv = rngx.Server(slots=4, max_inflight=8, memory_budget=256 << 20, seed=SEED)
    reqs = [(3, "xs1024w", 1000, False), (3, "xs1024w", 300_001, True), (7, "lcg64", 9000, False),
            (3, "philox4x32_10", 77, False), (7, "lcg64", 300, True), (7, "xorwow", 20_000, False),
            (9, "mwc", 4097, False), (9, "lcg32", 1, False), (3, "philox4x32_10", 4099, False),
            (3, "philox4x32_7", 10, True), (3, "philox4x32_7", 70_001, False)]  # a client's later Philox requests
    tickets = [srv.submit_fill(c, k, n, f) for c, k, n, f in reqs]
    gens = {}
    for (c, k, n, f), t in zip(reqs, tickets):
        host, r = _result_bytes(rngx, srv, t, 4 * n)
        assert r.n_values == n
        if (c, k) not in gens:
            gens[(c, k)] = rngx.rng_create(k, _unit(k), orc.splitmix(SEED, 16 * c + rngx.KINDS[k]))
        steps = -(-n // _unit(k))
        out = torch.empty(steps * _unit(k), dtype=torch.float32 if f else torch.int32, device="cuda")
        (rngx.rng_fill_f32 if f else rngx.rng_fill_u32)(gens[(c, k)], out, steps)
        want = out.cpu().numpy().view(np.uint32)[:n]
        assert np.array_equal(host.view(np.uint32), want), (c, k, n, f)
    with pytest.raises(rngx.RngxError):  # sub-stream LCGs are parts of one S-stream sequence
        srv.submit_fill(1, "lcg32_sub", 10, False)
    srv.destroy()


def test_server_ising_job_matches_oracle(rngx, orc):
    srv = rngx.Server(slots=2, max_inflight=4, memory_budget=64 << 20, seed=SEED)
    for j, (L, kind) in enumerate([(64, "xs1024w"), (512, "lcg32")]):
        t = srv.submit_ising(5, kind, L, 0.42, 3)
        host, r = _result_bytes(rngx, srv, t, L * L + 16 + 12)
        seed = orc.splitmix(SEED, (1 << 62) + (5 << 24) + j)
        sp, st = orc.ising_create(L, kind, seed)
        tr = orc.ising_sweeps(L, kind, 0.42, st, sp, 3)
        assert np.array_equal(host[: L * L].view(np.int8), sp), (L, kind)
        off = -(-(L * L) // 16) * 16
        assert np.array_equal(host[off: off + 12].view(np.int32), tr), (L, kind)
    srv.destroy()


def _client_script(rng):
    script = []
    for i in range(12):
        if rng.random() < 0.25:
            script.append(("ising", ["xs1024w", "mwc"][i % 2], int(rng.choice([64, 128, 256, 512])), 4))
        else:
            script.append(("fill", ["xs1024w", "lcg32", "philox4x32_10", "xorwow"][i % 4],
                           int(2 ** rng.uniform(10, 16)), bool(i % 3 == 0)))
    return script


def _run(rx, scripts, slots, inflight):
    srv = rx.Server(slots=slots, max_inflight=inflight, memory_budget=512 << 20, seed=SEED)
    order = [(c, i) for i in range(max(len(s) for s in scripts.values())) for c in scripts if i < len(scripts[c])]
    tickets = {}
    for c, i in order:
        op = scripts[c][i]
        if op[0] == "fill":
            tickets[(c, i)] = (srv.submit_fill(c, op[1], op[2], op[3]), 4 * op[2])
        else:
            L = op[2]
            tickets[(c, i)] = (srv.submit_ising(c, op[1], L, 0.4, op[3]), L * L)
    out = {}
    for key, (t, nbytes) in tickets.items():
        out[key], _ = _result_bytes(rx, srv, t, nbytes)
    srv.destroy()
    return out


def test_server_alone_equals_in_the_mix(rngx):
    rng = np.random.default_rng(4)
    scripts = {c: _client_script(rng) for c in range(6)}
    mixed = _run(rngx, scripts, slots=4, inflight=16)
    alone = _run(rngx, {2: scripts[2]}, slots=1, inflight=1)
    for i in range(len(scripts[2])):
        assert np.array_equal(alone[(2, i)], mixed[(2, i)]), i


def test_server_admission(rngx):
    srv = rngx.Server(slots=2, max_inflight=4, memory_budget=8 << 20, seed=SEED)
    with pytest.raises(rngx.RngxError) as e:
        srv.submit_fill(0, "lcg32", 4 << 20)      # 16 MiB > the whole budget
    assert e.value.status == -3
    # three requests of 2.6 MB: beside the jump tables only one fits at a
    # time; each is admitted when the previous one is released
    ts = [srv.submit_fill(0, "lcg32", 650_000) for _ in range(3)]
    for t in ts:
        r = srv.wait(t, 30.0)
        assert r.status == 0
        srv.release(t)
    srv.destroy()


def test_server_wait_any_reports_each_request_once(rngx):
    srv = rngx.Server(slots=4, max_inflight=8, memory_budget=64 << 20, seed=SEED)
    ts = {srv.submit_fill(c, "lcg32", 5000) for c in range(10)} | {srv.submit_ising(1, "xs1024w", 64, 0.4, 2)}
    seen = set()
    for _ in range(len(ts)):
        t, r = srv.wait_any(30.0)
        assert r.status == 0 and t in ts and t not in seen
        seen.add(t)
        srv.release(t)
    with pytest.raises(rngx.RngxError) as e:
        srv.wait_any(0.01)
    assert e.value.status == -7
    srv.destroy()


def _oracle_client_values(orc, rngx, kind, client, start, n, seed=SEED):
    """Values start .. start+n-1 of the (client, kind) stream from the oracle:
    stream 0 (XS1024W: instance 0, warp order) of the client seed, reached by
    the oracle's jump-ahead."""
    width = _unit(kind)
    st = orc.seed(kind, width, orc.splitmix(seed, 16 * client + rngx.KINDS[kind]))
    first = start // width
    if first:
        orc.jump(kind, width, st, first)
    steps = -(-(start + n) // width) - first
    vals = orc.generate(kind, width, st, steps).ravel()
    return vals[start - first * width: start - first * width + n]


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "philox4x32_7"])
def test_served_fill_near_the_maximum_matches_the_oracle(rngx, orc, kind):
    """A served fill of 2^28 - 5 values (the largest size, every chunk
    jump of the stream fill), then a second one that continues the stream
    (XS1024W: from the next whole instance step):
    sampled ranges -- the start, the middle, the last chunk -- equal the
    oracle's stream of the client seed; the second request starts where the
    first ended; both as uint32, the second also as FP32."""
    client, n = 11, (1 << 28) - 5
    print(f"case served 2^28 {kind}", flush=True)
    srv = rngx.Server(slots=2, max_inflight=2, memory_budget=(1 << 30) + (64 << 20), seed=SEED)
    t = srv.submit_fill(client, kind, n, False)
    r = srv.wait(t, 120.0)
    assert r.status == 0 and r.n_values == n
    for lo in (0, n // 2 - 1000, n - 5000):
        got = rngx.copy_to_host(r.d_output + 4 * lo, 4 * 5000, "uint32")
        want = _oracle_client_values(orc, rngx, kind, client, lo, 5000)
        assert np.array_equal(got, want), (kind, lo)
    srv.release(t)
    t = srv.submit_fill(client, kind, 3001, True)
    r = srv.wait(t, 60.0)
    got = rngx.copy_to_host(r.d_output, 4 * 3001, "float32")
    # XS1024W requests take whole instance steps (the unused lanes of a last
    # partial step are dropped), so the next request starts at a step
    nxt = -(-n // _unit(kind)) * _unit(kind)
    want = _oracle_client_values(orc, rngx, kind, client, nxt, 3001)
    assert np.array_equal(got.view(np.uint32), ((want >> 8).astype(np.float32) * np.float32(2.0 ** -24)).view(np.uint32))
    srv.release(t)
    srv.destroy()


def test_server_cancel(rngx, orc):
    """A request that waits for memory can be withdrawn: its ticket is gone
    and its (client, kind) stream does not advance."""
    srv = rngx.Server(slots=1, max_inflight=4, memory_budget=24 << 20, seed=SEED)
    hold = srv.submit_fill(1, "lcg32", 4 << 20)  # 16 MiB, kept unreleased
    assert srv.wait(hold, 30.0).status == 0
    blocked = srv.submit_fill(2, "lcg64", 4 << 20)  # cannot fit beside it
    with pytest.raises(rngx.RngxError) as e:
        srv.wait(blocked, 0.2)
    assert e.value.status == -7
    srv.cancel(blocked)
    with pytest.raises(rngx.RngxError):
        srv.wait(blocked, 0.0)
    srv.release(hold)
    t = srv.submit_fill(2, "lcg64", 1000)
    r = srv.wait(t, 30.0)
    got = rngx.copy_to_host(r.d_output, 4000, "uint32")
    assert np.array_equal(got, _oracle_client_values(orc, rngx, "lcg64", 2, 0, 1000))
    srv.release(t)
    with pytest.raises(rngx.RngxError) as e:
        srv.cancel(t)  # released: unknown
    assert e.value.status == -1
    srv.destroy()


def test_server_kill_and_restore(rngx):
    """Client states exported from a server, which is then destroyed, and
    imported into a new server with another seed: the clients continue
    exactly as on a server that served all their requests."""
    reqs = [(3, "xs1024w", 7000), (3, "philox4x32_10", 4001), (8, "mwc", 999), (8, "xorwow", 5000)]
    ref = rngx.Server(slots=2, max_inflight=4, memory_budget=64 << 20, seed=SEED)
    a = rngx.Server(slots=2, max_inflight=4, memory_budget=64 << 20, seed=SEED)
    for srv in (ref, a):
        for c, k, n in reqs:
            t = srv.submit_fill(c, k, n)
            assert srv.wait(t, 30.0).status == 0
            srv.release(t)
    images = {(c, k): a.get_client_state(c, k) for c, k, _ in reqs}
    a.destroy()
    b = rngx.Server(slots=3, max_inflight=4, memory_budget=64 << 20, seed=SEED + 1)
    for (c, k), img in images.items():
        b.set_client_state(c, k, img)
    for c, k, n in reqs:
        outs = []
        for srv in (ref, b):
            t = srv.submit_fill(c, k, n + 13, True)
            r = srv.wait(t, 30.0)
            outs.append(rngx.copy_to_host(r.d_output, 4 * (n + 13)))
            srv.release(t)
        assert np.array_equal(outs[0], outs[1]), (c, k)
    with pytest.raises(rngx.RngxError) as e:
        b.set_client_state(3, "xs1024w", np.zeros(8, dtype=np.uint8))  # wrong size
    assert e.value.status == -6
    ref.destroy()
    b.destroy()


def test_server_small_requests_pass_a_blocked_one(rngx, orc):
    """A request that waits for memory does not hold back later small ones
    of other clients, but does hold back later ones of its own (client,
    kind), whose values must follow its own."""
    srv = rngx.Server(slots=4, max_inflight=8, memory_budget=40 << 20, seed=SEED)
    hold = srv.submit_fill(1, "lcg32", 6 << 20)  # 24 MiB, kept
    assert srv.wait(hold, 30.0).status == 0
    big = srv.submit_fill(2, "xorwow", 4 << 20)  # 16 MiB: does not fit yet
    same = srv.submit_fill(2, "xorwow", 1000)    # same pair: must wait behind it
    small = [srv.submit_fill(c, "lcg64", 2000) for c in (3, 4, 5)]
    for t in small:  # admitted while `big` waits
        assert srv.wait(t, 30.0).status == 0
        srv.release(t)
    with pytest.raises(rngx.RngxError):
        srv.wait(same, 0.2)
    srv.release(hold)
    rb = srv.wait(big, 30.0)
    rs = srv.wait(same, 30.0)
    got = rngx.copy_to_host(rs.d_output, 4000, "uint32")
    assert np.array_equal(got, _oracle_client_values(orc, rngx, "xorwow", 2, 4 << 20, 1000))
    srv.release(big)
    srv.release(same)
    srv.destroy()
