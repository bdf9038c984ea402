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
            (9, "mwc", 4097, False), (9, "lcg32", 1, False)]
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
