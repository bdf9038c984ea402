"""GPU <-> oracle parity of uneven per-stream requests (rng_fill_ragged_u32)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

KINDS = ["lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "xs1024w", "philox4x32_7", "lcg32_sub", "lcg64_sub",
         "mwc_diff"]


def _lengths(kind, n_units, seed):
    rng = np.random.default_rng(seed)
    lens = np.floor(2.0 ** rng.uniform(0, 14, size=n_units)).astype(np.int64)
    lens[0] = 0                                  # an empty request
    lens[1] = 1
    lens[-1] = 600_000 if kind == "xs1024w" else 200_000  # several chunks
    if kind == "xs1024w":
        lens[2] = 262_144 + 31                   # one full chunk and a partial step
    else:
        lens[2], lens[3] = 65_536, 128           # a whole wave chunk, whole 64-value steps
    return lens


def _oracle_ragged(orc, kind, S, st, lens):
    parts = []
    if kind == "xs1024w":
        for g, n in enumerate(lens):
            steps = (int(n) + 31) // 32
            vals = orc.generate(kind, S, st, steps, lo=32 * g, hi=32 * g + 32).ravel()
            parts.append(vals[: int(n)])
    else:
        for s, n in enumerate(lens):
            parts.append(orc.generate(kind, S, st, int(n), lo=s, hi=s + 1).ravel())
    return np.concatenate(parts)


@pytest.mark.parametrize("kind", KINDS)
def test_ragged_parity(rngx, orc, kind):
    print(f"case ragged {kind}", flush=True)
    S = 320 if kind == "xs1024w" else 37
    n_units = S // 32 if kind == "xs1024w" else S
    lens = _lengths(kind, n_units, 3)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    g = rngx.rng_create(kind, S, 11)
    plan = rngx.rng_ragged_create(g, off)
    st = orc.seed(kind, S, 11)
    for rep in range(2):
        out = torch.full((int(off[-1]) + 8,), -1, dtype=torch.int32, device="cuda")
        rngx.rng_fill_ragged_u32(plan, out)
        got = out.cpu().numpy().view(np.uint32)
        want = _oracle_ragged(orc, kind, S, st, lens)
        assert np.array_equal(got[: int(off[-1])], want), (kind, rep)
        assert np.all(got[int(off[-1]):] == 0xFFFFFFFF)      # nothing written past the end
        assert np.array_equal(rngx.rng_get_state(g), st), (kind, rep)
    # a uniform fill continues from where the ragged requests left the streams
    u = torch.empty(S * 5, dtype=torch.int32, device="cuda")
    rngx.rng_fill_u32(g, u, 5)
    assert np.array_equal(u.cpu().numpy().view(np.uint32).reshape(5, S), orc.generate(kind, S, st, 5))


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "lcg64_sub", "mwc", "mwc_diff", "xorwow", "philox4x32_10"])
def test_ragged_every_shape_matches_oracle(rngx, orc, kind):
    """Every ragged shape (XS1024W: 128, 64, 32 generating rows per CU; the
    others: other chunk lengths, hence other jumps and cuts) writes the
    oracle's values and leaves the oracle's states; the fills follow each
    other from the same plan, the oracle advanced in step."""
    S = 320 if kind == "xs1024w" else 37
    n_units = S // 32 if kind == "xs1024w" else S
    lens = _lengths(kind, n_units, 5)
    lens[-2] = 900_000 if kind == "xs1024w" else 300_000  # more chunks at every chunk length
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    g = rngx.rng_create(kind, S, 13)
    plan = rngx.rng_ragged_create(g, off)
    st = orc.seed(kind, S, 13)
    for shape in range(len(rngx.rng_ragged_shapes(kind))):
        print(f"case ragged shape {kind} {shape}", flush=True)
        rngx.rng_ragged_set_shape(plan, shape)
        assert rngx.rng_ragged_get_shape(plan) == shape
        out = torch.full((int(off[-1]) + 8,), -1, dtype=torch.int32, device="cuda")
        rngx.rng_fill_ragged_u32(plan, out)
        got = out.cpu().numpy().view(np.uint32)
        want = _oracle_ragged(orc, kind, S, st, lens)
        assert np.array_equal(got[: int(off[-1])], want), (kind, shape)
        assert np.all(got[int(off[-1]):] == 0xFFFFFFFF), (kind, shape)
        assert np.array_equal(rngx.rng_get_state(g), st), (kind, shape)


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "xorwow"])
def test_ragged_autotune_restores_streams(rngx, orc, kind):
    """The ragged autotuner times every shape, keeps the fastest and leaves
    the streams as they were: the next fill equals the oracle's first."""
    S = 320 if kind == "xs1024w" else 37
    n_units = S // 32 if kind == "xs1024w" else S
    lens = _lengths(kind, n_units, 6)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    g = rngx.rng_create(kind, S, 17)
    plan = rngx.rng_ragged_create(g, off)
    st = orc.seed(kind, S, 17)
    out = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
    ms = rngx.rng_ragged_autotune(plan, out, reps=1)
    print(f"case ragged autotune {kind} ms={ms}", flush=True)
    assert len(ms) == len(rngx.rng_ragged_shapes(kind)) and all(m > 0 for m in ms)
    assert ms[rngx.rng_ragged_get_shape(plan)] == min(ms)
    assert np.array_equal(rngx.rng_get_state(g), st)
    rngx.rng_fill_ragged_u32(plan, out)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), _oracle_ragged(orc, kind, S, st, lens))
    assert np.array_equal(rngx.rng_get_state(g), st)


@pytest.mark.parametrize("kind,shape", [("xs1024w", 0), ("lcg32", 0), ("lcg32", 1), ("xorwow", 1)])
def test_ragged_graph_replay(rngx, orc, kind, shape):
    """A ragged fill captured in a HIP graph (plan at `shape`): every replay
    equals an eager fill from a plan left at the default shape."""
    print(f"case ragged graph {kind} shape {shape}", flush=True)
    S = 256 if kind == "xs1024w" else 37
    lens = _lengths(kind, S // 32 if kind == "xs1024w" else S, 8)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    ga, gb = rngx.rng_create(kind, S, 2), rngx.rng_create(kind, S, 2)
    pa, pb = rngx.rng_ragged_create(ga, off), rngx.rng_ragged_create(gb, off)
    rngx.rng_ragged_set_shape(pa, shape)
    oa = torch.zeros(int(off[-1]), dtype=torch.int32, device="cuda")
    ob = torch.zeros(int(off[-1]), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        rngx.rng_fill_ragged_u32(pa, oa, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        rngx.rng_fill_ragged_u32(pb, ob)
        torch.cuda.synchronize()
        assert torch.equal(oa, ob), rep
        assert np.array_equal(rngx.rng_get_state(ga), rngx.rng_get_state(gb)), rep


@pytest.mark.parametrize("kind", ["lcg32", "lcg64", "xs1024w", "mwc", "mwc_diff", "philox4x32_10", "philox4x32_7"])
def test_ragged_into_unaligned_view(rngx, orc, kind):
    """The output starts one word past a 16-byte boundary (a view of a larger
    buffer): values match the oracle and the words around it stay untouched."""
    print(f"case ragged unaligned {kind}", flush=True)
    S = 96 if kind == "xs1024w" else 37
    lens = _lengths(kind, S // 32 if kind == "xs1024w" else S, 12)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    total = int(off[-1])
    g = rngx.rng_create(kind, S, 4)
    plan = rngx.rng_ragged_create(g, off)
    buf = torch.full((total + 2,), -1, dtype=torch.int32, device="cuda")
    rngx.rng_fill_ragged_u32(plan, buf[1:])
    got = buf.cpu().numpy().view(np.uint32)
    st = orc.seed(kind, S, 4)
    assert np.array_equal(got[1:total + 1], _oracle_ragged(orc, kind, S, st, lens)), kind
    assert got[0] == 0xFFFFFFFF and got[total + 1] == 0xFFFFFFFF
    assert np.array_equal(rngx.rng_get_state(g), st), kind


def test_ragged_argument_errors(rngx):
    g = rngx.rng_create("lcg32", 8, 1)
    with pytest.raises(rngx.RngxError):
        rngx.rng_ragged_create(g, [0, 1, 2])            # wrong count
    with pytest.raises(rngx.RngxError):
        rngx.rng_ragged_create(g, [0, 5, 3, 6, 7, 8, 9, 10, 11])  # decreasing
    p = rngx.rng_ragged_create(g, list(range(0, 18, 2)))
    assert rngx.load().rng_destroy(g.handle) == -7     # held by the plan
    p.destroy()


def _runs(seed, target):
    """Requests in runs of equal length (the oracle's jump-ahead then covers a
    whole run in one call): run lengths log-uniform in [2^10, 2^22], 1..120
    requests per run, about `target` values in all; one run of empty
    requests and one of single values."""
    rng = np.random.default_rng(seed)
    runs, total = [(3, 0), (2, 1)], 0
    while total < target:
        ln, m = int(2.0 ** (10 + 12 * rng.random())), int(rng.integers(1, 121))
        runs.append((m, ln))
        total += m * ln
    order = rng.permutation(len(runs))
    return [runs[i] for i in order]


@pytest.mark.parametrize("kind,shape", [("xs1024w", 0), ("xs1024w", 1), ("xs1024w", 2), ("lcg32", 0), ("lcg32", 1),
                                        ("lcg32", 2), ("mwc", 0), ("mwc", 2), ("philox4x32_10", 0), ("mwc_diff", 0)])
def test_ragged_bench_shape_sampled(rngx, orc, kind, shape):
    """About 2.2e9 values in requests of 2^10 .. 2^22 values: large enough
    that the XS1024W plan uses every shape's full row count (128, 64 or 32
    per CU), with cuts inside many instances.  Sampled requests are compared
    with the oracle value by value, every stream's final state with the
    oracle's jump-ahead, and one word past the end stays untouched."""
    print(f"case ragged bench shape {kind} shape {shape}", flush=True)
    runs = _runs(5, 2.2e9)
    lens = np.concatenate([np.full(m, ln, dtype=np.int64) for m, ln in runs])
    n = len(lens)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    total = int(off[-1])
    width = 32 if kind == "xs1024w" else 1
    S = width * n
    g = rngx.rng_create(kind, S, 21)
    plan = rngx.rng_ragged_create(g, off)
    rngx.rng_ragged_set_shape(plan, shape)
    out = torch.empty(total + 1, dtype=torch.int32, device="cuda")
    out[total] = -1
    rngx.rng_fill_ragged_u32(plan, out)
    torch.cuda.synchronize()
    st0 = orc.seed(kind, S, 21)
    rng = np.random.default_rng(6)
    sample = sorted({0, int(np.argmax(lens)), int(np.argmin(lens)), n - 1,
                     *(int(u) for u in rng.choice(n, size=10, replace=False))})
    for u in sample:
        ln = int(lens[u])
        st = st0.copy()
        steps = (ln + 31) // 32 if kind == "xs1024w" else ln
        want = orc.generate(kind, S, st, steps, lo=width * u, hi=width * u + width).ravel()[:ln]
        got = out[int(off[u]): int(off[u]) + ln].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), (kind, u, ln)
    assert int(out[total].item()) == -1
    st, u = st0.copy(), 0
    for m, ln in runs:
        steps = (ln + 31) // 32 if kind == "xs1024w" else ln
        if steps:
            orc.jump(kind, S, st, steps, lo=width * u, hi=width * (u + m))
        u += m
    assert np.array_equal(rngx.rng_get_state(g), st), kind
    del out
    torch.cuda.empty_cache()
