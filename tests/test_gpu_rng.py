"""GPU <-> oracle parity of the generator calls, element by element, bit-exact.

Sizes span several tiles and ragged tails at small scale; the full-size case
(2^20 streams x 4096 outputs, the bulk-fill workload) compares sampled
stream ranges against the oracle and checks properties of the whole output.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

KINDS = ["lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "xs1024w", "philox4x32_7", "lcg32_sub", "lcg64_sub",
         "mwc_diff"]


def _sizes(kind):
    # XS1024W: whole instances (1 instance, 3 = less than a block, 33 = a
    # block plus one); small kinds: ragged S (scalar path) and S % 4 == 0.
    return [32, 96, 1056] if kind == "xs1024w" else [1, 7, 1000, 4096, 5003]


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _fill(rx, g, count, f32=False):
    out = torch.empty(g.n_streams * count + 4, dtype=torch.float32 if f32 else torch.int32, device="cuda")
    (rx.rng_fill_f32 if f32 else rx.rng_fill_u32)(g, out, count)
    host = out[: g.n_streams * count].cpu().numpy()
    return host.reshape(count, g.n_streams) if f32 else host.view(np.uint32).reshape(count, g.n_streams)


@pytest.mark.parametrize("kind", KINDS)
def test_seed_image_matches_oracle(rngx, orc, kind):
    for S in _sizes(kind):
        g = rngx.rng_create(kind, S, 0xC0FFEE)
        assert np.array_equal(rngx.rng_get_state(g), orc.seed(kind, S, 0xC0FFEE)), (kind, S)


@pytest.mark.parametrize("kind", KINDS)
def test_fill_u32_parity_and_continuation(rngx, orc, kind):
    for S in _sizes(kind):
        print(f"case fill_u32 {kind} S={S}", flush=True)
        g = rngx.rng_create(kind, S, 1)
        st = orc.seed(kind, S, 1)
        for count in (37, 1, 29):  # odd counts: Philox resumes mid-block
            got = _fill(rngx, g, count)
            want = orc.generate(kind, S, st, count)
            assert np.array_equal(got, want), (kind, S, count)
        assert np.array_equal(rngx.rng_get_state(g), st)


@pytest.mark.parametrize("kind", KINDS)
def test_fill_f32_parity(rngx, orc, kind):
    S = 96 if kind == "xs1024w" else 1000
    g = rngx.rng_create(kind, S, 5)
    st = orc.seed(kind, S, 5)
    got = _fill(rngx, g, 19, f32=True)
    want = orc.generate(kind, S, st, 19, mode=orc.OUT_F32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert np.array_equal(rngx.rng_get_state(g), st)


@pytest.mark.parametrize("kind", KINDS)
def test_consume_parity(rngx, orc, kind):
    for S in _sizes(kind):
        g = rngx.rng_create(kind, S, 9)
        st = orc.seed(kind, S, 9)
        out = torch.zeros(S, dtype=torch.int32, device="cuda")
        rngx.rng_consume(g, out, 301)
        want = orc.generate(kind, S, st, 301, mode=orc.OUT_XOR)
        assert np.array_equal(_u32(out), want), (kind, S)
        assert np.array_equal(rngx.rng_get_state(g), st)


@pytest.mark.parametrize("kind", KINDS)
def test_skip_parity(rngx, orc, kind):
    S = 64 if kind == "xs1024w" else 100
    g = rngx.rng_create(kind, S, 3)
    st = orc.seed(kind, S, 3)
    for n in (1, 2, 5, 1000, 4097, (1 << 40) + 7, (1 << 64) - 1):
        print(f"case skip {kind} n={n}", flush=True)
        rngx.rng_skip(g, n)
        orc.jump(kind, S, st, n)
        assert np.array_equal(rngx.rng_get_state(g), st), (kind, n)
        assert np.array_equal(_fill(rngx, g, 3), orc.generate(kind, S, st, 3)), (kind, n)


@pytest.mark.parametrize("kind", KINDS)
def test_set_state_roundtrip(rngx, orc, kind):
    S = 64 if kind == "xs1024w" else 64
    g = rngx.rng_create(kind, S, 1)
    st = orc.seed(kind, S, 77)  # a different seed's image
    orc.generate(kind, S, st, 11)
    rngx.rng_set_state(g, st)
    assert np.array_equal(rngx.rng_get_state(g), st)
    assert np.array_equal(_fill(rngx, g, 13), orc.generate(kind, S, st, 13))


def test_set_state_rejects_fixed_points(rngx, orc):
    g = rngx.rng_create("xs1024w", 64, 1)
    img = rngx.rng_get_state(g)
    bad = img.copy()
    bad[128:256] = 0  # instance 1 all-zero
    with pytest.raises(rngx.RngxError) as e:
        rngx.rng_set_state(g, bad)
    assert e.value.status == -6
    assert np.array_equal(rngx.rng_get_state(g), img)  # unchanged
    m = rngx.rng_create("mwc", 4, 1)
    mi = rngx.rng_get_state(m)
    mb = mi.copy()
    mb[8:16] = 0
    with pytest.raises(rngx.RngxError):
        rngx.rng_set_state(m, mb)
    with pytest.raises(rngx.RngxError):
        rngx.rng_set_state(m, mi[:-1])


def test_mwc_diff_image_checks(rngx, orc):
    """MWC_DIFF refuses an image whose multipliers are not the handle's, or
    with a stream at a fixed point, and more than 2^21 streams."""
    S = 16
    g = rngx.rng_create("mwc_diff", S, 1)
    img = rngx.rng_get_state(g)
    other = img.copy()
    other[8 * S: 8 * S + 4] = np.array([4294966893], dtype=np.uint32).view(np.uint8)  # stream 0 takes a_1
    fixed = img.copy()
    fixed[8:16] = 0  # stream 1: y = 0
    for bad in (other, fixed):
        with pytest.raises(rngx.RngxError) as e:
            rngx.rng_set_state(g, bad)
        assert e.value.status == -6
    assert np.array_equal(rngx.rng_get_state(g), img)
    with pytest.raises(rngx.RngxError) as e:
        rngx.rng_create("mwc_diff", (1 << 21) + 1, 1)
    assert e.value.status == -5


def test_mwc_diff_multipliers_at_the_maximum(rngx, orc):
    """The device search at the largest stream count, 2^21: the image's
    multipliers equal the oracle's list (its first 8192 by the oracle's own
    sequential search, all 2^21 and the 2^20 prefix by the digests of the
    oracle's list in tests/golden); the streams seed from them as the
    oracle does."""
    import hashlib
    import json
    import os
    S = 1 << 21
    print("case mwc_diff multipliers 2^21", flush=True)
    g = rngx.rng_create("mwc_diff", S, 1)
    img = rngx.rng_get_state(g)
    a = img[8 * S:].view(np.uint32)
    with open(os.path.join(os.path.dirname(__file__), "golden", "mwc_diff_multipliers.json")) as f:
        gold = json.load(f)
    for n in (1 << 20, 1 << 21):
        assert hashlib.sha256(a[:n].astype("<u4").tobytes()).hexdigest() == gold[str(n)]["sha256"], n
        assert int(a[n - 1]) == gold[str(n)]["last"]
    assert np.array_equal(a[:8192], orc.mwc_multipliers(8192))
    y = img[: 8 * S].view(np.uint64)
    assert np.array_equal(img[: 8 * 4096], orc.seed("mwc_diff", 4096, 1)[: 8 * 4096])
    # the last streams follow the seeding rule with their (digest-checked) multipliers
    for s in range(S - 64, S):
        z = orc.splitmix(1, 1 + s)
        x, c = z & 0xFFFFFFFF, (z >> 32) % (int(a[s]) - 1)
        assert int(y[s]) == (c << 32) | (x if (x or c) else 1), s
    del img, a, y


def test_count_zero_and_argument_errors(rngx):
    g = rngx.rng_create("lcg32", 64, 1)
    img = rngx.rng_get_state(g)
    out = torch.zeros(64 * 4 + 8, dtype=torch.int32, device="cuda")
    rngx.rng_fill_u32(g, out, 0)
    assert np.array_equal(rngx.rng_get_state(g), img)
    with pytest.raises(rngx.RngxError) as e:  # 4-byte but not 16-byte aligned
        rngx.rng_fill_u32(g, out.data_ptr() + 4, 1)
    assert e.value.status == -2
    with pytest.raises(rngx.RngxError) as e:
        rngx.rng_fill_u32(g, out.data_ptr(), 1 << 62)
    assert e.value.status == -5
    assert np.array_equal(rngx.rng_get_state(g), img)


def test_results_do_not_depend_on_the_stream(rngx):
    s1 = torch.cuda.Stream()
    outs = []
    for stream in (None, s1):
        g = rngx.rng_create("xs1024w", 4096, 2)
        out = torch.empty(4096 * 64, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(s1 if stream is not None else torch.cuda.current_stream()):
            rngx.rng_fill_u32(g, out, 64, stream=stream)
        torch.cuda.synchronize()
        outs.append(out.cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32"])
def test_paced_fill_graph_replays(rngx, kind):
    """A paced fill (counters cleared by a kernel, not a memset) captured in a
    HIP graph: every replay equals the same fill run eagerly on a twin
    handle, with eager work in between."""
    S, count = 1 << 19, 40
    print(f"case graph paced fill {kind}", flush=True)
    ga, gb = rngx.rng_create(kind, S, 6), rngx.rng_create(kind, S, 6)
    oa = torch.empty(S * count, dtype=torch.int32, device="cuda")
    ob = torch.empty(S * count, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        rngx.rng_fill_u32(ga, oa, count, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        rngx.rng_fill_u32(gb, ob, count)
        torch.cuda.synchronize()
        assert torch.equal(oa, ob), (kind, rep)
        assert np.array_equal(rngx.rng_get_state(ga), rngx.rng_get_state(gb)), (kind, rep)
    del oa, ob
    torch.cuda.empty_cache()


def test_xs1024w_config_4096_streams_x_1024(rngx, orc):
    """The paper's generator: 4096 streams seeded from master seed 1, 1024
    outputs each (4,194,304 values), the whole array bit-exact."""
    S, count = 4096, 1024
    g = rngx.rng_create("xs1024w", S, 1)
    got = _fill(rngx, g, count)
    want = orc.generate("xs1024w", S, orc.seed("xs1024w", S, 1), count)
    assert np.array_equal(got, want)


def _xor_fold(x):
    while x.shape[0] > 1:
        h = x.shape[0] // 2
        x = torch.bitwise_xor(x[:h], x[h:2 * h]) if x.shape[0] % 2 == 0 else torch.cat(
            [torch.bitwise_xor(x[:h], x[h:2 * h]), x[2 * h:]])
    return x[0]


def test_xs1024w_paced_fill_ragged_rows(rngx, orc):
    """A fill large enough to be paced (2^18 streams: 128 workgroups of 2048
    streams) with a row count that is not a multiple of the 8-row band, twice
    in a row (the pacing counters are reused), then once as FP32: sampled
    stream ranges equal the oracle and the whole output's XOR equals the
    consume variant on a second handle."""
    S, count = 1 << 18, 1003
    print("case paced fill xs1024w", flush=True)
    g = rngx.rng_create("xs1024w", S, 5)
    g2 = rngx.rng_create("xs1024w", S, 5)
    st = orc.seed("xs1024w", S, 5)
    ranges = ((0, 256), (S // 2 - 128, S // 2 + 128), (S - 256, S))
    acc = torch.empty(S, dtype=torch.int32, device="cuda")
    for rep in range(3):
        f32 = rep == 2
        out = torch.empty(S * count, dtype=torch.float32 if f32 else torch.int32, device="cuda")
        (rngx.rng_fill_f32 if f32 else rngx.rng_fill_u32)(g, out, count)
        view = out.view(count, S)
        for lo, hi in ranges:
            want = orc.generate("xs1024w", S, st, count, lo=lo, hi=hi, mode=orc.OUT_F32 if f32 else orc.OUT_U32)
            got = view[:, lo:hi].contiguous().cpu().numpy()
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (rep, lo, hi)
        rngx.rng_consume(g2, acc, count)
        if not f32:
            assert torch.equal(acc, _xor_fold(view)), rep
        del out, view
    assert np.array_equal(rngx.rng_get_state(g), rngx.rng_get_state(g2))
    torch.cuda.empty_cache()


def _sampled_fill_check(rngx, orc, kind, S, count, seed, index):
    """Fill of a fresh handle with configuration `index`: sampled stream
    ranges equal the oracle, the whole output's XOR equals rng_consume on a
    twin handle, and both end in the same state."""
    g = rngx.rng_create(kind, S, seed)
    twin = rngx.rng_create(kind, S, seed)
    if index is not None:
        rngx.rng_set_fill_config(g, index)
        assert rngx.rng_get_fill_config(g) == index
    st = orc.seed(kind, S, seed)
    out = torch.empty(S * count, dtype=torch.int32, device="cuda")
    rngx.rng_fill_u32(g, out, count)
    view = out.view(count, S)
    for lo, hi in ((0, 256), (S // 2 - 128, S // 2 + 128), (S - 256, S)):
        want = orc.generate(kind, S, st, count, lo=lo, hi=hi)
        assert np.array_equal(view[:, lo:hi].contiguous().cpu().numpy().view(np.uint32), want), (kind, index, lo)
    acc = torch.empty(S, dtype=torch.int32, device="cuda")
    rngx.rng_consume(twin, acc, count)
    assert torch.equal(acc, _xor_fold(view)), (kind, index)
    assert np.array_equal(rngx.rng_get_state(g), rngx.rng_get_state(twin)), (kind, index)
    return g


def _sampled_f32_check(rngx, orc, kind, S, count, seed, index):
    """As _sampled_fill_check for FP32 output: sampled stream ranges equal the
    oracle's (u >> 8) * 2^-24 bit for bit; the state equals a twin's after a
    u32 fill of the same count."""
    g = rngx.rng_create(kind, S, seed)
    twin = rngx.rng_create(kind, S, seed)
    rngx.rng_set_fill_config(g, index)
    st = orc.seed(kind, S, seed)
    out = torch.empty(S * count, dtype=torch.float32, device="cuda")
    rngx.rng_fill_f32(g, out, count)
    view = out.view(count, S)
    for lo, hi in ((0, 256), (S // 2 - 128, S // 2 + 128), (S - 256, S)):
        want = orc.generate(kind, S, st, count, lo=lo, hi=hi, mode=orc.OUT_F32)
        got = view[:, lo:hi].contiguous().cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (kind, index, lo)
    acc = torch.empty(S, dtype=torch.int32, device="cuda")
    rngx.rng_consume(twin, acc, count)
    assert np.array_equal(rngx.rng_get_state(g), rngx.rng_get_state(twin)), (kind, index)


@pytest.mark.parametrize("kind", KINDS)
def test_every_fill_configuration(rngx, orc, kind):
    """Each autotuner candidate at 2^19 streams x 37 (large enough that the
    paced candidates run paced) gives the same numbers, as uint32 and as
    FP32."""
    S, count = 1 << 19, 37
    for index in range(len(rngx.rng_fill_configs(kind))):
        print(f"case fill config {kind} #{index}", flush=True)
        _sampled_fill_check(rngx, orc, kind, S, count, 3, index)
        _sampled_f32_check(rngx, orc, kind, S, count, 4, index)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["philox4x32_10", "philox4x32_7"])
def test_philox_fills_off_block_boundaries(rngx, orc, kind):
    """Philox streams at positions that are not multiples of 4 (one block of
    the counter-based generator): the first half of the streams at block
    boundaries, the second half each at its own offset, so that paced
    workgroups run both the aligned and the unaligned band loop and
    unpaced threads both of their paths.  Every fill configuration, u32 and
    FP32, equals the oracle over the whole output and leaves the oracle's
    state; so does consume."""
    S, count, seed = 1 << 19, 37, 5
    img = orc.seed(kind, S, seed)
    pos = img[8 * S:16 * S].view(np.uint64)
    pos[S // 2:] += np.random.default_rng(11).integers(1, 8, size=S // 2, dtype=np.uint64)
    st = img.copy()
    want = orc.generate(kind, S, st, count)
    want_f = orc.generate(kind, S, img.copy(), count, mode=orc.OUT_F32)
    for index in range(len(rngx.rng_fill_configs(kind))):
        print(f"case philox off-boundary fill {kind} #{index}", flush=True)
        for f32 in (False, True):
            g = rngx.rng_create(kind, S, seed)
            rngx.rng_set_state(g, img)
            rngx.rng_set_fill_config(g, index)
            if f32:
                out = torch.empty(S * count, dtype=torch.float32, device="cuda")
                rngx.rng_fill_f32(g, out, count)
                got = out.view(count, S).cpu().numpy().view(np.uint32)
                assert np.array_equal(got, want_f.view(np.uint32)), (kind, index, "f32")
            else:
                out = torch.empty(S * count, dtype=torch.int32, device="cuda")
                rngx.rng_fill_u32(g, out, count)
                got = out.view(count, S).cpu().numpy().view(np.uint32)
                assert np.array_equal(got, want), (kind, index, "u32")
            assert np.array_equal(rngx.rng_get_state(g), st), (kind, index, f32)
            rngx.rng_destroy(g)
    g = rngx.rng_create(kind, S, seed)
    rngx.rng_set_state(g, img)
    acc = torch.empty(S, dtype=torch.int32, device="cuda")
    rngx.rng_consume(g, acc, count)
    assert np.array_equal(acc.cpu().numpy().view(np.uint32), np.bitwise_xor.reduce(want, axis=0))
    assert np.array_equal(rngx.rng_get_state(g), st)
    rngx.rng_destroy(g)
    torch.cuda.empty_cache()


def test_xs1024w_fill_from_unit_vector_states(rngx, orc):
    """1024 instances, instance g holding the single set bit g of the
    1024-bit word (the sparsest states; every word shift of the DPP step
    reads zeros from outside the row for most lanes): a fill of 200 steps
    equals the oracle stepping the same image, element by element."""
    G = 1024
    S = 32 * G
    g = rngx.rng_create("xs1024w", S, 1)
    img = rngx.rng_get_state(g)
    W = img[: 4 * S].view(np.uint32)
    W[:] = 0
    for inst in range(G):
        W[32 * inst + 31 - inst // 32] = np.uint32(1) << np.uint32(inst % 32)  # word 0 most significant
    rngx.rng_set_state(g, img)
    st = img.copy()
    got = _fill(rngx, g, 200)
    assert np.array_equal(got, orc.generate("xs1024w", S, st, 200))
    assert np.array_equal(rngx.rng_get_state(g), st)


@pytest.mark.parametrize("kind", ["xs1024w", "lcg32", "xorwow"])
def test_autotune_fill(rngx, orc, kind):
    """The autotuner times every candidate, keeps the fastest and leaves the
    stream state as it was; fills after it stay exact."""
    S, count = 1 << 19, 64
    print(f"case autotune {kind}", flush=True)
    g = rngx.rng_create(kind, S, 9)
    before = rngx.rng_get_state(g)
    out = torch.empty(S * count, dtype=torch.int32, device="cuda")
    ms = rngx.rng_autotune_fill(g, out, count, reps=2)
    assert len(ms) == len(rngx.rng_fill_configs(kind)) and all(m > 0 for m in ms)
    assert rngx.rng_get_fill_config(g) == int(np.argmin(ms))
    assert np.array_equal(rngx.rng_get_state(g), before)
    st = orc.seed(kind, S, 9)
    rngx.rng_fill_u32(g, out, count)
    view = out.view(count, S)
    want = orc.generate(kind, S, st, count, lo=S - 256, hi=S)
    assert np.array_equal(view[:, S - 256:].contiguous().cpu().numpy().view(np.uint32), want)
    with pytest.raises(rngx.RngxError):
        rngx.rng_set_fill_config(g, 99)
    del out, view
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", KINDS)
def test_full_size_sampled_parity(rngx, orc, kind):
    """2^20 streams x 4096 outputs (16 GiB) as the benchmark launches it:
    sampled stream ranges equal the oracle; the consume variant on a second
    handle equals the XOR of the full output; a skip of 4096 on a third
    handle lands on the first handle's state."""
    S, count = 1 << 20, 4096
    print(f"case full-size {kind}", flush=True)
    g = rngx.rng_create(kind, S, 1)
    out = torch.empty(S * count, dtype=torch.int32, device="cuda")
    rngx.rng_fill_u32(g, out, count)
    view = out.view(count, S)
    st = orc.seed(kind, S, 1)
    for lo, hi in ((0, 512), (S // 2 - 256, S // 2 + 256), (S - 512, S)):
        want = orc.generate(kind, S, st, count, lo=lo, hi=hi)
        got = view[:, lo:hi].contiguous().cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), (kind, lo, hi)
    xor_all = _xor_fold(view)
    del out, view
    g2 = rngx.rng_create(kind, S, 1)
    acc = torch.empty(S, dtype=torch.int32, device="cuda")
    rngx.rng_consume(g2, acc, count)
    assert torch.equal(acc, xor_all)
    g3 = rngx.rng_create(kind, S, 1)
    rngx.rng_skip(g3, count)
    assert np.array_equal(rngx.rng_get_state(g3), rngx.rng_get_state(g))
    assert np.array_equal(rngx.rng_get_state(g2), rngx.rng_get_state(g))
    torch.cuda.empty_cache()


def test_substream_seeding(rngx, orc):
    """Instance g = instance 0 of the plain seeding skipped g * 2^137 steps:
    sampled instances (indices with several bits set, up to 15 jumps)
    against the oracle's jump-ahead; counters 0; a fill continues them."""
    print("case substreams", flush=True)
    for S, sample in ((32 * 40, (1, 2, 3, 5, 39)), (32 * (1 << 15), (16384, 32767))):
        g = rngx.rng_create_substreams("xs1024w", S, 9)
        got = rngx.rng_get_state(g)
        plain = orc.seed("xs1024w", S, 9)
        W = got.view(np.uint32)
        assert np.array_equal(W[:32], plain.view(np.uint32)[:32])
        assert np.all(got[4 * S: 4 * S + 8 * (S // 32)].view(np.uint64) == 0)
        assert np.array_equal(got[-4:], plain[-4:])
        for inst in sample:
            one = orc.seed("xs1024w", 32, 9)  # one instance: words of instance 0, counter 0
            one.view(np.uint32)[:32] = plain.view(np.uint32)[:32]
            one[-4:] = plain[-4:]
            orc.jump("xs1024w", 32, one, inst << 137)
            assert np.array_equal(W[32 * inst: 32 * inst + 32], one.view(np.uint32)[:32]), (S, inst)
        del g
    g = rngx.rng_create_substreams("xs1024w", 32 * 40, 9)
    st = rngx.rng_get_state(g)
    out = torch.empty(32 * 40 * 16, dtype=torch.int32, device="cuda")
    rngx.rng_fill_u32(g, out, 16)
    want = orc.generate("xs1024w", 32 * 40, st, 16)
    assert np.array_equal(out.cpu().numpy().view(np.uint32).reshape(16, -1), want)
    with pytest.raises(rngx.RngxError):
        rngx.rng_create_substreams("lcg32", 64, 1)


def test_substream_lcg_state_header_is_checked(rngx, orc):
    """A sub-stream LCG image must carry the handle's S-step map; the image
    of a handle with another S is refused and the state is left as it was."""
    for kind in ("lcg32_sub", "lcg64_sub"):
        g = rngx.rng_create(kind, 100, 3)
        img = rngx.rng_get_state(g)
        assert np.array_equal(img, orc.seed(kind, 100, 3))
        other = orc.seed(kind, 100, 4)
        rngx.rng_set_state(g, other)                      # same S: accepted
        assert np.array_equal(rngx.rng_get_state(g), other)
        bad = other.copy()
        words = bad.view(np.uint32 if kind == "lcg32_sub" else np.uint64)
        words[100] += 2                                   # a different A_S
        with pytest.raises(rngx.RngxError):
            rngx.rng_set_state(g, bad)
        assert np.array_equal(rngx.rng_get_state(g), other)
