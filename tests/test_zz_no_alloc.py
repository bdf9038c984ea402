"""The ragged fill that allocates nothing (rng_fill_ragged_u32_noalloc)
against the planned ragged fill (rng_ragged_create + rng_fill_ragged_u32):
two calls in a row, the second with a smaller request list, give the same
values and the same stream states; a list that needs more than the static
scratch is refused before anything changes."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

KINDS = ["xs1024w", "lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "mwc_diff"]


def _lens(kind, n, seed, big):
    rng = np.random.default_rng(seed)
    top = 22 if big else 14
    lens = np.floor(2.0 ** rng.uniform(0, top, size=n)).astype(np.int64)
    lens[0] = 0
    lens[1] = 1
    return lens


@pytest.mark.parametrize("kind", KINDS)
def test_noalloc_ragged_equals_planned_ragged(rngx, kind):
    width = 32 if kind == "xs1024w" else 1
    n = 40
    S = width * n
    ga = rngx.rng_create(kind, S, 31)  # the no-alloc call's generator
    gb = rngx.rng_create(kind, S, 31)  # the planned path's twin
    for rep, big in enumerate((True, False)):  # the second call is smaller
        print(f"case noalloc {kind} call {rep}", flush=True)
        lens = _lens(kind, n, 100 + rep, big)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
        total = int(off[-1])
        oa = torch.full((total + 4,), -1, dtype=torch.int32, device="cuda")
        ob = torch.full((total + 4,), -1, dtype=torch.int32, device="cuda")
        rngx.rng_fill_ragged_u32_noalloc(ga, off, oa)
        plan = rngx.rng_ragged_create(gb, off)
        rngx.rng_fill_ragged_u32(plan, ob)
        torch.cuda.synchronize()
        plan.destroy()
        assert torch.equal(oa, ob), (kind, rep)
        assert int(oa[total].item()) == -1  # nothing past the end
        assert np.array_equal(rngx.rng_get_state(ga), rngx.rng_get_state(gb)), (kind, rep)


def test_noalloc_ragged_refuses_lists_beyond_the_scratch(rngx):
    """XORWOW chunks of 4096 values need 64 bytes of staging each, so 2^31
    values per stream over 1000 streams exceed 64 MiB: refused with
    RNGX_E_OVERFLOW, the streams unchanged."""
    g = rngx.rng_create("xorwow", 1000, 5)
    before = rngx.rng_get_state(g)
    off = np.arange(0, 1001, dtype=np.uint64) * np.uint64(1 << 31)
    dummy = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(rngx.RngxError) as e:
        rngx.load()  # the binding checks the buffer size, so call the C-ABI directly
        st = rngx.load().rng_fill_ragged_u32_noalloc(g.handle, off.ctypes.data, off.size, dummy.data_ptr(), None)
        rngx._check(st)
    assert e.value.status == -5
    assert np.array_equal(rngx.rng_get_state(g), before)
