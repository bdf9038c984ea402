"""The C-ABI library loads, exports every function include/rngx.h declares,
and rejects bad arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rngx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rngx_status|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("rng_create", "rng_fill_u32", "rng_fill_f32", "rng_consume", "rng_skip", "ising_create",
              "ising_sweep", "rngx_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(rngx):
    lib = rngx.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(rngx.SIGNATURES)


def test_library_links_no_oracle_code(rngx):
    # the product library must not carry the oracle's symbols
    lib = rngx.load()
    for name in ("orc_generate", "orc_seed", "orc_ising_sweeps"):
        assert not hasattr(lib, name)


def _err(lib):
    return lib.rngx_last_error().decode()


def test_create_validation(rngx):
    lib = rngx.load()
    h = ctypes.c_void_p()
    assert lib.rng_create(0, 16, 1, ctypes.byref(h)) == -1
    assert lib.rng_create(13, 16, 1, ctypes.byref(h)) == -1
    assert lib.rng_create(1, 0, 1, ctypes.byref(h)) == -1
    assert lib.rng_create(6, 48, 1, ctypes.byref(h)) == -2 and "% 32" in _err(lib)
    for lfg in (10, 11):  # lagged Fibonacci: whole 1024-stream instances
        assert lib.rng_create(lfg, 1000, 1, ctypes.byref(h)) == -2 and "% 1024" in _err(lib)
    assert lib.rng_create(12, (1 << 21) + 1, 1, ctypes.byref(h)) == -5  # MWC_DIFF: multipliers above 2^31
    assert lib.rng_create(1, (1 << 36) + 1, 1, ctypes.byref(h)) == -5
    assert lib.rng_create(1, 16, 1, None) == -1
    assert h.value is None  # nothing was written


@pytest.mark.parametrize("L", [0, 8, 17, 24, 100])
def test_ising_create_rejects_bad_L(rngx, L):
    lib = rngx.load()
    h = ctypes.c_void_p()
    assert lib.ising_create(L, 1, 1, ctypes.byref(h)) == -2
    assert lib.ising_create(32768, 1, 1, ctypes.byref(h)) == -5


@pytest.mark.parametrize("L", [16, 48, 80, 96])
def test_ising_create_rejects_lfg_lattices_of_partial_instances(rngx, L):
    lib = rngx.load()
    h = ctypes.c_void_p()
    for lfg in (10, 11):
        assert lib.ising_create(L, lfg, 1, ctypes.byref(h)) == -2 and "% 64" in _err(lib)


def test_unknown_handles_are_rejected(rngx):
    lib = rngx.load()
    bogus = ctypes.c_void_p(0x1234560)
    assert lib.rng_fill_u32(bogus, ctypes.c_void_p(0x1000), 4, None) == -1
    assert lib.rng_skip(None, 4, None) == -1
    assert lib.rng_destroy(bogus) == -1
    assert lib.ising_sweep(bogus, 0.4, 1, None, None) == -1
    assert lib.ising_destroy(None) == -1
    assert "unknown" in _err(lib)


def test_fill_configuration_lists(rngx):
    """The autotuner's candidates: every small-state kind has the same list
    (its first entry the default, XORWOW's the second); XS1024W threads
    always hold one lane pair."""
    lib = rngx.load()
    small = rngx.rng_fill_configs("lcg32")
    assert len(small) == 7 and small[0] == (1, 4, 512) and (0, 4, 256) in small
    for kind in ("lcg64", "mwc", "xorwow", "philox4x32_10", "philox4x32_7", "lcg32_sub", "lcg64_sub", "mwc_diff"):
        assert rngx.rng_fill_configs(kind) == small
    for kind in ("lfg521", "lfg1279"):  # one wave per 1024-stream instance, paced or not
        assert rngx.rng_fill_configs(kind) == [(1, 16, 256), (0, 16, 256)]
    xs = rngx.rng_fill_configs("xs1024w")
    assert len(xs) == 4 and all(v == 2 for _, v, _ in xs) and xs[0] == (1, 2, 1024)
    for paced, v, block in small + xs:
        assert paced in (0, 1) and v in (2, 4) and block in (256, 512, 1024)
    n = ctypes.c_int()
    assert lib.rng_fill_configs(13, None, ctypes.byref(n)) == -1
    assert lib.rng_fill_configs(1, None, None) == -1
    bogus = ctypes.c_void_p(0x1234560)
    assert lib.rng_set_fill_config(bogus, 0) == -1
    assert lib.rng_autotune_fill(bogus, ctypes.c_void_p(0x1000), 4, 1, None, None) == -1


def test_batch_shape_list(rngx):
    """The batch launch shapes: the default first (1024 threads, 64 sites per
    thread), every entry within a workgroup's limits."""
    lib = rngx.load()
    shapes = rngx.ising_batch_shapes()
    assert len(shapes) == 5 and shapes[0] == (1024, 64, 80 * 1024)
    for threads, sites, lds in shapes:
        assert threads in (256, 512, 1024) and 1 <= sites <= 64 and 0 < lds <= 160 * 1024
    assert len(set(shapes)) == len(shapes)
    assert lib.ising_batch_shapes(None, None) == -1
    bogus = ctypes.c_void_p(0x1234560)
    assert lib.ising_batch_set_shape(bogus, 0) == -1
    v = ctypes.c_int()
    assert lib.ising_batch_get_shape(bogus, ctypes.byref(v)) == -1
    assert lib.ising_batch_autotune(bogus, 10, 1, None, None) == -1


def test_ragged_shape_lists(rngx):
    """Ragged shapes: XS1024W rows per CU, wave kinds and per-lane kinds
    outputs per chunk, the default first; none for the lagged Fibonacci kinds."""
    lib = rngx.load()
    assert rngx.rng_ragged_shapes("xs1024w") == [128, 64, 32]
    for kind in ("lcg32", "lcg64", "lcg32_sub", "lcg64_sub", "mwc", "mwc_diff", "philox4x32_10", "philox4x32_7"):
        assert rngx.rng_ragged_shapes(kind) == [65536, 16384, 262144], kind
    assert rngx.rng_ragged_shapes("xorwow") == [4096, 1024, 16384]
    for kind in ("lfg521", "lfg1279"):
        with pytest.raises(rngx.RngxError):
            rngx.rng_ragged_shapes(kind)
    assert lib.rng_ragged_shapes(1, None, None) == -1
    bogus = ctypes.c_void_p(0x1234560)
    assert lib.rng_ragged_set_shape(bogus, 0) == -1
    v = ctypes.c_int()
    assert lib.rng_ragged_get_shape(bogus, ctypes.byref(v)) == -1
    assert lib.rng_ragged_autotune(bogus, ctypes.c_void_p(0x1000), 1, None, None) == -1


def test_last_error_is_per_thread(rngx):
    import threading
    lib = rngx.load()
    h = ctypes.c_void_p()
    lib.rng_create(99, 1, 1, ctypes.byref(h))
    seen = {}

    def other():
        seen["msg"] = lib.rngx_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == "" and "kind" in _err(lib)
