"""CPU oracle for the per-stream generators and the checkerboard Ising update.

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU-baseline
leg of the benchmark import this package; the product package
(`paper_1204_6193_amd`) never does, and this package imports nothing from it.
The arithmetic lives in plain C (`rng_oracle.c`, built to `liborc.so` with gcc)
and in `exact_ising.py` (high-precision exact finite-lattice values); this
module only marshals numpy buffers.

Kinds are named by string so that the oracle does not depend on the product's
enum values: "lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "xs1024w",
"philox4x32_7", "lcg32_sub", "lcg64_sub" (sub-stream LCGs sharing one
sequence), "lfg521", "lfg1279" (additive lagged Fibonacci, lags (521, 353)
and (1279, 861), 1024 lanes per block-shared instance), "mwc_diff" (MWC with
a different safe-prime multiplier per stream).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = [os.path.join(HERE, "rng_oracle.c")]

KINDS = ["lcg32", "lcg64", "mwc", "xorwow", "philox4x32_10", "xs1024w", "philox4x32_7", "lcg32_sub", "lcg64_sub",
         "lfg521", "lfg1279", "mwc_diff"]
LFG_W = 1024  # lanes (streams) of one lagged Fibonacci instance
LFG_LAGS = {"lfg521": (521, 353), "lfg1279": (1279, 861)}
_CODE = {k: i + 1 for i, k in enumerate(KINDS)}
OUT_U32, OUT_F32, OUT_XOR = 0, 1, 2


def build() -> str:
    """Compile the C oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", *SOURCES, "-o", LIB_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    """Load liborc.so, building it first only if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.orc_mix64.restype = u64
        L.orc_mix64.argtypes = [u64]
        L.orc_splitmix.restype = u64
        L.orc_splitmix.argtypes = [u64, u64]
        L.orc_state_bytes.restype = ctypes.c_size_t
        L.orc_state_bytes.argtypes = [i32, u64]
        L.orc_seed.restype = i32
        L.orc_seed.argtypes = [i32, u64, u64, vp]
        L.orc_generate.restype = i32
        L.orc_generate.argtypes = [i32, u64, vp, u64, u64, u64, i32, vp]
        L.orc_step_n.restype = i32
        L.orc_step_n.argtypes = [i32, u64, vp, u64, u64, u64]
        L.orc_jump.restype = i32
        L.orc_jump.argtypes = [i32, u64, vp, u64, u64, vp, i32]
        L.orc_ising_threshold.restype = u64
        L.orc_ising_threshold.argtypes = [ctypes.c_double, i32]
        L.orc_ising_hot_start.restype = i32
        L.orc_ising_hot_start.argtypes = [ctypes.c_uint32, u64, vp]
        L.orc_ising_energy.restype = ctypes.c_int32
        L.orc_ising_energy.argtypes = [ctypes.c_uint32, vp]
        L.orc_ising_sweeps.restype = i32
        L.orc_ising_sweeps.argtypes = [ctypes.c_uint32, i32, ctypes.c_double, vp, vp, u64, vp]
        L.orc_xs1024_variant_steps.restype = i32
        L.orc_xs1024_variant_steps.argtypes = [i32, vp, u64]
        L.orc_xs1024_equidistribution.restype = i32
        L.orc_xs1024_equidistribution.argtypes = [i32, i32, vp]
        L.orc_is_prime_u64.restype = i32
        L.orc_is_prime_u64.argtypes = [u64]
        L.orc_mwc_multipliers.restype = i32
        L.orc_mwc_multipliers.argtypes = [u64, vp]
        L.orc_mwc_candidates.restype = i32
        L.orc_mwc_candidates.argtypes = [ctypes.c_uint32, u64, vp]
        L.orc_seed_mwcd.restype = i32
        L.orc_seed_mwcd.argtypes = [u64, u64, vp, vp]
        L.orc_philox4x32_block.restype = None
        L.orc_philox4x32_block.argtypes = [vp, vp, i32, vp]
        L.orc_ising_sweeps_hits.restype = i32
        L.orc_ising_sweeps_hits.argtypes = [ctypes.c_uint32, i32, ctypes.c_double, vp, vp, u64, ctypes.c_uint32, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def code(kind: str) -> int:
    return _CODE[kind]


def mix64(z: int) -> int:
    return int(lib().orc_mix64(z))


def splitmix(seed: int, k: int) -> int:
    """SM(k) = mix64(seed + k * gamma)."""
    return int(lib().orc_splitmix(seed, k))


def state_bytes(kind: str, S: int) -> int:
    return int(lib().orc_state_bytes(_CODE[kind], S))


def seed(kind: str, S: int, seed_: int) -> np.ndarray:
    """Canonical state image (uint8) of S freshly seeded streams.
    mwc_diff with many streams takes its multipliers from the threaded
    enumeration below (the sequential search would take minutes)."""
    st = np.zeros(state_bytes(kind, S), dtype=np.uint8)
    if kind == "mwc_diff" and S > 8192:
        a = mwc_multipliers(S, threads=os.cpu_count() or 1)
        _check(lib().orc_seed_mwcd(S, seed_, _ptr(a), _ptr(st)), "seed")
        return st
    _check(lib().orc_seed(_CODE[kind], S, seed_, _ptr(st)), "seed")
    return st


def generate(kind: str, S: int, st: np.ndarray, count: int, lo: int = 0, hi: int | None = None,
             mode: int = OUT_U32) -> np.ndarray:
    """`count` outputs of streams [lo, hi); advances `st` in place.

    U32/F32: array [count, hi-lo] (out[k, s-lo] is output k of stream s).
    XOR: array [hi-lo] with the XOR of each stream's outputs.
    """
    hi = S if hi is None else hi
    w = hi - lo
    if mode == OUT_XOR:
        out = np.zeros(w, dtype=np.uint32)
    else:
        out = np.zeros((count, w), dtype=np.float32 if mode == OUT_F32 else np.uint32)
    _check(lib().orc_generate(_CODE[kind], S, _ptr(st), lo, hi, count, mode, _ptr(out)), "generate")
    return out


def philox4x32_block(ctr, key, rounds: int = 10) -> list:
    """Philox4x32-`rounds` of a full 128-bit counter (4 words) under a
    64-bit key (2 words); returns the 4 output words."""
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_block(_ptr(c), _ptr(k), rounds, _ptr(out))
    return [int(v) for v in out]


def is_prime_u64(n: int) -> bool:
    return bool(lib().orc_is_prime_u64(n))


_MULT_CACHE = np.zeros(0, dtype=np.uint32)
_MULT_BLOCK = 1 << 22  # candidates per enumeration block


def mwc_multipliers(n: int, threads: int = 1) -> np.ndarray:
    """The n largest a < 2^32 with a*2^32 - 1 a safe prime, decreasing.
    threads = 1: the oracle's downward search.  threads > 1: the same test
    applied to blocks of consecutive candidates (from 2^32 - 1 down) on that
    many threads, the qualifying ones concatenated block by block in
    decreasing order; kept for later calls of the process."""
    global _MULT_CACHE
    if threads <= 1:
        out = np.zeros(n, dtype=np.uint32)
        _check(lib().orc_mwc_multipliers(n, _ptr(out)), "mwc multipliers")
        return out
    if _MULT_CACHE.size < n:
        from concurrent.futures import ThreadPoolExecutor

        def block(top):
            flags = np.zeros(_MULT_BLOCK, dtype=np.uint8)
            _check(lib().orc_mwc_candidates(top, _MULT_BLOCK, _ptr(flags)), "mwc candidates")
            return top - np.nonzero(flags)[0].astype(np.int64)

        found, top = [], (1 << 32) - 1
        with ThreadPoolExecutor(max_workers=threads) as ex:
            while sum(len(f) for f in found) < n:
                tops = [top - i * _MULT_BLOCK for i in range(threads)]
                found.extend(ex.map(block, tops))
                top -= threads * _MULT_BLOCK
        _MULT_CACHE = np.concatenate(found).astype(np.uint32)
    return _MULT_CACHE[:n].copy()


def step_n(kind: str, S: int, st: np.ndarray, n: int, lo: int = 0, hi: int | None = None):
    hi = S if hi is None else hi
    _check(lib().orc_step_n(_CODE[kind], S, _ptr(st), lo, hi, n), "step_n")


def _words(n: int) -> np.ndarray:
    nw = max(1, (n.bit_length() + 63) // 64)
    return np.array([(n >> (64 * i)) & ((1 << 64) - 1) for i in range(nw)], dtype=np.uint64)


def jump(kind: str, S: int, st: np.ndarray, n: int, lo: int = 0, hi: int | None = None):
    """Advance streams [lo, hi) by n outputs (n may exceed 2^64)."""
    hi = S if hi is None else hi
    w = _words(n)
    _check(lib().orc_jump(_CODE[kind], S, _ptr(st), lo, hi, _ptr(w), len(w)), "jump")


SUBSTREAM_LOG2 = 137  # XS1024W instances are 2^137 steps apart (Sec. XORShift generators)


def seed_substreams(kind: str, S: int, seed_: int, lo_inst: int = 0, hi_inst: int | None = None) -> np.ndarray:
    """XS1024W sub-stream seeding: every instance starts from the state of
    instance 0 of seed(kind, S, seed_) and skips g * 2^137 steps (the paper
    partitions the sequence into blocks of 2^137 numbers, one per instance).
    Composed of the pinned seeding and jump-ahead.  Only instances
    [lo_inst, hi_inst) are filled in (the rest keep their plain seeding),
    since each costs one jump."""
    if kind != "xs1024w":
        raise ValueError("sub-stream seeding is defined for xs1024w")
    st = seed(kind, S, seed_)
    G = S // 32
    hi_inst = G if hi_inst is None else hi_inst
    W = st.view(np.uint32)
    base = W[:32].copy()
    for g in range(max(lo_inst, 1), hi_inst):
        W[32 * g: 32 * g + 32] = base
        jump(kind, S, st, g << SUBSTREAM_LOG2, lo=32 * g, hi=32 * g + 32)
    return st


XS1024_VARIANTS = ("L329 R347 L344", "R329 L347 R344", "L344 R347 L329", "R344 L347 R329")


def xs1024_variant_steps(variant: int, words, n: int) -> np.ndarray:
    """n steps of a shift-direction variant of the XORShift-1024 part on 32
    words (word 0 most significant); variant 0 is the generator's."""
    W = np.array(words, dtype=np.uint32).copy()
    _check(lib().orc_xs1024_variant_steps(variant, _ptr(W), n), "variant steps")
    return W


def xs1024_equidistribution(variant: int, lane: int) -> np.ndarray:
    """t_l for l = 1..32 (lane -1: warp order); see orc_xs1024_equidistribution."""
    t = np.zeros(32, dtype=np.int32)
    _check(lib().orc_xs1024_equidistribution(variant, lane, _ptr(t)), "equidistribution")
    return t


def ising_threshold(beta: float, dE: int) -> int:
    return int(lib().orc_ising_threshold(beta, dE))


def ising_hot_start(L: int, seed_: int) -> np.ndarray:
    sp = np.zeros(L * L, dtype=np.int8)
    _check(lib().orc_ising_hot_start(L, seed_, _ptr(sp)), "hot start")
    return sp


def ising_energy(L: int, spins: np.ndarray) -> int:
    return int(lib().orc_ising_energy(L, _ptr(np.ascontiguousarray(spins, dtype=np.int8))))


def ising_sweeps(L: int, kind: str, beta: float, st: np.ndarray, spins: np.ndarray, n_sweeps: int,
                 trace: bool = True, hits: int = 1):
    """Run n_sweeps checkerboard sweeps in place, `hits` Metropolis updates
    per visited site; returns the energy trace (int32) or None."""
    tr = np.zeros(max(n_sweeps, 1), dtype=np.int32) if trace else None
    _check(lib().orc_ising_sweeps_hits(L, _CODE[kind], beta, _ptr(st), _ptr(spins), n_sweeps, hits,
                                       _ptr(tr) if trace else None), "ising sweeps")
    return tr[:n_sweeps] if trace else None


def ising_create(L: int, kind: str, seed_: int):
    """Hot-started lattice and its S = L*L/4 freshly seeded streams."""
    return ising_hot_start(L, seed_), seed(kind, L * L // 4, seed_)
