"""Pins of the oracle's Philox4x32 and XORWOW against sources outside this
repository.

Philox4x32-10 and -7 (counter-based section; Salmon et al. 2011): the block
function on full 128-bit counters equals the published known-answer vectors
(tests/golden/philox_kat.txt), and the oracle's per-stream outputs (key from
the seeding, counter = output position / 4) equal rocRAND's philox4x32_10
engine, an independent implementation whose source headers ship with ROCm.
XORWOW (XORShift section; Marsaglia 2003): from any oracle state, the
oracle's outputs equal rocRAND's xorwow engine stepped from the same state
(rocRAND's own seeding is bypassed; the seeding is this library's).
LCG64 (LCG section): the plain step written with Python integers.

The rocRAND program (tests/kat/rocrand_kat.cpp) is compiled for the host
only and runs on the CPU.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
M32 = (1 << 32) - 1
M64 = (1 << 64) - 1


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                w = line.split()
                rows.append((int(w[0]), [int(x, 16) for x in w[1:5]], [int(x, 16) for x in w[5:7]],
                             [int(x, 16) for x in w[7:11]]))
    return rows


@pytest.mark.parametrize("row", _kat_rows(), ids=lambda r: f"r{r[0]}-{r[1][0]:08x}")
def test_philox_published_known_answers(orc, row):
    rounds, ctr, key, want = row
    assert orc.philox4x32_block(ctr, key, rounds) == want


@pytest.fixture(scope="module")
def kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_xorwow.h"):
        pytest.skip("hipcc or rocRAND headers not installed")
    exe = str(tmp_path_factory.mktemp("kat") / "rocrand_kat")
    subprocess.run([hipcc, "--offload-host-only", "-O1", "-x", "hip", os.path.join(HERE, "kat", "rocrand_kat.cpp"),
                    "-o", exe], check=True, capture_output=True)

    def run(*args):
        out = subprocess.run([exe, *[str(a) for a in args]], check=True, capture_output=True, text=True).stdout
        return [int(x, 16) for x in out.split()]
    return run


def test_philox_block_matches_rocrand_on_random_counters(orc, kat):
    rng = np.random.default_rng(5)
    cases = [[0, 0, 0, 0, 0, 0], [M32] * 6, [M32, 0, M32, 0, 1, 2]]
    cases += [[int(v) for v in rng.integers(0, 1 << 32, 6, dtype=np.uint64)] for _ in range(40)]
    for c in cases:
        assert orc.philox4x32_block(c[:4], c[4:], 10) == kat("block", *c), c


@pytest.mark.parametrize("kind", ["philox4x32_10"])
def test_philox_streams_match_rocrand_engine(orc, kat, kind):
    # Streams of the oracle's seeding: key = SM(1+s); output 4b+j = word j of
    # block b.  Several streams, with starts on both sides of the carry from
    # block 2^32 - 1 into the counter's second word.
    S = 8
    st = orc.seed(kind, S, 17)
    keys = st.view(np.uint32)
    total = 0
    for s in range(S):
        key = int(keys[s]) | int(keys[S + s]) << 32
        for b0 in (0, 1000, (1 << 32) - 40, (1 << 40) + 7):
            a = st.copy()
            orc.jump(kind, S, a, 4 * b0, lo=s, hi=s + 1)
            got = orc.generate(kind, S, a, 320, lo=s, hi=s + 1)[:, 0]
            want = kat("philox", key, b0, 320)
            assert [int(v) for v in got] == want, (s, b0)
            total += len(want)
    assert total >= 10000


def test_xorwow_matches_rocrand_engine(orc, kat):
    S = 16
    st = orc.seed("xorwow", S, 23)
    img = st.view(np.uint32)
    starts = [[int(img[q * S + s]) for q in range(6)] for s in range(S)]
    starts.append([1, 0, 0, 0, 0, 0])            # a single set bit
    starts.append([0, 0, 0, 0, M32, M32])        # only v set, d about to wrap
    total = 0
    for x in starts:
        one = np.array([[v] for v in x], dtype=np.uint32).reshape(-1).view(np.uint8).copy()
        got = orc.generate("xorwow", 1, one, 1000)[:, 0]
        assert [int(v) for v in got] == kat("xorwow", *x, 1000), x
        total += 1000
    assert total >= 10000


def test_lcg64_step_in_python_integers(orc):
    S = 5
    st = orc.seed("lcg64", S, 3)
    x = [int(v) for v in st.view(np.uint64)]
    out = orc.generate("lcg64", S, st, 50)
    for k in range(50):
        x = [(2862933555777941757 * v + 1442695040888963407) & M64 for v in x]
        assert [int(v) for v in out[k]] == [v >> 32 for v in x]
    assert [int(v) for v in st.view(np.uint64)] == x
