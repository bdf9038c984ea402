"""The XS1024W step as the kernels lay it out, emulated on the CPU.

One 1024-bit instance lives in a 16-lane row, lane j holding words 2j and
2j+1 (word 0 most significant).  The kernels make, in each lane, the funnel
shift of its own words that the lane 5 positions away needs, and move it
with a row shift whose lanes outside the row read zero.  This emulation of
that data movement must equal the generator's definition X ^= X << 329;
X ^= X >> 347; X ^= X << 344 on the 1024-bit number (XORShift section).
"""
import random

M32 = 0xFFFFFFFF


def _from_plus(v, n):   # lane j <- lane j+n of the row, zero outside
    return [v[j + n] if j + n < 16 else 0 for j in range(16)]


def _from_minus(v, n):  # lane j <- lane j-n of the row, zero outside
    return [v[j - n] if j - n >= 0 else 0 for j in range(16)]


def _funnel(hi, lo, s):  # (hi << (32 - s)) | (lo >> s)
    return [((h << (32 - s)) | (l >> s)) & M32 for h, l in zip(hi, lo)]


def _xor(x, y):
    return [p ^ q for p, q in zip(x, y)]


def row_step(a, b):
    ta, tb = _funnel(a, b, 23), _funnel(b, _from_plus(a, 1), 23)
    a, b = _xor(a, _from_plus(ta, 5)), _xor(b, _from_plus(tb, 5))
    ta, tb = _funnel(_from_minus(b, 1), a, 27), _funnel(a, b, 27)
    a, b = _xor(a, _from_minus(ta, 5)), _xor(b, _from_minus(tb, 5))
    ta, tb = _funnel(a, b, 8), _funnel(b, _from_plus(a, 1), 8)
    a, b = _xor(a, _from_plus(ta, 5)), _xor(b, _from_plus(tb, 5))
    return a, b


def definition_step(a, b):
    x = 0
    for j in range(16):
        x = (x << 64) | (a[j] << 32) | b[j]
    m = (1 << 1024) - 1
    x ^= (x << 329) & m
    x ^= x >> 347
    x ^= (x << 344) & m
    w = [(x >> (32 * (31 - i))) & M32 for i in range(32)]
    return w[0::2], w[1::2]


def test_row_form_equals_the_definition():
    rnd = random.Random(1)
    for t in range(1500):
        a = [rnd.getrandbits(32) for _ in range(16)]
        b = [rnd.getrandbits(32) for _ in range(16)]
        assert row_step(a, b) == definition_step(a, b), t


def test_row_form_on_single_bits():
    """Every one of the 1024 unit vectors: each bit's three shifted copies
    land in the right word and lane, including the ones shifted out."""
    for i in range(1024):
        a, b = [0] * 16, [0] * 16
        w = i // 32
        (a if w % 2 == 0 else b)[w // 2] = 1 << (i % 32)
        assert row_step(a, b) == definition_step(a, b), i
