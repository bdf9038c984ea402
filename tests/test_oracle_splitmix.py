"""Pins of the oracle's seeding generator (splitmix64).

The paper only asks for seeding each instance "with another RNG" (LCG and
XORShift sections); splitmix64 (Steele, Lea & Flood 2014) is the project's
choice.  Pins: the counter form equals the sequential generator, mix64 is a
bijection (inverted here by an independent inverse), and the generator's
well-known first output for seed 0.
"""
import random

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _unxorshift(z, s):
    # inverse of z ^= z >> s on 64 bits
    x = z
    for _ in range(64 // s + 1):
        x = z ^ (x >> s)
    return x & M64


def _inv_mix64(z):
    z = _unxorshift(z, 31)
    z = (z * pow(0x94D049BB133111EB, -1, 1 << 64)) & M64
    z = _unxorshift(z, 27)
    z = (z * pow(0xBF58476D1CE4E5B9, -1, 1 << 64)) & M64
    z = _unxorshift(z, 30)
    return z


def test_counter_form_equals_sequential(orc):
    for seed in (0, 1, 0xDEADBEEFCAFEF00D, M64):
        state = seed
        for k in range(1, 200):
            state = (state + GAMMA) & M64
            assert orc.splitmix(seed, k) == orc.mix64(state)


def test_mix64_is_a_bijection(orc):
    rnd = random.Random(7)
    for _ in range(2000):
        z = rnd.getrandbits(64)
        assert _inv_mix64(orc.mix64(z)) == z


def test_first_output_seed0(orc):
    # Soft pin: the widely quoted first output of splitmix64 started at 0.
    assert orc.splitmix(0, 1) == 0xE220A8397B1DCDAF
