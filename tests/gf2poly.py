"""GF(2) polynomial tools for the oracle pins (test code, independent of the oracle).

Polynomials are Python ints: bit i is the coefficient of x^i.
"""
from __future__ import annotations

_SPREAD = [0] * 256
for _b in range(256):
    _v = 0
    for _i in range(8):
        if (_b >> _i) & 1:
            _v |= 1 << (2 * _i)
    _SPREAD[_b] = _v


def deg(p: int) -> int:
    return p.bit_length() - 1


def weight(p: int) -> int:
    return bin(p).count("1")


def square(a: int) -> int:
    """a(x)^2 over GF(2): spread the bits (cross terms cancel)."""
    out = 0
    shift = 0
    while a:
        out |= _SPREAD[a & 0xFF] << shift
        a >>= 8
        shift += 16
    return out


def mul(a: int, b: int) -> int:
    """Carry-less product."""
    out = 0
    while b:
        low = b & -b
        out ^= a << (low.bit_length() - 1)
        b ^= low
    return out


def mod(a: int, p: int) -> int:
    dp = deg(p)
    da = deg(a)
    while da >= dp:
        a ^= p << (da - dp)
        da = deg(a)
    return a


def powmod_x(e: int, p: int) -> int:
    """x^e mod p by square-and-multiply."""
    r = 1
    base = mod(2, p)
    for bit in bin(e)[2:]:
        r = mod(square(r), p)
        if bit == "1":
            r = mod(mul(r, base), p)
    return r


def x_pow_2k_mod(k: int, p: int) -> int:
    """x^(2^k) mod p by k squarings."""
    r = mod(2, p)
    for _ in range(k):
        r = mod(square(r), p)
    return r


def gcd(a: int, b: int) -> int:
    while b:
        a, b = b, mod(a, b)
    return a


def is_irreducible(p: int, prime_factors_of_degree) -> bool:
    """Rabin's test: x^(2^n) = x mod p and gcd(x^(2^(n/q)) - x, p) = 1."""
    n = deg(p)
    if x_pow_2k_mod(n, p) != mod(2, p):
        return False
    for q in prime_factors_of_degree:
        if gcd(x_pow_2k_mod(n // q, p) ^ 2, p) != 1:
            return False
    return True


def is_primitive(p: int, prime_factors_of_order) -> bool:
    """p irreducible of degree n is primitive iff x^((2^n-1)/q) != 1 for all prime q | 2^n-1."""
    n = deg(p)
    order = (1 << n) - 1
    if powmod_x(order, p) != 1:
        return False
    return all(powmod_x(order // q, p) != 1 for q in prime_factors_of_order)


def berlekamp_massey(bits) -> int:
    """Minimal connection polynomial of a GF(2) sequence, returned as the
    minimal polynomial (reciprocal of the connection polynomial, degree = L)."""
    C, B = 1, 1
    L, m = 0, 1
    window = 0  # bit j holds s[i - j]
    for i, bit in enumerate(bits):
        window = (window << 1) | (bit & 1)
        d = bin(C & window).count("1") & 1
        if d == 0:
            m += 1
        elif 2 * L <= i:
            T = C
            C ^= B << m
            L = i + 1 - L
            B = T
            m = 1
        else:
            C ^= B << m
            m += 1
    # C(x) = 1 + c1 x + ... + cL x^L ; minimal polynomial = x^L C(1/x)
    rev = 0
    for i in range(L + 1):
        if (C >> i) & 1:
            rev |= 1 << (L - i)
    return rev
