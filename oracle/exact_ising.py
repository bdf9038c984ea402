"""Exact finite-lattice energy and specific heat of the 2D Ising ferromagnet.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The paper compares its Monte Carlo estimates with the exact values for finite
periodic lattices (Ferdinand & Fisher 1969; the Table 2 "exact" row) but does
not print the formula.  This module writes out Kaufman's partition function of
the L x L torus (Kaufman 1949, as used by Ferdinand & Fisher) with J = 1,
h = 0 and K = beta:

    Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4),   N = L^2
    Z1 = prod_{r=0}^{L-1} 2 cosh(L g_{2r+1} / 2)
    Z2 = prod_{r=0}^{L-1} 2 sinh(L g_{2r+1} / 2)
    Z3 = prod_{r=0}^{L-1} 2 cosh(L g_{2r} / 2)
    Z4 = prod_{r=0}^{L-1} 2 sinh(L g_{2r} / 2)
    cosh g_l = cosh 2K coth 2K - cos(pi l / L)      (l >= 1)
    g_0 = 2K + ln tanh K                              (signed)

Observables, as in the paper's Table 2: e = -<E>/N (positive) and
C_V = beta^2 (<E^2> - <E>^2) / N = (K^2 / N) d^2 ln Z / dK^2.

Onsager's infinite-lattice energy is included for the L -> infinity
check.  All arithmetic is mpmath at `DPS` significant digits; mpmath numbers
have an unbounded exponent, so the products need no rescaling.
"""
from __future__ import annotations

import mpmath as mp

DPS = 60
BETA_C = float(mp.log(1 + mp.sqrt(2)) / 2)  # ln(1 + sqrt 2) / 2


def _lnZ(K, L: int):
    """ln Z of the L x L periodic lattice at coupling K (mpmath number)."""
    L = int(L)
    N = L * L
    c2 = mp.cosh(2 * K) * mp.coth(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mp.log(mp.tanh(K))
        return mp.acosh(c2 - mp.cos(mp.pi * l / L))

    z1 = z2 = z3 = z4 = mp.mpf(1)
    for r in range(L):
        go = gamma(2 * r + 1) * L / 2
        ge = gamma(2 * r) * L / 2
        z1 *= 2 * mp.cosh(go)
        z2 *= 2 * mp.sinh(go)
        z3 *= 2 * mp.cosh(ge)
        z4 *= 2 * mp.sinh(ge)
    return mp.log(mp.mpf(1) / 2) + (mp.mpf(N) / 2) * mp.log(2 * mp.sinh(2 * K)) + mp.log(z1 + z2 + z3 + z4)


def exact(L: int, beta: float) -> tuple[float, float]:
    """(e, C_V) of the L x L periodic lattice at inverse temperature beta."""
    with mp.workdps(DPS):
        K = mp.mpf(beta)
        N = L * L
        f = lambda k: _lnZ(k, L)
        d1 = mp.diff(f, K, 1)
        d2 = mp.diff(f, K, 2)
        # <E> = -d lnZ / dK (with beta = K, J = 1), e = -<E>/N = d1 / N
        e = d1 / N
        cv = K * K * d2 / N
        return float(e), float(cv)


def _onsager_u(K):
    """Onsager's internal energy per site u(K) (J = 1, L -> infinity)."""
    t2 = mp.tanh(2 * K)
    k = 2 * mp.sinh(2 * K) / mp.cosh(2 * K) ** 2              # elliptic modulus
    return -mp.coth(2 * K) * (1 + (2 / mp.pi) * (2 * t2 * t2 - 1) * mp.ellipk(k * k))  # mpmath takes m = k^2


def onsager(beta: float) -> tuple[float, float]:
    """Onsager's L -> infinity (e, C_V) per site for J = 1.

    C_V = beta^2 Var(E)/N = -K^2 du/dK, taken by differentiating the closed
    form of u rather than from a second closed form."""
    with mp.workdps(DPS):
        K = mp.mpf(beta)
        u = _onsager_u(K)
        c = -K * K * mp.diff(_onsager_u, K)
        return float(-u), float(c)
