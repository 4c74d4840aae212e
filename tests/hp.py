"""High-precision spherical separation in pure Python ``decimal`` (tests only).

An independent yardstick for the oracle: pi from Machin's formula, sin/cos
from their Taylor series, asin by Newton's method on sin, all at 60 digits.
It shares nothing with ``oracle/`` or the GPU library. Inputs are FP64
degrees converted exactly (Decimal(float) is exact).
"""
from __future__ import annotations

from decimal import Decimal, getcontext, localcontext
from fractions import Fraction

PREC = 60


def _atan_inv(n: int) -> Decimal:
    # atan(1/n) = sum (-1)^k / ((2k+1) n^(2k+1))
    x = Decimal(1) / n
    x2 = x * x
    term, s, k = x, Decimal(0), 0
    eps = Decimal(10) ** (-(PREC + 5))
    while abs(term) > eps:
        s += term / (2 * k + 1) if k % 2 == 0 else -term / (2 * k + 1)
        term *= x2
        k += 1
    return s


def pi() -> Decimal:
    with localcontext() as c:
        c.prec = PREC + 10
        return 16 * _atan_inv(5) - 4 * _atan_inv(239)


def _reduce(x: Decimal, P: Decimal) -> Decimal:
    # into (-pi, pi]
    two = 2 * P
    k = (x / two).to_integral_value()
    return x - k * two


def sin(x: Decimal) -> Decimal:
    with localcontext() as c:
        c.prec = PREC + 10
        x = _reduce(x, pi())
        term, s, k = x, Decimal(0), 1
        eps = Decimal(10) ** (-(PREC + 8))
        while abs(term) > eps:
            s += term
            term = -term * x * x / ((k + 1) * (k + 2))
            k += 2
        return s


def cos(x: Decimal) -> Decimal:
    with localcontext() as c:
        c.prec = PREC + 10
        x = _reduce(x, pi())
        term, s, k = Decimal(1), Decimal(0), 0
        eps = Decimal(10) ** (-(PREC + 8))
        while abs(term) > eps:
            s += term
            term = -term * x * x / ((k + 1) * (k + 2))
            k += 2
        return s


def asin(y: Decimal) -> Decimal:
    """Newton on sin(z) = y, for |y| well below 1 (small separations)."""
    with localcontext() as c:
        c.prec = PREC + 10
        z = Decimal(float(y))  # FP64 start
        import math
        z = Decimal(math.asin(float(y)))
        for _ in range(8):
            z = z - (sin(z) - y) / cos(z)
        return z


def haversine(ra1, dec1, ra2, dec2) -> Decimal:
    """sin^2(theta/2) for two FP64 positions in degrees."""
    with localcontext() as c:
        c.prec = PREC + 10
        K = pi() / 180
        d1, d2 = Decimal(dec1), Decimal(dec2)
        a1, a2 = Decimal(ra1), Decimal(ra2)
        s1 = sin((d1 - d2) * K / 2)
        s2 = sin((a1 - a2) * K / 2)
        return s1 * s1 + cos(d1 * K) * cos(d2 * K) * s2 * s2


def sep_arcsec(ra1, dec1, ra2, dec2) -> Decimal:
    with localcontext() as c:
        c.prec = PREC + 10
        h = haversine(ra1, dec1, ra2, dec2)
        return 2 * asin(h.sqrt()) * 648000 / pi()


def within(ra1, dec1, ra2, dec2, r_arcsec) -> bool:
    """Exact-real style decision theta <= r, at PREC digits."""
    with localcontext() as c:
        c.prec = PREC + 10
        h = haversine(ra1, dec1, ra2, dec2)
        s = sin(Decimal(r_arcsec) / 3600 * pi() / 360)
        return h <= s * s


def frac(x: float) -> Fraction:
    return Fraction(x)
