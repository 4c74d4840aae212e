"""Print the double-double constants hard-coded in hlc_device.hpp.

pi comes from Machin's formula evaluated with Python's decimal module at 80
digits; each constant is split into an FP64 head and an FP64 tail.
Run: python gen_constants.py
"""
from decimal import Decimal, getcontext

getcontext().prec = 80


def _atan_inv(n: int) -> Decimal:
    x = Decimal(1) / n
    x2, t, s, k = x * x, x, Decimal(0), 0
    while abs(t) > Decimal(10) ** -75:
        s += t / (2 * k + 1) if k % 2 == 0 else -t / (2 * k + 1)
        t *= x2
        k += 1
    return s


PI = 16 * _atan_inv(5) - 4 * _atan_inv(239)


def split(v: Decimal):
    hi = float(v)
    lo = float(v - Decimal(hi))
    return hi, lo


if __name__ == "__main__":
    for name, v in (("DEG2RAD", PI / 180), ("RAD2ARCSEC", 648000 / PI)):
        hi, lo = split(v)
        print(f"{name}_HI = {hi.hex()}  ({hi!r})")
        print(f"{name}_LO = {lo.hex()}  ({lo!r})")
