"""CPU: the device's sin/cos of an angle in degrees stays within 1.5 ulp.

The kernels compute the unit vectors of the filter and the haversine of the
certification with sincos_deg: the angle is reduced by the nearest multiple of
90 degrees, converted to radians with a two-part pi/180, and sin and cos of
the reduced radian argument (|r| <= pi/4) are summed from their Taylor series
through r^17 and r^16 in Horner form, every step one FMA or product. The
error budgets of the FP64 filter (unit-vector components within ~4 ulp) and
of the FP32 filter's bound assume sin and cos each within 1.5 ulp.

These tests replay that operation sequence exactly on the CPU (every FMA and
product rounded once to the nearest double, with exact rational arithmetic)
and compare the results with a 60-digit evaluation of sin and cos of the same
FP64 degrees, at random angles over [-360, 360] and at the awkward ones
(multiples of 45 degrees and their neighbours, tiny angles, signed zeros).
This checks the formula and its constants, not the GPU: the GPU parity tests
check the kernels that use it.
"""
import math
import random
from decimal import Decimal, localcontext
from fractions import Fraction

from tests import hp

DEG2RAD_HI = float.fromhex("0x1.1df46a2529d39p-6")
DEG2RAD_LO = float.fromhex("0x1.5c1d8becdd291p-62")


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def mul(a, b):
    return float(Fraction(a) * Fraction(b))


def add(a, b):
    return float(Fraction(a) + Fraction(b))


def sincos_small(r):
    z = mul(r, r)
    ps = 1.0 / 355687428096000.0
    for k in (-1.0 / 1307674368000.0, 1.0 / 6227020800.0, -1.0 / 39916800.0, 1.0 / 362880.0, -1.0 / 5040.0,
              1.0 / 120.0, -1.0 / 6.0):
        ps = fma(ps, z, k)
    s = fma(ps, mul(z, r), r)
    pc = 1.0 / 20922789888000.0
    for k in (-1.0 / 87178291200.0, 1.0 / 479001600.0, -1.0 / 3628800.0, 1.0 / 40320.0, -1.0 / 720.0,
              1.0 / 24.0, -0.5):
        pc = fma(pc, z, k)
    c = fma(pc, z, 1.0)
    return s, c


def sincos_deg(x):
    q = float(round(mul(x, 1.0 / 90.0)))  # rint: round half to even
    y = fma(-q, 90.0, x)
    p = mul(y, DEG2RAD_HI)
    e = fma(y, DEG2RAD_HI, -p)
    r = add(p, fma(y, DEG2RAD_LO, e))
    sr, cr = sincos_small(r)
    qi = int(q) & 3
    if qi == 0:
        return sr, cr
    if qi == 1:
        return cr, -sr
    if qi == 2:
        return -sr, -cr
    return -cr, sr


def exact(x):
    """60-digit sin and cos of x degrees; exact zeros where x is a multiple
    of 180 (sin) or 90 plus a multiple of 180 (cos)."""
    with localcontext() as c:
        c.prec = hp.PREC
        a = Decimal(x) * hp.pi() / 180
        if abs(a) < Decimal("1e-10"):
            # (the helpers' series stop at an absolute tolerance of 1e-68)
            s, co = a - a ** 3 / 6 + a ** 5 / 120, 1 - a * a / 2 + a ** 4 / 24
        else:
            s, co = hp.sin(a), hp.cos(a)
    if (Fraction(x) / 180).denominator == 1:
        s = Decimal(0)
    if ((Fraction(x) - 90) / 180).denominator == 1:
        co = Decimal(0)
    return s, co


def ulp_err(got, ref):
    """|got - ref| in units of the last place of the double nearest ref (an
    exact zero must come out as zero)."""
    if ref == 0:
        return 0.0 if got == 0.0 else math.inf
    e = math.frexp(float(ref))[1] - 53
    return float(abs(Decimal(got) - ref) / (Decimal(2) ** e))


def angles():
    rng = random.Random(20230117)
    xs = [rng.uniform(-360.0, 360.0) for _ in range(1500)]
    xs += [rng.uniform(-1.0, 1.0) * 10.0 ** rng.uniform(-12, 1) for _ in range(300)]
    for k in range(-8, 9):
        b = 45.0 * k
        xs += [b, math.nextafter(b, math.inf), math.nextafter(b, -math.inf), b + 1e-9, b - 1e-9]
    xs += [0.0, -0.0, 1e-300, 5e-324, 2.0 ** -30, 89.99999999, 90.00000001, 359.9999999999, -359.9999999999]
    return xs


def test_sincos_deg_within_1_5_ulp():
    worst_s = worst_c = 0.0
    for x in angles():
        s, c = sincos_deg(x)
        rs, rc = exact(x)
        es, ec = ulp_err(s, rs), ulp_err(c, rc)
        worst_s, worst_c = max(worst_s, es), max(worst_c, ec)
        assert es <= 1.5 and ec <= 1.5, (x, s, c, es, ec)
    # the series and constants are what they claim: well inside the bound
    assert worst_s < 1.5 and worst_c < 1.5


def test_reduction_stays_within_the_series_range():
    # |r| <= pi/4 (plus the rounding of the conversion) for every reduced angle
    for x in angles():
        q = float(round(mul(x, 1.0 / 90.0)))
        y = fma(-q, 90.0, x)
        assert abs(y) <= 45.0
        r = add(mul(y, DEG2RAD_HI), fma(y, DEG2RAD_LO, fma(y, DEG2RAD_HI, -mul(y, DEG2RAD_HI))))
        assert abs(r) <= math.pi / 4 * (1 + 1e-15)


def test_series_truncation_is_negligible():
    # the first omitted terms at |r| = pi/4, relative to the smallest results there
    r = math.pi / 4
    assert r ** 19 / math.factorial(19) / math.sin(r) < 2.0 ** -62
    assert r ** 18 / math.factorial(18) / math.cos(r) < 2.0 ** -58
