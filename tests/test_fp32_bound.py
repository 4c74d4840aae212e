"""CPU: the FP32 filter's rounding bound never rejects a true pair.

The FP32 form of the filter (the precision form) tests chord^2 in FP32 on
offsets from a group centre, with each record stored as an FP32 lattice
corner plus a 10-bit fixed-point offset at 2^-34 per axis; each lane tests
against (c_r32 + E)^2 (1 + 2^-18), E bounding the rounding (the derivation is
in the kernel's header). These tests emulate that arithmetic step by step
with numpy float32 (every operation the kernel performs, in its order) on
pairs at exactly the radius and just inside it, for group centres from zero
up to far beyond a group's extent, and check that every such pair passes
and that the bound stays tight (far below the 0.04 arcsec of an FP32 filter
on unit vectors). This checks the derivation, not the GPU: the GPU parity
tests check the kernel itself at the threshold.
"""
import math

import numpy as np

F32 = np.float32
UNIT = 2.0 ** -34
AS = math.pi / 180.0 / 3600.0  # radians per arcsec


def unit(ra_deg, dec_deg):
    a, d = np.radians(ra_deg), np.radians(dec_deg)
    return np.stack([np.cos(d) * np.cos(a), np.cos(d) * np.sin(a), np.sin(d)], axis=-1)


def round_down_f32(x):
    f = x.astype(F32)
    up = f.astype(np.float64) > x
    f[up] = np.nextafter(f[up], F32(-np.inf))
    return f


def encode(u):
    """Cell record of FP64 unit vectors: FP32 corners (rounded down) and counts of 2^-34."""
    corner = round_down_f32(u)
    t = np.floor((u - corner.astype(np.float64)) * 2.0 ** 34)
    assert np.all(t >= 0) and np.all(t <= 1023)
    return corner, t


def offset(corner, count, c):
    # fl(fl(corner - c) + count * 2^-34): the product is exact in FP32
    return (corner - c).astype(F32) + (count * UNIT).astype(F32)


def chord2_f32(a, b):
    d = (a - b).astype(F32)
    dz2 = (d[..., 2].astype(np.float64) ** 2).astype(F32)
    s = (d[..., 1].astype(np.float64) ** 2 + dz2).astype(F32)          # fma(dy, dy, dz^2)
    return (d[..., 0].astype(np.float64) ** 2 + s).astype(F32)         # fma(dx, dx, .)


def threshold(a_off, c_r32):
    x, y, z = (a_off[..., k].astype(np.float64) for k in range(3))
    zz = (z * z).astype(F32).astype(np.float64)
    yy = (y * y + zz).astype(F32).astype(np.float64)                   # fma(ay, ay, az^2)
    an = np.sqrt((x * x + yy).astype(F32)).astype(F32)                  # sqrt(fma(ax, ax, .))
    e = F32(float.fromhex("0x1.bb68p-34")) + F32(2e-15) + F32(2.0 ** -24) * (F32(4.01) * an + F32(2.01) * c_r32 + F32(2.0 ** -30))
    cr = (c_r32 + e).astype(F32)
    return (cr * cr * F32(1.0 + 2.0 ** -18)).astype(F32)


def c_r32_of(r_arcsec):
    c = 2.0 * math.sin(0.5 * r_arcsec * AS) * (1.0 + 8.0 * 2.0 ** -53)
    f = F32(c)
    if float(f) < c:
        f = np.nextafter(f, F32(np.inf))
    return f


def pairs_at(rng, n, r_arcsec, shrink):
    """A random; B at separation r * (1 - shrink) in a random direction (exact
    great-circle construction in FP64 on the unit sphere)."""
    ra = rng.uniform(0, 360, n)
    dec = np.degrees(np.arcsin(rng.uniform(-1, 1, n)))
    a = unit(ra, dec)
    # orthonormal tangent basis at a
    z = np.array([0.0, 0.0, 1.0])
    e1 = np.cross(z, a)
    bad = np.linalg.norm(e1, axis=1) < 1e-6
    e1[bad] = np.cross(np.array([1.0, 0.0, 0.0]), a[bad])
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(a, e1)
    th = rng.uniform(0, 2 * np.pi, n)
    t = (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2)
    rho = r_arcsec * AS * (1.0 - shrink)
    b = np.cos(rho) * a + np.sin(rho) * t
    b /= np.linalg.norm(b, axis=1)[:, None]
    return a, b


def group_centres(rng, a, spread_rad):
    """A centre corner near each A: the FP32 corner of a point up to spread_rad away."""
    n = len(a)
    v = a + rng.normal(0, 1, (n, 3)) * spread_rad
    v /= np.linalg.norm(v, axis=1)[:, None]
    return round_down_f32(v)


def run(r_arcsec, spread_rad, shrink, n=40000, seed=0):
    rng = np.random.default_rng(seed)
    a, b = pairs_at(rng, n, r_arcsec, shrink)
    # the true chord in FP64 (error ~1e-16, far below the 1e-9 shrink margins used)
    true_c = np.linalg.norm(a - b, axis=1)
    c = group_centres(rng, a, spread_rad)
    ca, na_ = encode(a)
    cb, nb_ = encode(b)
    ao = offset(ca, na_, c)
    bo = offset(cb, nb_, c)
    s = chord2_f32(ao, bo)
    thr = threshold(ao, c_r32_of(r_arcsec))
    return true_c, s, thr


def test_true_pairs_pass_at_the_threshold():
    for r in (0.5, 1.0, 2.0, 5.0, 60.0):
        for spread in (0.0, 1e-5, 1e-3, 3e-2, 0.5):
            true_c, s, thr = run(r, spread, shrink=1e-9, seed=int(r * 10) + int(spread * 1e6))
            c_r = 2.0 * math.sin(0.5 * r * AS)
            inside = true_c <= c_r
            assert inside.mean() > 0.99
            assert np.all(s[inside] <= thr[inside]), (r, spread, float(np.max(s[inside] / thr[inside])))


def test_bound_is_tight_for_compact_groups():
    # a group half extent of 1e-3 rad (about 200 arcsec): the bound admits
    # chords within about 1e-3 r of r at r = 0.5 arcsec
    r = 0.5
    _, _, thr = run(r, 1e-3, shrink=0.0, n=2000, seed=7)
    c_r = 2.0 * math.sin(0.5 * r * AS)
    widen = np.sqrt(thr.astype(np.float64)) / c_r - 1.0
    assert np.max(widen) < 2e-3
    # the unit-vector form needed about 0.043 arcsec, 8.6 % of this radius
    assert np.max(widen) * r < 0.043 / 20


def test_encoding_is_within_one_unit_below():
    rng = np.random.default_rng(3)
    u = unit(rng.uniform(0, 360, 100000), np.degrees(np.arcsin(rng.uniform(-1, 1, 100000))))
    corner, count = encode(u)
    stored = corner.astype(np.float64) + count * UNIT
    err = u - stored
    assert np.all(err >= 0) and np.all(err < UNIT)
