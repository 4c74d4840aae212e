"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:
  * closed-form separations (tests/golden), exact by geometry;
  * exact rational decisions where the separation is a plain difference
    (same meridian, the equator, across a pole);
  * an independent 60-digit ``decimal`` evaluation for generic geometry;
  * brute force over all pairs on small adversarial inputs (completeness of
    the zone join);
  * symmetries of the exact pair set (swap, RA rotation, reflections);
  * the expected number of counterpart and chance pairs of the small patch
    workload.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests import hp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_form_separations.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, kind, ra1, dec1, ra2, dec2, sep = line.split()
        rows.append((name, kind, float(ra1), float(dec1), float(ra2), float(dec2), Fraction(sep)))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: r[0])
def test_closed_form_separations(row):
    name, kind, ra1, dec1, ra2, dec2, sep = row
    exact = float(sep)
    # FP64 path (a radius just above the separation so the pair is "in")
    code, s64 = oracle.pair(ra1, dec1, ra2, dec2, min(max(exact * 1.5, 1e-3), 648000.0))
    assert code in (oracle.IN_FP64, oracle.IN_QUAD, oracle.IN_TIE)
    assert abs(s64 - exact) <= 1e-12 + 1e-14 * exact, (name, s64, exact)
    # binary128 path
    sq = oracle.sep_q(ra1, dec1, ra2, dec2)
    assert abs(sq - exact) <= 1e-12 + 4e-16 * exact, (name, sq, exact)
    # symmetric in the two points
    assert oracle.sep_q(ra2, dec2, ra1, dec1) == sq


def _exact_in(sep_exact: Fraction, r_arcsec: float) -> bool:
    return sep_exact <= Fraction(r_arcsec) / 3600


def _decisions_match(ra1, dec1, ra2, dec2, r, truth):
    code, _ = oracle.pair(ra1, dec1, ra2, dec2, r)
    got = code in (oracle.IN_FP64, oracle.IN_QUAD, oracle.IN_TIE)
    assert got == truth, (ra1, dec1, ra2, dec2, r, code, truth)
    assert oracle.pair_q(ra1, dec1, ra2, dec2, r) == truth
    return code


@pytest.mark.parametrize("r", [0.5, 1.0, 2.0, 3.515625, 5.0, 0.87890625])
def test_meridian_threshold_exact(r):
    """Same RA: theta = |dDec| exactly. B at dDec = r then +-k ulp."""
    g = np.random.default_rng(11)
    rdeg = r / 3600.0
    codes = []
    for _ in range(40):
        ra = float(g.uniform(0, 360))
        dec = float(g.uniform(-80, 80))
        d2 = dec + rdeg
        for k in range(-3, 4):
            dd = d2
            for _ in range(abs(k)):
                dd = np.nextafter(dd, math.inf if k > 0 else -math.inf)
            sep = abs(Fraction(dd) - Fraction(dec))
            codes.append(_decisions_match(ra, dec, ra, float(dd), r, _exact_in(sep, r)))
    # dyadic radii give exact ties on the meridian; they must be counted in
    if r in (3.515625, 0.87890625):
        assert oracle.IN_TIE in codes


@pytest.mark.parametrize("r", [0.5, 2.0, 3.515625])
def test_equator_threshold_exact(r):
    """dec = 0 on both sides: theta = |dRA| (folded) exactly."""
    g = np.random.default_rng(12)
    rdeg = r / 3600.0
    for _ in range(40):
        ra = float(g.uniform(0, 360))
        for sgn in (1, -1):
            r2 = ra + sgn * rdeg
            for k in range(-2, 3):
                x = r2
                for _ in range(abs(k)):
                    x = np.nextafter(x, math.inf if k > 0 else -math.inf)
                x = float(x)
                if x < 0:
                    x += 360.0
                if x > 360.0:
                    x -= 360.0
                d = abs(Fraction(x) - Fraction(ra))
                d = min(d, 360 - d)
                _decisions_match(ra, 0.0, x, 0.0, r, _exact_in(d, r))


@pytest.mark.parametrize("r", [1.0, 3.515625])
def test_crosspole_threshold_exact(r):
    """RAs 180 apart in one hemisphere: theta = 180 - |dec1| - |dec2| exactly."""
    g = np.random.default_rng(13)
    rdeg = r / 3600.0
    for _ in range(30):
        ra = float(g.uniform(0, 180))
        hemi = 1.0 if g.random() < 0.5 else -1.0
        x1 = float(g.uniform(0, rdeg))
        dec1 = hemi * (90.0 - x1)
        d2 = 90.0 - (rdeg - (90.0 - abs(dec1)))
        for k in range(-2, 3):
            dd = d2
            for _ in range(abs(k)):
                dd = np.nextafter(dd, math.inf if k > 0 else -math.inf)
            dd = min(float(dd), 90.0)
            sep = (90 - abs(Fraction(dec1))) + (90 - Fraction(dd))
            _decisions_match(ra, dec1, ra + 180.0, hemi * dd, r, _exact_in(sep, r))


def test_generic_threshold_against_decimal():
    """Random geometry, B placed at ~r then nudged; truth from 60-digit decimal."""
    g = synth.rng(900, 0)
    n = 60
    ra, dec = synth.uniform_sphere(g, n)
    dec = np.clip(dec, -89.9, 89.9)
    for r in (0.5, 2.0, 5.0):
        rdeg = r / 3600.0
        for f in (1 - 1e-6, 1 - 1e-12, 1.0, 1 + 1e-12, 1 + 1e-6):
            b_ra, b_dec = synth.direct(ra, dec, np.full(n, rdeg * f), g.uniform(0, 2 * math.pi, n))
            for i in range(n):
                truth = hp.within(ra[i], dec[i], b_ra[i], b_dec[i], r)
                code, s = oracle.pair(ra[i], dec[i], b_ra[i], b_dec[i], r)
                got = code in (oracle.IN_FP64, oracle.IN_QUAD, oracle.IN_TIE)
                assert got == truth, (i, r, f, code)


def test_separation_accuracy_against_decimal():
    """|sep - sep_exact| within 1e-12 arcsec + 1e-14 relative, 1e-6'' .. 1 deg."""
    g = synth.rng(901, 0)
    n = 30
    ra, dec = synth.uniform_sphere(g, n)
    for sep_as in (1e-6, 1e-3, 0.3, 1.0, 2.0, 10.0, 300.0, 3600.0):
        b_ra, b_dec = synth.direct(ra, dec, np.full(n, sep_as / 3600.0), g.uniform(0, 2 * math.pi, n))
        for i in range(n):
            exact = float(hp.sep_arcsec(ra[i], dec[i], b_ra[i], b_dec[i]))
            code, s = oracle.pair(ra[i], dec[i], b_ra[i], b_dec[i], 3600.0 * 2)
            assert code != oracle.OUT
            assert abs(s - exact) <= 1e-12 + 1e-14 * exact, (sep_as, s, exact)
            assert abs(oracle.sep_q(ra[i], dec[i], b_ra[i], b_dec[i]) - exact) <= 1e-15 + 4e-16 * exact


KINDS = ["random", "pole", "seam", "grid", "dup", "same", "dense"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zone_join_matches_brute_force(kind, seed):
    for r in (0.5, 2.0, 7.0):
        a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 600, seed, r)
        z = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        bf = oracle.brute(a_ra, a_dec, b_ra, b_dec, r)
        assert len(z) == len(bf)
        assert np.array_equal(z.keys(), bf.keys())
        assert np.array_equal(z.sep, bf.sep)


def test_zone_join_brute_force_large_radius():
    """Radius of an arc-minute or more: many zones per window, wide RA windows."""
    g = synth.rng(902, 0)
    a_ra, a_dec = synth.polar_caps(g, 800, 2.0)
    b_ra, b_dec = synth.polar_caps(g, 800, 2.0)
    for r in (60.0, 900.0, 3600.0):
        z = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        bf = oracle.brute(a_ra, a_dec, b_ra, b_dec, r)
        assert np.array_equal(z.keys(), bf.keys()), r
        assert len(z) > 0


def _pairset(res):
    return res.keys()


def test_invariants_swap_shift_reflect():
    g = synth.rng(903, 0)
    for kind in ("seam", "pole", "dense", "grid"):
        a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 1500, 7, 2.0)
        a_ra, a_dec, b_ra, b_dec = (synth.quantize(x) for x in (a_ra, a_dec, b_ra, b_dec))
        a_ra[a_ra >= 360.0] = 0.0
        b_ra[b_ra >= 360.0] = 0.0
        r = 2.0
        base = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        assert len(base) > 0
        # swap A and B: the transposed set, identical separations
        sw = oracle.xmatch(b_ra, b_dec, a_ra, a_dec, r)
        t = (sw.b.astype(np.uint64) << np.uint64(32)) | sw.a.astype(np.uint64)
        order = np.argsort(t)
        assert np.array_equal(t[order], base.keys())
        assert np.array_equal(sw.sep[order], base.sep)
        # RA rotation by a multiple of 2^-30 deg (exact on the quantised grid)
        for shift in (2.0 ** -30 * 12345, 180.0, 359.5):
            ar = np.mod(a_ra + shift, 360.0)
            br = np.mod(b_ra + shift, 360.0)
            assert np.array_equal(np.mod(ar - shift, 360.0), a_ra)  # exact
            rot = oracle.xmatch(ar, a_dec, br, b_dec, r)
            assert np.array_equal(rot.keys(), base.keys()), (kind, shift)
        # dec -> -dec and ra -> 360 - ra
        fl = oracle.xmatch(a_ra, -a_dec, b_ra, -b_dec, r)
        assert np.array_equal(fl.keys(), base.keys())
        mi = oracle.xmatch(np.where(a_ra > 0, 360.0 - a_ra, 0.0), a_dec,
                           np.where(b_ra > 0, 360.0 - b_ra, 0.0), b_dec, r)
        assert np.array_equal(mi.keys(), base.keys())


def test_patch_counts_match_expectation():
    """Counterpart + chance pairs of the 100k patch workload (r = 1'')."""
    c = synth.patch_pair()
    res = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)
    sig = 0.3
    p_in = 1.0 - math.exp(-1.0 / (2 * sig * sig))
    exp_cp = 30000 * p_in
    area_as2 = math.radians(10.0) * (math.sin(math.radians(10.0)) - 0.0) * (180 / math.pi * 3600) ** 2
    exp_ch = 1e5 * (1e5 / area_as2) * math.pi * 1.0 ** 2
    mean = exp_cp + exp_ch
    var = 30000 * p_in * (1 - p_in) + exp_ch
    assert abs(len(res) - mean) <= 5 * math.sqrt(var), (len(res), mean)
    assert res.sep.max() <= 1.0 and res.sep.min() >= 0.0


@pytest.mark.parametrize("bad", [(float("nan"), 0.0), (0.0, float("inf")), (-1e-300, 0.0),
                                 (360.0000000001, 0.0), (10.0, 90.0000000001), (10.0, -91.0)])
def test_invalid_positions_rejected(bad):
    a_ra = np.array([1.0, bad[0]])
    a_dec = np.array([1.0, bad[1]])
    with pytest.raises(oracle.OracleError):
        oracle.xmatch(a_ra, a_dec, np.array([1.0]), np.array([1.0]), 1.0)
    with pytest.raises(oracle.OracleError):
        oracle.xmatch(np.array([1.0]), np.array([1.0]), a_ra, a_dec, 1.0)


def test_bad_radius_and_empty():
    one = np.array([1.0])
    for r in (0.0, -1.0, float("nan"), 3600.5):
        with pytest.raises(oracle.OracleError):
            oracle.xmatch(one, one, one, one, r)
    e = np.array([], dtype=np.float64)
    assert len(oracle.xmatch(e, e, one, one, 1.0)) == 0
    assert len(oracle.xmatch(one, one, e, e, 1.0)) == 0


def test_ra_360_is_ra_0():
    res = oracle.xmatch(np.array([360.0]), np.array([5.0]), np.array([0.0]), np.array([5.0]), 0.1)
    assert len(res) == 1 and res.sep[0] == 0.0


# ---------------------------------------------------------------------------
# per-source error radii (eq. 4): theta <= k sqrt(ea^2 + eb^2)
# ---------------------------------------------------------------------------
def _errs(g, n, lo=0.05, hi=1.2):
    return g.uniform(lo, hi, n)


@pytest.mark.parametrize("kind", ["random", "pole", "seam", "dense", "dup", "same"])
def test_radii_zone_join_matches_brute_force(kind):
    g = synth.rng(910, 0)
    a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 700, 4, 2.0)
    ea, eb = _errs(g, len(a_ra)), _errs(g, len(b_ra))
    z = oracle.xmatch_radii(a_ra, a_dec, ea, b_ra, b_dec, eb, 3.0)
    bf = oracle.xmatch_radii(a_ra, a_dec, ea, b_ra, b_dec, eb, 3.0, brute=True)
    assert np.array_equal(z.keys(), bf.keys()) and np.array_equal(z.sep, bf.sep)
    assert len(z) > 0 or kind == "random"


def test_radii_exact_pythagorean_ties():
    """ea = 45/64, eb = 60/64: k sqrt(ea^2 + eb^2) = 3 * 75/64 = 2^-10 deg exactly."""
    g = np.random.default_rng(21)
    ea_v, eb_v, r = 0.703125, 0.9375, 3.515625
    A_ra, A_dec, B_ra, B_dec, truth = [], [], [], [], []
    for _ in range(60):
        ra, dec = float(g.uniform(0, 360)), float(g.uniform(-80, 80))
        for k in range(-2, 3):
            dd = dec + r / 3600.0
            for _ in range(abs(k)):
                dd = float(np.nextafter(dd, math.inf if k > 0 else -math.inf))
            A_ra.append(ra); A_dec.append(dec); B_ra.append(ra); B_dec.append(dd)
            truth.append(abs(Fraction(dd) - Fraction(dec)) <= Fraction(r) / 3600)
    n = len(A_ra)
    res = oracle.xmatch_radii(A_ra, A_dec, np.full(n, ea_v), B_ra, B_dec, np.full(n, eb_v), 3.0)
    got = set(int(k) for k in res.keys())
    for i, t in enumerate(truth):
        assert ((i << 32) | i in got) == t, i
    assert res.ties > 0
    # constant errors reduce to the fixed-radius join
    fixed = oracle.xmatch(A_ra, A_dec, B_ra, B_dec, r)
    assert np.array_equal(fixed.keys(), res.keys())


def test_radii_per_pair_threshold_against_decimal():
    g = synth.rng(911, 0)
    n = 80
    ra, dec = synth.uniform_sphere(g, n)
    ea, eb = _errs(g, n), _errs(g, n)
    rr = 3.0 * np.sqrt(ea * ea + eb * eb)
    for f in (1 - 1e-9, 1 - 1e-13, 1 + 1e-13, 1 + 1e-9):
        b_ra, b_dec = synth.direct(ra, dec, rr * f / 3600.0, g.uniform(0, 2 * math.pi, n))
        res = oracle.xmatch_radii(ra, dec, ea, b_ra, b_dec, eb, 3.0, brute=True)
        got = set(int(k) for k in res.keys())
        for i in range(n):
            from decimal import Decimal, localcontext
            with localcontext() as c:
                c.prec = 70
                r_exact = 3 * (Decimal(ea[i]) ** 2 + Decimal(eb[i]) ** 2).sqrt()
                h = hp.haversine(ra[i], dec[i], b_ra[i], b_dec[i])
                s = hp.sin(r_exact / 3600 * hp.pi() / 360)
                truth = h <= s * s
            assert ((i << 32) | i in got) == truth, (i, f)


def test_radii_invalid_and_zero_errors():
    one = np.array([1.0])
    with pytest.raises(oracle.OracleError):
        oracle.xmatch_radii(one, one, np.array([-0.1]), one, one, one, 3.0)
    with pytest.raises(oracle.OracleError):
        oracle.xmatch_radii(one, one, np.array([float("nan")]), one, one, one, 3.0)
    with pytest.raises(oracle.OracleError):
        oracle.xmatch_radii(one, one, one, one, one, one, 0.0)
    with pytest.raises(oracle.OracleError):
        oracle.xmatch_radii(one, one, np.array([2000.0]), one, one, one, 3.0)  # radius beyond 3600"
    # zero errors: only identical positions match (theta = 0 <= 0)
    ra = np.array([10.0, 10.0, 10.0 + 1e-9])
    dec = np.array([5.0, 5.0, 5.0])
    res = oracle.xmatch_radii(ra, dec, np.zeros(3), ra[:1], dec[:1], np.zeros(1), 3.0)
    assert sorted(res.a.tolist()) == [0, 1]


# ---------------------------------------------------------------------------
# the paper's partition, emulated: HEALPix nested pixels + quad-direction copies
# ---------------------------------------------------------------------------
def test_healpix_base_faces():
    """Nside = 1: the twelve base pixels are centred at z = 2/3, 0, -2/3 and phi = 45 + 90k / 90k."""
    d = math.degrees(math.asin(2.0 / 3.0))
    assert [oracle.hp_nest(0, 45 + 90 * k, d) for k in range(4)] == [0, 1, 2, 3]
    assert [oracle.hp_nest(0, (90 * k) % 360, 0.0) for k in range(4)] == [4, 5, 6, 7]
    assert [oracle.hp_nest(0, 45 + 90 * k, -d) for k in range(4)] == [8, 9, 10, 11]
    assert oracle.hp_nest(0, 10.0, 90.0) == 0 and oracle.hp_nest(0, 10.0, -90.0) == 8


def test_healpix_in_face_orientation():
    """Order 1: each base face splits into four sub-pixels numbered, in the
    nested scheme's Z order, from the face's southern corner (0) through its
    eastern (1) and western (2) corners to its northern corner (3); the
    in-face x axis runs from the southern towards the eastern corner, y
    towards the western one (Gorski et al. 2005, the nested numbering). The
    points sit well inside one sub-pixel each, placed from the faces' corner
    positions alone: an equatorial face's corners are at Dec -/+ asin(2/3)
    on its central meridian and at Dec 0, 45 deg east and west of it; a north
    polar face's at (its meridian, Dec 0), 45 deg east and west of it at
    Dec asin(2/3), and the pole; a south polar face's mirror those.
    Transposing or mirroring the in-face axes swaps east and west, or north
    and south."""
    cases = [
        # face 4: equatorial, centred on RA 0
        (4, (0.0, -30.0), (30.0, 0.0), (330.0, 0.0), (0.0, 30.0)),
        # face 6: equatorial, centred on RA 180
        (6, (180.0, -30.0), (210.0, 0.0), (150.0, 0.0), (180.0, 30.0)),
        # face 0: north polar, centred on RA 45 (southern corner at RA 45, Dec 0)
        (0, (45.0, 15.0), (75.0, 40.0), (15.0, 40.0), (45.0, 70.0)),
        # face 9: south polar, centred on RA 135 (northern corner at RA 135, Dec 0)
        (9, (135.0, -70.0), (165.0, -40.0), (105.0, -40.0), (135.0, -15.0)),
    ]
    for face, south, east, west, north in cases:
        got = [oracle.hp_nest(1, ra, dec) for ra, dec in (south, east, west, north)]
        assert got == [4 * face + k for k in range(4)], (face, got)


def test_healpix_nesting_and_range():
    """Nested scheme: the parent of a pixel at order k+1 is its index >> 2 at order k."""
    g = synth.rng(930, 0)
    ra, dec = synth.uniform_sphere(g, 3000)
    for k in range(0, 13):
        for i in range(0, 3000, 7):
            p1 = oracle.hp_nest(k + 1, ra[i], dec[i])
            p0 = oracle.hp_nest(k, ra[i], dec[i])
            assert p1 >> 2 == p0
            assert 0 <= p1 < 12 * 4 ** (k + 1)


def test_healpix_equal_areas():
    """Uniform points fill the 192 pixels of order 2 equally (chi-square, 191 dof)."""
    g = synth.rng(931, 0)
    n = 96000
    ra, dec = synth.uniform_sphere(g, n)
    counts = np.bincount([oracle.hp_nest(2, ra[i], dec[i]) for i in range(n)], minlength=192)
    e = n / 192
    chi2 = float(((counts - e) ** 2 / e).sum())
    assert chi2 < 191 + 5 * math.sqrt(2 * 191)


def _alg1_plain(a_ra, a_dec, b_ra, b_dec, r, order):
    """Algorithm 1 and the per-pixel join written out with Python dicts (tiny inputs)."""
    R = r / 3600.0

    def pix(ra, dec):
        out = []
        for (x, y) in ((ra, dec), ((ra + R) % 360.0, dec), ((ra - R) % 360.0, dec),
                       (ra, min(dec + R, 90.0)), (ra, max(dec - R, -90.0))):
            p = oracle.hp_nest(order, x, y)
            if p not in out:
                out.append(p)
        return out

    PB = {}
    pb_all = [pix(b_ra[j], b_dec[j]) for j in range(len(b_ra))]
    for j, ps in enumerate(pb_all):
        for p in ps:
            PB.setdefault(p, []).append(j)
    found = set()
    for i in range(len(a_ra)):
        for p in pix(a_ra[i], a_dec[i]):
            for j in PB.get(p, []):
                code, _ = oracle.pair(a_ra[i], a_dec[i], b_ra[j], b_dec[j], r)
                if code in (oracle.IN_FP64, oracle.IN_QUAD, oracle.IN_TIE):
                    found.add((i << 32) | j)
    return np.array(sorted(found), dtype=np.uint64)


@pytest.mark.parametrize("order", [6, 9, 12])
def test_quad_direction_against_plain_algorithm(order):
    for kind in ("dense", "pole", "seam"):
        a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 250, 8, 2.0)
        q = oracle.quad_direction(a_ra, a_dec, b_ra, b_dec, 2.0, order)
        assert np.array_equal(q.keys(), _alg1_plain(a_ra, a_dec, b_ra, b_dec, 2.0, order))


def test_quad_direction_subset_and_loss():
    """The emulated scheme finds only true pairs; at high Dec, where a shift of R
    in RA covers only R cos(Dec) on the sky, it loses some, more at finer orders."""
    g = synth.rng(932, 0)
    a_ra, a_dec = synth.uniform_patch(g, 30000, 20.0, 21.5, 88.0, 88.3)
    b_ra, b_dec = synth.uniform_patch(g, 30000, 20.0, 21.5, 88.0, 88.3)
    r = 3.0
    exact = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
    lost = []
    for order in (8, 10, 13):
        q = oracle.quad_direction(a_ra, a_dec, b_ra, b_dec, r, order)
        assert np.all(np.isin(q.keys(), exact.keys()))
        lost.append(len(exact) - len(q))
    assert lost[0] < lost[1] < lost[2] and 0 < lost[2] < len(exact) // 100
