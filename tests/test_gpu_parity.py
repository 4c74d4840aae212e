"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Every comparison is a bit-exact pair set and |sep_gpu - sep_oracle| <= 1e-9
arcsec, for both filter precisions.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import SEP_TOL_ARCSEC, assert_same, gpu_xmatch, to_dev

pytestmark = pytest.mark.gpu

PRECISIONS = [pytest.param(1, id="fp64"), pytest.param(0, id="fp32")]


@pytest.fixture(scope="module")
def hlc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_07331_amd as m
    m.load()
    return m


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_patch_100k(hlc, prec):
    c = synth.patch_pair()
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)
    keys, sep = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, prec)
    n = assert_same(keys, sep, ref, label=f"patch prec={prec}")
    _print("patch pairs", n, hlc.last_stats())


KINDS = ["random", "pole", "seam", "grid", "dup", "same", "dense"]


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("kind", KINDS)
def test_adversarial(hlc, kind, prec):
    for seed, r in ((0, 0.5), (1, 2.0), (2, 7.0)):
        a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 2999, seed, r)
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec)
        assert_same(keys, sep, ref, label=f"{kind} seed={seed} r={r}")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_zone_heights_and_bins(hlc, prec):
    """Tuned geometries: thin zones (many halo copies), wide zones, coarse and fine RA bins."""
    a_ra, a_dec, b_ra, b_dec = synth.adversarial("dense", 3001, 5, 2.0)
    pr, pd = synth.polar_caps(synth.rng(77, 0), 3000, 0.05)
    a_ra, a_dec = np.concatenate([a_ra, pr[:1500]]), np.concatenate([a_dec, pd[:1500]])
    b_ra, b_dec = np.concatenate([b_ra, pr[1500:]]), np.concatenate([b_dec, pd[1500:]])
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, 2.0)
    for zh in (4.01, 5.0, 30.0, 700.0, 3600.0 * 4):
        for bins in (0, 1, 6, 14, 30):
            tun = {"zone_height_arcsec": zh, "ra_bins_log2": bins}
            keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, 2.0, prec, tuning=tun)
            assert_same(keys, sep, ref, label=f"zh={zh} bins={bins}")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_ragged_sizes(hlc, prec):
    g = synth.rng(200, 0)
    for na, nb in ((1, 1), (1, 50), (15, 16), (16, 17), (17, 15), (63, 65), (64, 64), (4095, 4097),
                   (100_003, 7), (7, 100_003), (65_537, 65_535)):
        a_ra, a_dec = synth.uniform_patch(g, na, 10.0, 10.2, -5.0, -4.8)
        b_ra, b_dec = synth.uniform_patch(g, nb, 10.0, 10.2, -5.0, -4.8)
        r = 30.0
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec)
        assert_same(keys, sep, ref, label=f"na={na} nb={nb}")


def test_empty_and_invalid(hlc):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    one_ra = to_dev([10.0])
    one_dec = to_dev([20.0])
    out = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(4, dtype=torch.float64, device="cuda")
    for prec in (0, 1):
        st, n = hlc.hlc_xmatch(e, e, one_ra, one_dec, 1.0, out, sep, precision=prec)
        assert st == hlc.HLC_OK and n == 0
        st, n = hlc.hlc_xmatch(one_ra, one_dec, e, e, 1.0, out, sep, precision=prec)
        assert st == hlc.HLC_OK and n == 0
        st, n = hlc.hlc_xmatch(e, e, e, e, 1.0, out, sep, precision=prec)
        assert st == hlc.HLC_OK and n == 0
        # empty side does not hide a bad coordinate on the other
        st, n = hlc.hlc_xmatch(e, e, to_dev([10.0]), to_dev([91.0]), 1.0, out, sep, precision=prec)
        assert st == hlc.HLC_E_INVAL
    bad = [(float("nan"), 0.0), (0.0, float("nan")), (-1e-300, 0.0), (360.0000001, 0.0), (10.0, 90.5),
           (10.0, -90.0000001), (float("inf"), 0.0)]
    g = synth.rng(201, 0)
    ra, dec = synth.uniform_sphere(g, 1000)
    for prec in (0, 1):
        for (x, y) in bad:
            ra2, dec2 = ra.copy(), dec.copy()
            ra2[517], dec2[517] = x, y
            st, _ = hlc.hlc_xmatch(to_dev(ra2), to_dev(dec2), to_dev(ra), to_dev(dec), 1.0, out, sep,
                                   precision=prec)
            assert st == hlc.HLC_E_INVAL, (x, y)
            st, _ = hlc.hlc_xmatch(to_dev(ra), to_dev(dec), to_dev(ra2), to_dev(dec2), 1.0, out, sep,
                                   precision=prec)
            assert st == hlc.HLC_E_INVAL, (x, y)
        # the boundary values themselves are valid
        ra2, dec2 = ra.copy(), dec.copy()
        ra2[:4] = [0.0, 360.0, 0.0, 360.0]
        dec2[:4] = [90.0, -90.0, -90.0, 90.0]
        st, _ = hlc.hlc_xmatch(to_dev(ra2), to_dev(dec2), to_dev(ra), to_dev(dec), 1.0, out, sep,
                               precision=prec)
        assert st in (hlc.HLC_OK, hlc.HLC_E_OVERFLOW)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_overflow_reports_required_count(hlc, prec):
    import torch
    c = synth.patch_pair(scale=0.2)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)
    args = [to_dev(x) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]
    for cap in (0, 1, len(ref) - 1):
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda")
        sep = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
        st, n = hlc.hlc_xmatch(*args, c.r_arcsec, out, sep, precision=prec, capacity=cap)
        assert st == hlc.HLC_E_OVERFLOW and n == len(ref)
    out = torch.empty((len(ref), 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(len(ref), dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch(*args, c.r_arcsec, out, sep, precision=prec)
    assert st == hlc.HLC_OK and n == len(ref)
    # HLC_NO_SEP: no separation buffer needed
    st, n = hlc.hlc_xmatch(*args, c.r_arcsec, out, None, precision=prec, flags=hlc.HLC_NO_SEP)
    assert st == hlc.HLC_OK and n == len(ref)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_overflow_writes_within_capacity(hlc, prec):
    """A call whose pairs exceed its capacity fills exactly the capacity's
    slots with distinct true pairs (their separations the oracle's) and
    writes nothing past them."""
    import torch
    c = synth.patch_pair(scale=0.2, seed_sub=3)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)
    rk = ref.keys()
    order = np.argsort(rk)
    rk, rsep = rk[order], ref.sep[order]
    args = [to_dev(x) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]
    pad = 257
    for cap in (1, 777, len(ref) // 2, len(ref) - 1):
        out = torch.full((cap + pad, 2), -7, dtype=torch.int32, device="cuda")
        sep = torch.full((cap + pad,), -7.0, dtype=torch.float64, device="cuda")
        st, n = hlc.hlc_xmatch(*args, c.r_arcsec, out, sep, precision=prec, capacity=cap)
        assert st == hlc.HLC_E_OVERFLOW and n == len(ref), (cap, st, n)
        o, s_ = out.cpu().numpy(), sep.cpu().numpy()
        assert np.all(o[cap:] == -7) and np.all(s_[cap:] == -7.0), f"cap {cap}: written past the capacity"
        p = o[:cap].view(np.uint32)
        keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
        assert len(np.unique(keys)) == cap, f"cap {cap}: duplicate pairs"
        at = np.searchsorted(rk, keys)
        assert np.all(at < len(rk)) and np.array_equal(rk[np.minimum(at, len(rk) - 1)], keys), \
            f"cap {cap}: pairs that are not matches"
        assert np.max(np.abs(s_[:cap] - rsep[at])) <= SEP_TOL_ARCSEC


@pytest.mark.parametrize("prec", PRECISIONS)
def test_threshold_ties_exact(hlc, prec):
    """B at exactly r (dyadic radius) along meridians, the equator and across a pole, +-k ulp."""
    g = np.random.default_rng(5)
    r = 3.515625  # 2^-10 deg
    rdeg = r / 3600.0
    A_ra, A_dec, B_ra, B_dec, truth = [], [], [], [], []
    for _ in range(300):
        ra = float(g.uniform(0, 360))
        dec = float(g.uniform(-80, 80))
        for k in range(-2, 3):
            dd = dec + rdeg
            for _ in range(abs(k)):
                dd = float(np.nextafter(dd, math.inf if k > 0 else -math.inf))
            A_ra.append(ra); A_dec.append(dec); B_ra.append(ra); B_dec.append(dd)
            truth.append(abs(Fraction(dd) - Fraction(dec)) <= Fraction(r) / 3600)
    for _ in range(100):
        ra = float(g.uniform(0, 360))
        for k in range(-2, 3):
            x = ra + rdeg
            for _ in range(abs(k)):
                x = float(np.nextafter(x, math.inf if k > 0 else -math.inf))
            if x >= 360.0:
                x -= 360.0
            d = abs(Fraction(x) - Fraction(ra))
            d = min(d, 360 - d)
            A_ra.append(ra); A_dec.append(0.0); B_ra.append(x); B_dec.append(0.0)
            truth.append(d <= Fraction(r) / 3600)
    # spread the pairs out so each A only meets its own B
    a_ra, a_dec = np.array(A_ra), np.array(A_dec)
    b_ra, b_dec = np.array(B_ra), np.array(B_dec)
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
    keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec)
    assert_same(keys, sep, ref, label="ties")
    own = set(int(k) for k in keys if (k >> np.uint64(32)) == (k & np.uint64(0xffffffff)))
    for i, t in enumerate(truth):
        assert ((i << 32) | i in own) == t, i
    st = hlc.last_stats()
    assert st["n_ties"] > 0


@pytest.mark.parametrize("prec", PRECISIONS)
def test_invariants(hlc, prec):
    a_ra, a_dec, b_ra, b_dec = (synth.quantize(x) for x in synth.adversarial("seam", 3000, 9, 2.0))
    a_ra[a_ra >= 360.0] = 0.0
    b_ra[b_ra >= 360.0] = 0.0
    base, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, 2.0, prec)
    assert len(base) > 0
    sw, sep_sw = gpu_xmatch(b_ra, b_dec, a_ra, a_dec, 2.0, prec)
    t = ((sw & np.uint64(0xffffffff)) << np.uint64(32)) | (sw >> np.uint64(32))
    order = np.argsort(t)
    assert np.array_equal(t[order], base)
    assert np.max(np.abs(sep_sw[order] - sep)) <= 1e-12
    for shift in (180.0, 2.0 ** -30 * 98765):
        rot, _ = gpu_xmatch(np.mod(a_ra + shift, 360.0), a_dec, np.mod(b_ra + shift, 360.0), b_dec, 2.0, prec)
        assert np.array_equal(rot, base)
    fl, _ = gpu_xmatch(a_ra, -a_dec, b_ra, -b_dec, 2.0, prec)
    assert np.array_equal(fl, base)


def test_precisions_agree_and_deterministic(hlc):
    c = synth.patch_pair(scale=0.5, seed_sub=3)
    k64, s64 = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, 1)
    k32, s32 = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, 0)
    assert np.array_equal(k64, k32)
    assert np.max(np.abs(s64 - s32)) <= 1e-9
    k64b, s64b = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, 1)
    assert np.array_equal(k64, k64b) and np.array_equal(s64, s64b)
    k32b, s32b = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, 0)
    assert np.array_equal(k32, k32b) and np.array_equal(s32, s32b)


def test_allocation_failure_injection(hlc):
    c = synth.patch_pair(scale=0.05)
    hlc.shutdown()
    os.environ["HLC_TEST_FAIL_ALLOC"] = "1"
    try:
        args = [to_dev(x) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]
        import torch
        out = torch.empty((10000, 2), dtype=torch.int32, device="cuda")
        sep = torch.empty(10000, dtype=torch.float64, device="cuda")
        st, _ = hlc.hlc_xmatch(*args, 1.0, out, sep, precision=1)
        assert st == hlc.HLC_E_NOMEM
    finally:
        del os.environ["HLC_TEST_FAIL_ALLOC"]
    keys, sep = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, 1.0, 1)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, 1.0)
    assert_same(keys, sep, ref, label="after NOMEM")


@pytest.fixture(scope="module")
def fullsky():
    return synth.fullsky_pair()


@pytest.fixture(scope="module")
def fullsky_ref(fullsky):
    c = fullsky
    return oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_fullsky_10M(hlc, fullsky, fullsky_ref, prec):
    """The headline workload at full size, every pair compared."""
    c = fullsky
    keys, sep = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, prec)
    n = assert_same(keys, sep, fullsky_ref, label=f"fullsky prec={prec}")
    _print("fullsky pairs", n, hlc.last_stats())


@pytest.mark.timeout(900)
@pytest.mark.parametrize("r", [0.5, 1.0, 5.0])
def test_stress_full_20M(hlc, r):
    """The precision-stress workload at full size (20M x 20M, 10,000 clumps,
    counterparts on [0.99 r, 1.01 r]) with the geometry a plain call picks.
    Both precisions, every pair and separation compared (about 174M pairs at
    5 arcsec)."""
    import time
    from tests.gpu_util import assert_same_sorted, sorted_on_gpu
    import paper_2301_07331_amd as m
    t0 = time.time()
    c = synth.stress_pair(r)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, r)
    ref_keys = ref.keys()
    _print("stress full r", r, "oracle pairs", len(ref), f"{time.time() - t0:.1f}s")
    for prec in (1, 0):
        pairs, sep = m.xmatch(to_dev(c.a_ra), to_dev(c.a_dec), to_dev(c.b_ra), to_dev(c.b_dec), r,
                              precision=prec)
        keys, sp = sorted_on_gpu(pairs, sep)
        del pairs, sep
        assert_same_sorted(keys, sp, ref_keys, ref.sep, label=f"stress full r={r} prec={prec}")
        _print("stress full r", r, "prec", prec, "ok", f"{time.time() - t0:.1f}s", hlc.last_stats())


@pytest.mark.parametrize("r", [0.5, 1.0, 5.0])
@pytest.mark.parametrize("prec", PRECISIONS)
def test_stress_2M(hlc, r, prec):
    """Precision-stress recipe at 2M x 2M (1000 clumps): counterparts on [0.99 r, 1.01 r]."""
    c = synth.stress_pair(r, n=2_000_000, n_clumps=1000)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, r)
    keys, sep = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, r, prec,
                           tuning={"zone_height_arcsec": 10.0 * r})
    n = assert_same(keys, sep, ref, label=f"stress r={r}")
    _print("stress", r, "pairs", n, hlc.last_stats())


@pytest.mark.parametrize("prec", PRECISIONS)
def test_self_match(hlc, prec):
    """HLC_SELF: each unordered pair once as (i, j), i < j, never (i, i)."""
    import torch
    a_ra, a_dec, _, _ = synth.adversarial("dense", 3000, 11, 2.0)
    c = synth.patch_pair(scale=0.3, seed_sub=5)
    ra = np.concatenate([a_ra, c.a_ra, c.b_ra])
    dec = np.concatenate([a_dec, c.a_dec, c.b_dec])
    full = oracle.xmatch(ra, dec, ra, dec, 1.0)
    keep = full.a < full.b
    R = type("R", (), {})()
    R.keys = lambda: full.keys()[keep]
    R.sep = full.sep[keep]
    t_ra, t_dec = to_dev(ra), to_dev(dec)
    pairs, sep = hlc.xmatch(t_ra, t_dec, t_ra, t_dec, 1.0, precision=prec, flags=hlc.HLC_SELF)
    p = pairs.cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    order = np.argsort(keys)
    assert_same(keys[order], sep.cpu().numpy()[order], R, label="self")
    # B must be the same arrays
    out = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    s = torch.empty(4, dtype=torch.float64, device="cuda")
    st, _ = hlc.hlc_xmatch(t_ra, t_dec, t_ra.clone(), t_dec, 1.0, out, s, flags=hlc.HLC_SELF)
    assert st == hlc.HLC_E_INVAL


def test_dense_fp32_sorted_radec(hlc):
    """FP32 calls on dense data: after a call with many candidates per B
    entry the library gathers B's (ra, dec) into sorted order for the
    certification instead of reading them by original index; the first call
    (by index) and the later ones (sorted), a self-match and a sparse call
    after them all match the oracle."""
    g = synth.rng(640, 0)
    a_ra, a_dec = synth.uniform_patch(g, 50_000, 150.0, 150.05, 2.0, 2.05)
    b_ra, b_dec = synth.uniform_patch(g, 50_000, 150.0, 150.05, 2.0, 2.05)
    r = 1.5
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
    for call in range(3):
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, 0)
        assert_same(keys, sep, ref, label=f"dense call {call}")
        st = hlc.last_stats()
        assert st["n_candidates"] >= 2 * st["nb_halo"], st  # (B entries, halo copies included)
    # a self-match in the sorted form (A is B: A's (ra, dec) from the sorted array)
    full = oracle.xmatch(b_ra, b_dec, b_ra, b_dec, r)
    keep = full.a < full.b
    R = type("R", (), {})()
    R.keys = lambda: full.keys()[keep]
    R.sep = full.sep[keep]
    t_ra, t_dec = to_dev(b_ra), to_dev(b_dec)
    pairs, sep = hlc.xmatch(t_ra, t_dec, t_ra, t_dec, r, precision=0, flags=hlc.HLC_SELF)
    p = pairs.cpu().numpy().view(np.uint32).reshape(-1, 2)
    k = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    order = np.argsort(k)
    assert_same(k[order], sep.cpu().numpy()[order], R, label="dense self")
    # a sparse call right after (sorted form, as the last call was dense), then by index again
    c = synth.patch_pair(scale=0.2, seed_sub=9)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)
    for call in range(2):
        keys, sep = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, 0)
        assert_same(keys, sep, ref, label=f"sparse call {call}")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_error_radii(hlc, prec):
    """Eq. (4): theta <= 3 sqrt(ea^2 + eb^2), per pair, against the oracle."""
    import torch
    g = synth.rng(920, 0)
    for kind in ("dense", "pole", "seam", "dup"):
        a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 2500, 6, 2.0)
        ea, eb = g.uniform(0.05, 1.2, len(a_ra)), g.uniform(0.05, 1.2, len(b_ra))
        ref = oracle.xmatch_radii(a_ra, a_dec, ea, b_ra, b_dec, eb, 3.0)
        cap = len(ref) + 100
        out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
        sep = torch.empty(cap, dtype=torch.float64, device="cuda")
        st, n = hlc.hlc_xmatch_radii(to_dev(a_ra), to_dev(a_dec), to_dev(ea), to_dev(b_ra), to_dev(b_dec),
                                     to_dev(eb), 3.0, out, sep, precision=prec)
        assert st == hlc.HLC_OK, hlc.strerror(st)
        p = out[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
        keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
        o = np.argsort(keys)
        assert_same(keys[o], sep[:n].cpu().numpy()[o], ref, label=f"radii {kind}")
    # Pythagorean radii give exact ties on the meridian; they are matches
    gg = np.random.default_rng(22)
    A_ra, A_dec, B_dec = [], [], []
    for _ in range(200):
        ra, dec = float(gg.uniform(0, 360)), float(gg.uniform(-80, 80))
        A_ra.append(ra); A_dec.append(dec); B_dec.append(dec + 3.515625 / 3600.0)
    A_ra, A_dec, B_dec = map(np.array, (A_ra, A_dec, B_dec))
    ea, eb = np.full(len(A_ra), 0.703125), np.full(len(A_ra), 0.9375)
    ref = oracle.xmatch_radii(A_ra, A_dec, ea, A_ra, B_dec, eb, 3.0)
    out = torch.empty((1000, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(1000, dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch_radii(to_dev(A_ra), to_dev(A_dec), to_dev(ea), to_dev(A_ra), to_dev(B_dec),
                                 to_dev(eb), 3.0, out, sep, precision=prec)
    assert st == hlc.HLC_OK and n == len(ref)
    assert hlc.last_stats()["n_ties"] > 0
    bad = eb.copy()
    bad[3] = -1.0
    st, _ = hlc.hlc_xmatch_radii(to_dev(A_ra), to_dev(A_dec), to_dev(ea), to_dev(A_ra), to_dev(B_dec),
                                 to_dev(bad), 3.0, out, sep, precision=prec)
    assert st == hlc.HLC_E_INVAL


@pytest.mark.parametrize("prec", PRECISIONS)
def test_sorted_output(hlc, prec):
    """HLC_SORTED: the pair list comes back in (a, b) order, element by element equal to the
    oracle's sorted list; also for a self-match, a partition pair and the batched form."""
    import torch
    c = synth.patch_pair(scale=0.2)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)  # sorted by (a, b)
    rk = ref.keys()
    cap = len(rk) + 100
    args = [to_dev(x) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]

    def check(out, sep, n, rk, rs, label):
        p = out[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
        k = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
        assert np.array_equal(k, rk), label
        assert np.max(np.abs(sep[:n].cpu().numpy() - rs)) <= 1e-9, label

    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(cap, dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch(*args, c.r_arcsec, out, sep, precision=prec, flags=hlc.HLC_SORTED)
    assert st == hlc.HLC_OK
    check(out, sep, n, rk, ref.sep, "xmatch")

    st, A = hlc.hlc_partition(args[0], args[1], c.r_arcsec)
    assert st == hlc.HLC_OK
    st, B = hlc.hlc_partition(args[2], args[3], c.r_arcsec)
    assert st == hlc.HLC_OK
    st, n = hlc.hlc_xmatch_part(A, B, c.r_arcsec, out, sep, precision=prec, flags=hlc.HLC_SORTED)
    assert st == hlc.HLC_OK
    check(out, sep, n, rk, ref.sep, "part")
    A.free()
    B.free()

    jobs = [(0, len(c.a_ra), 0, len(c.b_ra), c.r_arcsec)]
    st, n = hlc.hlc_xmatch_batch(jobs, *args, out, sep, precision=prec, flags=hlc.HLC_SORTED)
    assert st == hlc.HLC_OK
    check(out, sep, n, rk, ref.sep, "batch")

    sref = oracle.xmatch(c.b_ra, c.b_dec, c.b_ra, c.b_dec, c.r_arcsec)
    keep = sref.a < sref.b
    sk = sref.keys()[keep]
    st, n = hlc.hlc_xmatch(args[2], args[3], args[2], args[3], c.r_arcsec, out, sep, precision=prec,
                           flags=hlc.HLC_SORTED | hlc.HLC_SELF)
    assert st == hlc.HLC_OK
    check(out, sep, n, sk, sref.sep[keep], "self")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_bin_edges_and_fractions(hlc, prec):
    """Sources exactly on, just inside and just outside RA bin edges (and at sub-bin fraction
    edges), with partners at 0.999 r to 1.001 r across the edge: the group windows built from
    bin edges and sub-bin fractions must keep every pair."""
    g = synth.rng(601, 0)
    rb = 12
    w = 360.0 / (1 << rb)             # bin width of the tuned geometry (deg)
    fw = w / 256.0                    # sub-bin fraction width
    r = 2.0
    n = 4000
    k = g.integers(0, 1 << rb, n)
    sub = g.integers(0, 256, n)
    off = g.choice([0.0, 1e-13, -1e-13, 0.5 * fw, fw - 1e-12], n)
    a_ra = np.mod(k * w + sub * fw + off, 360.0)
    a_dec = g.uniform(-60.0, 60.0, n)
    sgn = g.choice([-1.0, 1.0], n)
    dist = g.uniform(0.999, 1.001, n) * r / 3600.0
    b_ra = np.mod(a_ra + sgn * dist / np.cos(np.radians(a_dec)), 360.0)
    b_dec = a_dec + g.normal(0.0, 1e-6, n)
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
    assert len(ref) > n // 4
    for zh in (30.0, 600.0):
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec,
                               tuning={"zone_height_arcsec": zh, "ra_bins_log2": rb})
        assert_same(keys, sep, ref, label=f"zh={zh}")
        keys, sep = gpu_xmatch(b_ra, b_dec, a_ra, a_dec, r, prec,
                               tuning={"zone_height_arcsec": zh, "ra_bins_log2": rb})
        ref2 = oracle.xmatch(b_ra, b_dec, a_ra, a_dec, r)
        assert_same(keys, sep, ref2, label=f"swapped zh={zh}")


@pytest.mark.parametrize("items", [1, 2, 3, 5])
def test_filter_items_per_wave(hlc, items):
    """The filter's items-per-wave tuning changes the schedule, not the result."""
    a_ra, a_dec, b_ra, b_dec = synth.adversarial("dense", 6000, 11, 2.0)
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, 2.0)
    for prec in (1, 0):
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, 2.0, prec, tuning={"filter_items": items})
        assert_same(keys, sep, ref, label=f"items={items} prec={prec}")


def _framed_cases():
    """Footprints for the data-framed partition: a dense patch (partial RA frame), a polar
    sector under 170 deg of RA with pairs across the pole, a thin equatorial ring (whole RA,
    Dec framed) with pairs across RA 0/360, a 169.9-deg RA band, and a dense patch with a
    few far outliers that a sample of the catalogues misses."""
    g = synth.rng(602, 0)
    ARC = 1.0 / 3600.0
    out = []
    a = synth.uniform_patch(g, 20000, 150.0, 150.2, 10.0, 10.2)
    b = synth.gaussian_offset(g, a[0][:8000], a[1][:8000], 0.7 * ARC)
    out.append(("dense patch", a[0], a[1], b[0], b[1], 1.0))
    ra = g.uniform(10.0, 175.0, 3000)
    dec = 90.0 - g.uniform(0.0, 30.0 * ARC, 3000)
    ra2 = g.uniform(10.0, 175.0, 3000)
    dec2 = 90.0 - g.uniform(0.0, 30.0 * ARC, 3000)
    out.append(("polar sector", ra, dec, ra2, dec2, 5.0))
    ra = synth._wrap_ra(g.uniform(0.0, 360.0, 30000))
    dec = g.uniform(-0.01, 0.01, 30000)
    rb_, db_ = synth.gaussian_offset(g, ra[:15000], dec[:15000], 1.0 * ARC)
    ra[:50] = synth._wrap_ra(g.uniform(-1e-4, 1e-4, 50))
    rb_[:50] = synth._wrap_ra(ra[:50] + g.uniform(-5e-4, 5e-4, 50))
    db_[:50] = dec[:50] + g.uniform(-5e-4, 5e-4, 50)
    out.append(("equatorial ring", ra, dec, rb_, db_, 2.0))
    a = synth.uniform_patch(g, 20000, 100.0, 269.9, -0.2, 0.2)
    b = synth.gaussian_offset(g, a[0][:10000], a[1][:10000], 20.0 * ARC)
    out.append(("169.9-deg band", a[0], a[1], b[0], b[1], 30.0))
    a_ra, a_dec = synth.uniform_patch(g, 200000, 150.0, 150.5, 10.0, 10.5)
    b_ra, b_dec = synth.gaussian_offset(g, a_ra[:50000], a_dec[:50000], 0.5 * ARC)
    a_ra[7:10] = [200.0, 210.0, 150.25]
    a_dec[7:10] = [-60.0, 45.0, -89.9999]
    b_ra[11:14] = a_ra[7:10] + 1e-5
    b_dec[11:14] = a_dec[7:10] + 1e-4 * ARC
    out.append(("patch with outliers", a_ra, a_dec, b_ra, b_dec, 1.0))
    return out


@pytest.mark.parametrize("prec", PRECISIONS)
def test_framed_geometry(hlc, prec):
    """Zones and RA bins span the data's footprint (frame edges, partial RA frames, poles)."""
    for name, a_ra, a_dec, b_ra, b_dec, r in _framed_cases():
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        assert len(ref) > 0, name
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec)
        assert_same(keys, sep, ref, label=name)
        st = hlc.last_stats()
        _print(name, len(ref), "zones", st["n_zones"], "ra_bits", st["ra_bits"],
               "h", round(st["zone_height_arcsec"], 3))
        keys, sep = gpu_xmatch(b_ra, b_dec, a_ra, a_dec, r, prec)
        assert_same(keys, sep, oracle.xmatch(b_ra, b_dec, a_ra, a_dec, r), label=name + " swapped")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_frame_transitions(hlc, prec):
    """Whole-sphere and framed calls in alternation: A's keys computed ahead under the
    whole-sphere frame must be kept only when the call's frame is the whole sphere."""
    g = synth.rng(603, 0)
    ARC = 1.0 / 3600.0
    sphere = synth.uniform_sphere(g, 30000)
    sphere_b = synth.gaussian_offset(g, sphere[0][:12000], sphere[1][:12000], 0.8 * ARC)
    patch = synth.uniform_patch(g, 30000, 40.0, 40.3, -20.0, -19.7)
    patch_b = synth.gaussian_offset(g, patch[0][:12000], patch[1][:12000], 0.8 * ARC)
    cases = {"sphere": (sphere, sphere_b), "patch": (patch, patch_b)}
    refs = {k: oracle.xmatch(a[0], a[1], b[0], b[1], 2.0) for k, (a, b) in cases.items()}
    for k in ("sphere", "patch", "patch", "sphere", "sphere", "patch", "sphere"):
        (a, b) = cases[k]
        keys, sep = gpu_xmatch(a[0], a[1], b[0], b[1], 2.0, prec)
        assert_same(keys, sep, refs[k], label=k)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_fraction_sort(hlc, prec):
    """fraction_sort = 1: the sub-bin key bits sorted too and B's windows cut at
    sub-bin resolution, on the adversarial kinds, tuned geometries (fine and
    coarse bins, thin and wide zones), the framed footprints and clumps."""
    fs = {"fraction_sort": 1}
    for kind in KINDS:
        for seed, r in ((0, 0.5), (1, 2.0), (2, 7.0)):
            a_ra, a_dec, b_ra, b_dec = synth.adversarial(kind, 2999, seed, r)
            ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
            keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec, tuning=fs)
            assert_same(keys, sep, ref, label=f"fraction_sort {kind} seed={seed} r={r}")
    a_ra, a_dec, b_ra, b_dec = synth.adversarial("dense", 3001, 5, 2.0)
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, 2.0)
    for zh in (4.01, 30.0, 3600.0 * 4):
        for bins in (0, 1, 6, 14, 24):
            tun = dict(fs, zone_height_arcsec=zh, ra_bins_log2=bins)
            keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, 2.0, prec, tuning=tun)
            assert_same(keys, sep, ref, label=f"fraction_sort zh={zh} bins={bins}")
    for name, a_ra, a_dec, b_ra, b_dec, r in _framed_cases():
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec, tuning=fs)
        assert_same(keys, sep, ref, label=f"fraction_sort {name}")
    c = synth.stress_pair(1.0, n=2_000_000, n_clumps=1000)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, 1.0)
    keys, sep = gpu_xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, 1.0, prec, tuning=fs)
    assert_same(keys, sep, ref, label="fraction_sort stress 2M")
    _print("fraction_sort stress 2M", hlc.last_stats())


@pytest.mark.parametrize("prec", PRECISIONS)
def test_polar_band_edges(hlc, prec):
    """Whole-sphere frame with the polar cap bands: dense sources around
    |Dec| = 89 deg (where the zone height changes) and around the poles, with
    counterparts on rings of about r, so that pairs cross the band edges and
    the thin cap zones; a uniform background keeps the frame whole."""
    g = synth.rng(909, 0)
    ARC = 1.0 / 3600.0
    bg_a = synth.uniform_sphere(g, 20000)
    bg_b = synth.uniform_sphere(g, 20000)
    for r in (0.5, 2.0, 7.0):
        parts_a, parts_b = [bg_a], [bg_b]
        for d0 in (89.0, -89.0, 89.9999, -89.9999):
            n = 6000
            ra = g.uniform(0.0, 360.0, n)
            dec = np.clip(d0 + g.uniform(-30.0, 30.0, n) * r * ARC, -90.0, 90.0)
            parts_a.append((ra, dec))
            parts_b.append(synth.ring_offset(g, ra[: n // 2], dec[: n // 2], 0.9 * r * ARC, 1.1 * r * ARC))
        a_ra = synth._wrap_ra(np.concatenate([p[0] for p in parts_a]))
        a_dec = np.concatenate([p[1] for p in parts_a])
        b_ra = synth._wrap_ra(np.concatenate([p[0] for p in parts_b]))
        b_dec = np.clip(np.concatenate([p[1] for p in parts_b]), -90.0, 90.0)
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        assert len(ref) > 1000, r
        for tun in (None, {"fraction_sort": 1}):
            keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec, tuning=tun)
            assert_same(keys, sep, ref, label=f"polar band edges r={r} tuning={tun}")
        _print("polar band edges r", r, "pairs", len(ref), hlc.last_stats())


@pytest.mark.parametrize("prec", PRECISIONS)
def test_sparse_key_space(hlc, prec):
    """A whole-sphere frame that is almost empty: three dense clumps far
    apart and a few isolated sources at the extremes of Dec and RA. Most of
    the coarse key index then lies in long empty runs (the stretches one wave
    writes together) and most radix digits are empty."""
    g = synth.rng(910, 0)
    ARC = 1.0 / 3600.0
    for r in (1.0, 20.0):
        parts_a, parts_b = [], []
        for (ra0, dec0) in ((10.0, 60.0), (200.0, -30.0), (359.99, 0.0)):
            ra, dec = synth.cone(g, 4000, ra0, dec0, 200 * r * ARC)
            parts_a.append((ra, dec))
            parts_b.append(synth.gaussian_offset(g, ra[:2500], dec[:2500], 0.5 * r * ARC))
        iso = (np.array([0.0, 90.0, 180.0, 270.0, 359.999999]), np.array([-89.99, -45.0, 0.0, 45.0, 89.99]))
        parts_a.append(iso)
        parts_b.append(iso)
        a_ra = synth._wrap_ra(np.concatenate([p[0] for p in parts_a]))
        a_dec = np.concatenate([p[1] for p in parts_a])
        b_ra = synth._wrap_ra(np.concatenate([p[0] for p in parts_b]))
        b_dec = np.concatenate([p[1] for p in parts_b])
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        assert len(ref) > 1000, r
        keys, sep = gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, prec)
        assert_same(keys, sep, ref, label=f"sparse key space r={r}")
        _print("sparse key space r", r, "pairs", len(ref), hlc.last_stats())
