"""GPU: the streaming form (host catalogues, resident B, A slabs, bounded ring) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hlc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_07331_amd as m
    m.load()
    return m


def _pinned(x):
    import torch
    t = torch.empty(len(x), dtype=torch.float64, pin_memory=True)
    t.numpy()[:] = x
    return t


def _keys(pairs):
    return (pairs[:, 0].astype(np.uint64) << np.uint64(32)) | pairs[:, 1].astype(np.uint64)


@pytest.mark.parametrize("prec", [1, 0])
def test_stream_small_ring_many_drains(hlc, prec):
    """A tiny ring forces chunk splitting and many drains; the set must not change."""
    c = synth.patch_pair(scale=0.5, seed_sub=9)
    a2, d2, b2, e2 = synth.adversarial("pole", 4000, 1, 1.0)
    a_ra = np.concatenate([c.a_ra, a2]); a_dec = np.concatenate([c.a_dec, d2])
    b_ra = np.concatenate([c.b_ra, b2]); b_dec = np.concatenate([c.b_dec, e2])
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, 1.0)
    for ring in (2048, 0):
        pairs, sep = hlc.xmatch_stream(_pinned(a_ra), _pinned(a_dec), _pinned(b_ra), _pinned(b_dec), 1.0,
                                       precision=prec, ring_pairs=ring)
        k = _keys(pairs)
        o = np.argsort(k)
        assert_same(k[o], sep[o], ref, label=f"stream ring={ring}")


def test_stream_errors_and_abort(hlc):
    g = synth.rng(400, 0)
    ra, dec = synth.uniform_patch(g, 5000, 0, 1, 0, 1)
    bad = dec.copy()
    bad[3] = 91.0
    st, _ = hlc.hlc_xmatch_stream(_pinned(ra), _pinned(bad), _pinned(ra), _pinned(dec), 5.0,
                                  lambda p, s, n: 0)
    assert st == hlc.HLC_E_INVAL
    st, _ = hlc.hlc_xmatch_stream(_pinned(ra), _pinned(dec), _pinned(ra), _pinned(dec), 5.0,
                                  lambda p, s, n: 1)  # the sink asks to stop
    assert st == hlc.HLC_E_INVAL


@pytest.mark.parametrize("prec", [1, 0])
def test_stream_several_slabs_full_oracle(hlc, prec):
    """3M A in slabs of about 1M (copies overlapping the cross-match), a patch with A
    outliers far from B and just outside its footprint; the whole set against the oracle."""
    g = synth.rng(401, 0)
    a_ra, a_dec = synth.uniform_patch(g, 3_000_000, 150.0, 152.0, 0.0, 2.0)
    b_ra, b_dec = synth.uniform_patch(g, 1_000_000, 150.0, 152.0, 0.0, 2.0)
    # A sources outside B's footprint (clamped into the edge zones and bins)
    a_ra[:1000] = g.uniform(0.0, 360.0, 1000)
    a_dec[:1000] = g.uniform(-89.0, 89.0, 1000)
    # A just outside B's box, within r of its edge
    a_ra[1000:1100] = 150.0 - g.uniform(0.0, 2e-4, 100)
    a_dec[1000:1100] = g.uniform(0.0, 2.0, 100)
    r = 1.0
    ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
    pairs, sep = hlc.xmatch_stream(_pinned(a_ra), _pinned(a_dec), _pinned(b_ra), _pinned(b_dec), r,
                                   precision=prec, ring_pairs=1 << 20)
    k = _keys(pairs)
    o = np.argsort(k)
    assert_same(k[o], sep[o], ref, label=f"slabs prec={prec}")


@pytest.mark.timeout(1200)
def test_stream_large_400M_x_100M_full(hlc):
    """The large workload at full size, both precisions: every pair and separation
    against the oracle's whole join (the exact result is the completeness reference,
    as the paper's section 5.3 takes the exact serial result)."""
    import time
    from tests.gpu_util import assert_same_sorted, sorted_on_gpu
    t0 = time.time()
    c = synth.large_pair()
    print(f"generated in {time.time() - t0:.1f}s", flush=True)
    arrs = [_pinned(x) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]
    got = {}
    for prec in (0, 1):
        t0 = time.time()
        pairs, sep = hlc.xmatch_stream(*arrs, c.r_arcsec, precision=prec, ring_pairs=1 << 26)
        print(f"precision {prec}: streamed {len(pairs)} pairs in {time.time() - t0:.1f}s", flush=True)
        got[prec] = sorted_on_gpu(pairs, sep)
        del pairs, sep
    del arrs
    t0 = time.time()
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec)
    print(f"oracle: {len(ref)} pairs in {time.time() - t0:.1f}s", flush=True)
    ref_keys = ref.keys()
    for prec in (0, 1):
        keys, sep = got[prec]
        n = assert_same_sorted(keys, sep, ref_keys, ref.sep, label=f"400M x 100M prec={prec}")
        print(f"precision {prec}: {n} pairs identical to the oracle", flush=True)


def test_transfer_model_fit(hlc):
    """Eq. (5): T(d) = alpha + beta d fits the timed pinned copies."""
    m = hlc.transfer_model()
    print("transfer model", m, flush=True)
    for d in ("h2d", "d2h"):
        beta = m[f"beta_{d}"]
        assert 1.0 / 400e9 < beta < 1.0 / 1e9, (d, beta)   # 1 .. 400 GB/s
        assert -1e-4 < m[f"alpha_{d}"] < 1e-3, (d, m[f"alpha_{d}"])
        assert m[f"r2_{d}"] > 0.95
