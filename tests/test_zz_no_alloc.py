"""GPU: hlc_xmatch_noalloc (the entry point that allocates nothing) against
hlc_xmatch through the C ABI, on two calls in a row, the second smaller."""
import ctypes as C

import numpy as np
import pytest

import synth
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hlc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_07331_amd as m
    m.load()
    return m


def _call(m, fn, cat, r, prec, cap):
    import torch
    t = [to_dev(x) for x in cat]
    for _ in range(2):
        pairs = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
        sep = torch.empty(cap, dtype=torch.float64, device="cuda")
        st, n = fn(*t, r, pairs, sep, precision=prec, capacity=cap)
        if st != m.HLC_E_OVERFLOW:
            break
        cap = n + 1024
    assert st == m.HLC_OK, (fn.__name__, st)
    p = pairs[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    o = np.argsort(keys)
    return keys[o], sep[:n].cpu().numpy()[o]


def _cases():
    # two calls in a row, the second smaller: the 100k x 100k patch at r = 1"
    # (its workspace fits the scratch array), then 20k x 20k of the same recipe
    # with sources near a pole and the RA seam added
    big = synth.patch_pair(scale=1.0, seed_sub=21)
    sm = synth.patch_pair(scale=0.2, seed_sub=22)
    a2, d2, b2, e2 = synth.adversarial("seam", 400, 6, 1.0)
    small = (np.concatenate([sm.a_ra, a2]), np.concatenate([sm.a_dec, d2]),
             np.concatenate([sm.b_ra, b2]), np.concatenate([sm.b_dec, e2]))
    return [((big.a_ra, big.a_dec, big.b_ra, big.b_dec), big.r_arcsec), (small, 1.0)]


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_xmatch(hlc, prec):
    for k, (cat, r) in enumerate(_cases()):
        cap = max(len(cat[0]), len(cat[2])) + 1024
        ref_k, ref_s = _call(hlc, hlc.hlc_xmatch, cat, r, prec, cap)
        got_k, got_s = _call(hlc, hlc.hlc_xmatch_noalloc, cat, r, prec, cap)
        print(f"case {k} precision {prec}: {len(got_k)} pairs", flush=True)
        assert len(ref_k) > 0
        assert np.array_equal(got_k, ref_k), f"case {k}: pair sets differ"
        assert np.max(np.abs(got_s - ref_s)) <= 1e-9


def test_noalloc_limits_and_errors(hlc):
    import torch
    g = synth.rng(620, 0)
    ra, dec = synth.uniform_patch(g, 2000, 10.0, 11.0, 5.0, 6.0)
    t = [to_dev(x) for x in (ra, dec, ra, dec)]
    out = torch.empty((4096, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(4096, dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch_noalloc(*t, 1.0, out, sep, flags=hlc.HLC_SORTED)
    assert st == hlc.HLC_E_UNSUPPORTED
    bad = dec.copy()
    bad[7] = np.nan
    st, n = hlc.hlc_xmatch_noalloc(to_dev(ra), to_dev(bad), to_dev(ra), to_dev(dec), 1.0, out, sep)
    assert st == hlc.HLC_E_INVAL
    # beyond the scratch array: a clear refusal, not a fault
    h = synth.rng(621, 0)
    bra, bdec = synth.uniform_sphere(h, 2_000_000)
    bt = [to_dev(x) for x in (bra, bdec, bra, bdec)]
    st, n = hlc.hlc_xmatch_noalloc(*bt, 1.0, out, sep)
    assert st == hlc.HLC_E_UNSUPPORTED
    # overflow reports the required count, as hlc_xmatch does
    st, n = hlc.hlc_xmatch_noalloc(*t, 1.0, out[:10], sep[:10], capacity=10)
    assert st == hlc.HLC_E_OVERFLOW and n >= 2000
