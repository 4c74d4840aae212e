"""GPU: reusable partitions (hlc_partition / hlc_xmatch_part) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hlc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_07331_amd as m
    m.load()
    return m


def _run(hlc, A, B, r, prec, cap):
    import torch
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(cap, dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch_part(A, B, r, out, sep, precision=prec)
    assert st == hlc.HLC_OK, hlc.strerror(st)
    p = out[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    order = np.argsort(keys)
    return keys[order], sep[:n].cpu().numpy()[order]


@pytest.mark.parametrize("prec", [1, 0])
def test_parts_reuse_both_roles(hlc, prec):
    c = synth.patch_pair(scale=0.5, seed_sub=7)
    # crowd the seam and a pole too
    a2, d2, b2, e2 = synth.adversarial("seam", 3000, 3, 3.0)
    a3, d3, b3, e3 = synth.adversarial("pole", 3000, 4, 3.0)
    a_ra = np.concatenate([c.a_ra, a2, a3]); a_dec = np.concatenate([c.a_dec, d2, d3])
    b_ra = np.concatenate([c.b_ra, b2, b3]); b_dec = np.concatenate([c.b_dec, e2, e3])
    st, PA = hlc.hlc_partition(to_dev(a_ra), to_dev(a_dec), 3.0)
    assert st == hlc.HLC_OK
    st, PB = hlc.hlc_partition(to_dev(b_ra), to_dev(b_dec), 3.0)
    assert st == hlc.HLC_OK
    for r in (3.0, 1.0, 0.25):
        ref = oracle.xmatch(a_ra, a_dec, b_ra, b_dec, r)
        keys, sep = _run(hlc, PA, PB, r, prec, len(ref) + 100)
        assert_same(keys, sep, ref, label=f"A-B r={r}")
        ref = oracle.xmatch(b_ra, b_dec, a_ra, a_dec, r)
        keys, sep = _run(hlc, PB, PA, r, prec, len(ref) + 100)
        assert_same(keys, sep, ref, label=f"B-A r={r}")
    ref = oracle.xmatch(a_ra, a_dec, a_ra, a_dec, 1.0)
    keys, sep = _run(hlc, PA, PA, 1.0, prec, len(ref) + 100)
    assert_same(keys, sep, ref, label="A-A")
    assert np.all(np.isin((np.arange(len(a_ra), dtype=np.uint64) << np.uint64(32)) |
                          np.arange(len(a_ra), dtype=np.uint64), keys))
    PA.free()
    PB.free()


@pytest.mark.parametrize("prec", [1, 0])
def test_part_overflow(hlc, prec):
    """Reused partitions: a capacity below the pair count reports the
    required count and writes true pairs into exactly its slots."""
    import torch
    c = synth.patch_pair(scale=0.3, seed_sub=11)
    ref = oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, 2.0)
    rk = np.sort(ref.keys())
    st, PA = hlc.hlc_partition(to_dev(c.a_ra), to_dev(c.a_dec), 2.0)
    assert st == hlc.HLC_OK
    st, PB = hlc.hlc_partition(to_dev(c.b_ra), to_dev(c.b_dec), 2.0)
    assert st == hlc.HLC_OK
    cap, pad = len(ref) // 3, 100
    out = torch.full((cap + pad, 2), -7, dtype=torch.int32, device="cuda")
    sep = torch.full((cap + pad,), -7.0, dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch_part(PA, PB, 2.0, out, sep, precision=prec, capacity=cap)
    assert st == hlc.HLC_E_OVERFLOW and n == len(ref)
    o = out.cpu().numpy()
    assert np.all(o[cap:] == -7) and np.all(sep[cap:].cpu().numpy() == -7.0)
    p = o[:cap].view(np.uint32)
    keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    assert len(np.unique(keys)) == cap and np.all(np.isin(keys, rk))
    PA.free()
    PB.free()


def test_part_errors(hlc):
    import torch
    g = synth.rng(300, 0)
    ra, dec = synth.uniform_sphere(g, 1000)
    st, P1 = hlc.hlc_partition(to_dev(ra), to_dev(dec), 2.0)
    assert st == hlc.HLC_OK
    st, P2 = hlc.hlc_partition(to_dev(ra), to_dev(dec), 2.0, tuning={"zone_height_arcsec": 500.0})
    assert st == hlc.HLC_OK
    out = torch.empty((10, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(10, dtype=torch.float64, device="cuda")
    st, _ = hlc.hlc_xmatch_part(P1, P1, 2.5, out, sep)  # radius beyond the halo
    assert st == hlc.HLC_E_INVAL
    st, _ = hlc.hlc_xmatch_part(P1, P2, 1.0, out, sep)  # different geometry
    assert st == hlc.HLC_E_INVAL
    bad = dec.copy()
    bad[10] = 95.0
    st, P3 = hlc.hlc_partition(to_dev(ra), to_dev(bad), 2.0)
    assert st == hlc.HLC_E_INVAL and P3 is None
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    st, P4 = hlc.hlc_partition(e, e, 2.0)
    assert st == hlc.HLC_OK
    st, n = hlc.hlc_xmatch_part(P4, P1, 1.0, out, sep)
    assert st == hlc.HLC_OK and n == 0
    for P in (P1, P2, P4):
        P.free()
