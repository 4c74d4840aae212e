"""GPU: the paper's HEALPix + quad-direction partition, emulated, against the oracle's emulation."""
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


def _quad(hlc, a_ra, a_dec, b_ra, b_dec, r, order, cap):
    import torch
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(cap, dtype=torch.float64, device="cuda")
    st, n = hlc.hlc_xmatch_quad(to_dev(a_ra), to_dev(a_dec), to_dev(b_ra), to_dev(b_dec), r, order, out, sep)
    assert st == hlc.HLC_OK, hlc.strerror(st)
    p = out[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
    k = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    o = np.argsort(k)
    return k[o], sep[:n].cpu().numpy()[o]


@pytest.mark.parametrize("order", [6, 9, 12, 13])
def test_quad_direction_matches_oracle(hlc, order):
    g = synth.rng(940, order)
    sets = [synth.adversarial(kind, 3000, 2, 3.0) for kind in ("pole", "seam", "dense", "grid")]
    a_ra, a_dec = synth.uniform_patch(g, 40000, 20.0, 21.5, 88.0, 88.3)
    b_ra, b_dec = synth.uniform_patch(g, 40000, 20.0, 21.5, 88.0, 88.3)
    sets.append((a_ra, a_dec, b_ra, b_dec))
    for k, (ar, ad, br, bd) in enumerate(sets):
        ref = oracle.quad_direction(ar, ad, br, bd, 3.0, order)
        keys, sep = _quad(hlc, ar, ad, br, bd, 3.0, order, len(ref) + 100)
        assert_same(keys, sep, ref, label=f"quad order={order} set={k}")
        exact = oracle.xmatch(ar, ad, br, bd, 3.0)
        assert np.all(np.isin(keys, exact.keys()))
