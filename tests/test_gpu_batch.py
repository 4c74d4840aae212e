"""GPU: the batched form (many jobs, one persistent graph-captured pass) against the oracle."""
import numpy as np
import pytest

import oracle
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


def _oracle_batch(jobs, a_ra, a_dec, b_ra, b_dec):
    keys, seps, counts = [], [], []
    for (ao, na, bo, nb, r) in jobs:
        if na == 0 or nb == 0:
            counts.append(0)
            continue
        res = oracle.xmatch(a_ra[ao:ao + na], a_dec[ao:ao + na], b_ra[bo:bo + nb], b_dec[bo:bo + nb], r)
        k = ((res.a.astype(np.uint64) + np.uint64(ao)) << np.uint64(32)) | (res.b.astype(np.uint64) + np.uint64(bo))
        keys.append(k)
        seps.append(res.sep)
        counts.append(len(res))
    keys = np.concatenate(keys) if keys else np.empty(0, np.uint64)
    seps = np.concatenate(seps) if seps else np.empty(0)
    return keys, seps, np.array(counts, np.int64)


def _run(hlc, jobs, arrs, prec, cap, tuning=None):
    import torch
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(cap, dtype=torch.float64, device="cuda")
    cnt = torch.empty(len(jobs), dtype=torch.int64, device="cuda")
    st, n = hlc.hlc_xmatch_batch(jobs, *arrs, out, sep, cnt, precision=prec, tuning=tuning)
    assert st == hlc.HLC_OK, hlc.strerror(st)
    p = out[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
    k = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    return k, sep[:n].cpu().numpy(), cnt.cpu().numpy()


def _compare(k, s, c, ref, label):
    rk, rs, rc = ref
    o = np.argsort(k)
    ro = np.argsort(rk)
    assert len(k) == len(rk), (label, len(k), len(rk))
    assert np.array_equal(k[o], rk[ro]), label
    if len(k):
        assert np.max(np.abs(s[o] - rs[ro])) <= 1e-9, label
    assert np.array_equal(c, rc), label


def _mixed_batch():
    b = synth.batch_jobs(njobs=300, median=400, nmin=20, nmax=20000, seed_sub=1)
    a_ra, a_dec, b_ra, b_dec = [b.a_ra], [b.a_dec], [b.b_ra], [b.b_dec]
    jobs = [(int(b.a_off[j]), int(b.na[j]), int(b.b_off[j]), int(b.nb[j]), float(b.r_arcsec[j]))
            for j in range(b.njobs)]
    na_tot, nb_tot = len(b.a_ra), len(b.b_ra)
    for kind, r in (("pole", 2.0), ("seam", 1.5), ("dense", 3.0), ("grid", 2.0), ("same", 1.0)):
        ar, ad, br, bd = synth.adversarial(kind, 1500, 3, r)
        jobs.append((na_tot, len(ar), nb_tot, len(br), r))
        a_ra.append(ar); a_dec.append(ad); b_ra.append(br); b_dec.append(bd)
        na_tot += len(ar); nb_tot += len(br)
    # empty jobs, and jobs whose ranges overlap earlier ones
    jobs.append((0, 0, 0, 100, 1.0))
    jobs.append((5, 100, 0, 0, 1.0))
    jobs.append((jobs[0][0], jobs[0][1], jobs[0][2], jobs[0][3], 2.5))
    jobs.append((jobs[-2 - 5][0], jobs[-2 - 5][1], jobs[-2 - 5][2], jobs[-2 - 5][3], 0.7))
    cat = tuple(np.concatenate(x) for x in (a_ra, a_dec, b_ra, b_dec))
    return jobs, cat


@pytest.mark.parametrize("prec", [1, 0])
def test_batch_mixed_jobs(hlc, prec):
    jobs, cat = _mixed_batch()
    ref = _oracle_batch(jobs, *cat)
    arrs = [to_dev(x) for x in cat]
    cap = len(ref[0]) + 1000
    for tuning in (None, {"zone_height_factor": 0.5}, {"zone_height_factor": 3.0}):
        k, s, c = _run(hlc, jobs, arrs, prec, cap, tuning)
        _compare(k, s, c, ref, f"mixed tuning={tuning}")


def test_batch_every_tuning_candidate(hlc):
    """Every configuration the batched autotuner can choose (zone-height factor
    x partition tile x match blocks per compute unit), each run against the
    oracle; then the autotuned call, whose choice is reported in the stats."""
    jobs, cat = _mixed_batch()
    ref = _oracle_batch(jobs, *cat)
    arrs = [to_dev(x) for x in cat]
    cap = len(ref[0]) + 1000
    factors, tiles, grids = (0.35, 0.5, 0.7, 1.0, 1.4, 2.0, 2.8), (256, 512, 1024, 2048), (1, 2, 4, 8)
    n = 0
    for f in factors:
        for t in tiles:
            for g in grids:
                tu = {"zone_height_factor": f, "batch_tile": t, "batch_blocks_per_cu": g}
                k, s, c = _run(hlc, jobs, arrs, 0, cap, tu)
                _compare(k, s, c, ref, f"fp32 {tu}")
                st = hlc.last_stats()
                assert (st["batch_tile"], st["batch_blocks_per_cu"]) == (t, g)
                n += 1
    # the FP64 filter over each knob's candidates, the others at their defaults
    for tu in ([{"zone_height_factor": f} for f in factors] + [{"batch_tile": t} for t in tiles] +
               [{"batch_blocks_per_cu": g} for g in grids]):
        k, s, c = _run(hlc, jobs, arrs, 1, cap, tu)
        _compare(k, s, c, ref, f"fp64 {tu}")
        n += 1
    for prec in (0, 1):
        k, s, c = _run(hlc, jobs, arrs, prec, cap, None)
        _compare(k, s, c, ref, f"autotuned prec={prec}")
        st = hlc.last_stats()
        assert st["zone_height_arcsec"] in factors and st["batch_tile"] in tiles
        assert st["batch_blocks_per_cu"] in grids
        print("autotuned", prec, st["zone_height_arcsec"], st["batch_tile"], st["batch_blocks_per_cu"], flush=True)
    print("configurations compared with the oracle:", n + 2, flush=True)


def test_batch_tuning_errors(hlc):
    jobs, cat = _mixed_batch()
    arrs = [to_dev(x) for x in cat]
    import torch
    out = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(16, dtype=torch.float64, device="cuda")
    for tu in ({"batch_tile": 300}, {"batch_blocks_per_cu": 9}, {"batch_blocks_per_cu": -1}):
        st, _ = hlc.hlc_xmatch_batch(jobs, *arrs, out, sep, tuning=tu)
        assert st == hlc.HLC_E_INVAL, tu


def test_batch_graph_replay(hlc):
    """Replays of the captured graph, with eager work in between, match the first result."""
    import torch
    jobs, cat = _mixed_batch()
    ref = _oracle_batch(jobs, *cat)
    arrs = [to_dev(x) for x in cat]
    cap = len(ref[0]) + 1000
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(cap, dtype=torch.float64, device="cuda")
    cnt = torch.empty(len(jobs), dtype=torch.int64, device="cuda")
    c = synth.patch_pair(scale=0.05)
    for rep in range(4):
        out.fill_(-1)
        sep.fill_(-1.0)
        cnt.fill_(-7)
        st, n = hlc.hlc_xmatch_batch(jobs, *arrs, out, sep, cnt, precision=0,
                                     tuning={"zone_height_factor": 1.0})
        assert st == hlc.HLC_OK
        p = out[:n].cpu().numpy().view(np.uint32).reshape(-1, 2)
        k = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
        _compare(k, sep[:n].cpu().numpy(), cnt.cpu().numpy(), ref, f"replay {rep}")
        # eager work on the same stream and device between replays
        hlc.xmatch(to_dev(c.a_ra), to_dev(c.a_dec), to_dev(c.b_ra), to_dev(c.b_dec), 1.0)
        torch.cuda.synchronize()


def test_batch_errors(hlc):
    import torch
    g = synth.rng(500, 0)
    ra, dec = synth.uniform_patch(g, 1000, 0, 1, 0, 1)
    out = torch.empty((10, 2), dtype=torch.int32, device="cuda")
    sep = torch.empty(10, dtype=torch.float64, device="cuda")
    args = [to_dev(ra), to_dev(dec), to_dev(ra), to_dev(dec)]
    st, _ = hlc.hlc_xmatch_batch([(0, 1000, 0, 1000, 0.0)], *args, out, sep)
    assert st == hlc.HLC_E_INVAL
    st, _ = hlc.hlc_xmatch_batch([(0, 1000, 0, 1000, 4000.0)], *args, out, sep)
    assert st == hlc.HLC_E_INVAL
    bad = dec.copy()
    bad[500] = float("nan")
    st, _ = hlc.hlc_xmatch_batch([(0, 1000, 0, 1000, 1.0)], to_dev(ra), to_dev(bad), to_dev(ra), to_dev(dec),
                                 out, sep)
    assert st == hlc.HLC_E_INVAL
    st, n = hlc.hlc_xmatch_batch([], *args, out, sep)
    assert st == hlc.HLC_OK and n == 0
    # overflow reports the required count
    st, n = hlc.hlc_xmatch_batch([(0, 1000, 0, 1000, 3600.0)], *args, out, sep)
    assert st == hlc.HLC_E_OVERFLOW and n > 10


@pytest.mark.timeout(900)
def test_batch_10k_jobs(hlc):
    """The batched workload at full size: 10,000 jobs, every pair of every job compared."""
    import time
    t0 = time.time()
    b = synth.batch_jobs()
    print(f"generated {b.njobs} jobs, {len(b.a_ra)} + {len(b.b_ra)} sources in {time.time() - t0:.1f}s",
          flush=True)
    jobs = [(int(b.a_off[j]), int(b.na[j]), int(b.b_off[j]), int(b.nb[j]), float(b.r_arcsec[j]))
            for j in range(b.njobs)]
    t0 = time.time()
    ref = _oracle_batch(jobs, b.a_ra, b.a_dec, b.b_ra, b.b_dec)
    print(f"oracle {len(ref[0])} pairs in {time.time() - t0:.1f}s", flush=True)
    arrs = [to_dev(x) for x in (b.a_ra, b.a_dec, b.b_ra, b.b_dec)]
    for prec in (0, 1):
        k, s, c = _run(hlc, jobs, arrs, prec, len(ref[0]) + 10000)
        _compare(k, s, c, ref, f"10k prec={prec}")
        print("batch", prec, hlc.last_stats(), flush=True)
