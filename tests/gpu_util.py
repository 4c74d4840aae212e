"""Helpers for the GPU parity tests: run the HIP path, compare with the oracle."""
from __future__ import annotations

import numpy as np

SEP_TOL_ARCSEC = 1e-9  # separations must agree with the FP64 oracle within this


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def gpu_xmatch(a_ra, a_dec, b_ra, b_dec, r, precision, tuning=None, want_sep=True):
    """Run the library; return pair keys (a<<32|b, sorted) and matching seps."""
    import paper_2301_07331_amd as hlc
    pairs, sep = hlc.xmatch(to_dev(a_ra), to_dev(a_dec), to_dev(b_ra), to_dev(b_dec), r,
                            precision=precision, tuning=tuning, want_sep=want_sep)
    p = pairs.cpu().numpy().view(np.uint32).reshape(-1, 2)
    keys = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    order = np.argsort(keys, kind="stable")
    s = sep.cpu().numpy()[order] if want_sep else None
    return keys[order], s


def assert_same(keys, sep, ref, tol=SEP_TOL_ARCSEC, label=""):
    """Bit-exact pair set and |sep - sep_oracle| <= tol (arcsec)."""
    rk = ref.keys()
    assert len(np.unique(keys)) == len(keys), f"{label}: duplicate pairs"
    if len(keys) != len(rk) or not np.array_equal(keys, rk):
        extra = np.setdiff1d(keys, rk)
        missing = np.setdiff1d(rk, keys)
        raise AssertionError(f"{label}: {len(keys)} vs oracle {len(rk)}; extra {len(extra)} "
                             f"e.g. {[(int(k >> 32), int(k & 0xffffffff)) for k in extra[:5]]}; "
                             f"missing {len(missing)} e.g. "
                             f"{[(int(k >> 32), int(k & 0xffffffff)) for k in missing[:5]]}")
    if sep is not None and len(sep):
        err = np.abs(sep - ref.sep)
        assert err.max() <= tol, f"{label}: max |dsep| = {err.max():.3e} arcsec"
    return len(keys)


def sorted_on_gpu(pairs, sep):
    """Pair keys (a << 32 | b) sorted on the GPU, with the separations in the
    same order, both returned as numpy (for results of 1e8 pairs and more).
    pairs: (n, 2) uint32 numpy array or an (n, 2) int32 device tensor."""
    import torch
    if isinstance(pairs, np.ndarray):
        p = torch.from_numpy(pairs.view(np.int32)).to("cuda")
    else:
        p = pairs
    a = p[:, 0].to(torch.int64) & 0xFFFFFFFF
    b = p[:, 1].to(torch.int64) & 0xFFFFFFFF
    keys = (a << 32) | b
    del a, b
    k, order = torch.sort(keys)
    del keys
    s = torch.as_tensor(sep).to("cuda")[order] if sep is not None else None
    out_k = k.cpu().numpy().view(np.uint64)
    out_s = s.cpu().numpy() if s is not None else None
    del k, order, s
    torch.cuda.empty_cache()
    return out_k, out_s


def assert_same_sorted(keys, sep, ref_keys, ref_sep, tol=SEP_TOL_ARCSEC, label=""):
    """assert_same for large results whose keys are already sorted (linear-time checks)."""
    assert len(keys) < 2 or not np.any(keys[1:] == keys[:-1]), f"{label}: duplicate pairs"
    if len(keys) != len(ref_keys) or not np.array_equal(keys, ref_keys):
        extra = np.setdiff1d(keys, ref_keys)
        missing = np.setdiff1d(ref_keys, keys)
        raise AssertionError(f"{label}: {len(keys)} vs oracle {len(ref_keys)}; extra {len(extra)} "
                             f"e.g. {[(int(k >> 32), int(k & 0xffffffff)) for k in extra[:5]]}; "
                             f"missing {len(missing)} e.g. "
                             f"{[(int(k >> 32), int(k & 0xffffffff)) for k in missing[:5]]}")
    if sep is not None and len(sep):
        err = float(np.max(np.abs(sep - ref_sep)))
        assert err <= tol, f"{label}: max |dsep| = {err:.3e} arcsec"
    return len(keys)
