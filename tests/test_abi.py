"""The C ABI library builds, loads and exports what include/hlc.h declares (no GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hlc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(hlc_[a-z_]+)\s*\(", text))
    # typedef'd function-pointer types are not exports
    names -= {n for n in re.findall(r"\(\*\s*(hlc_[a-z_]+)\)", text)}
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_2301_07331_amd as hlc
    if not os.path.exists(hlc.LIB_PATH):
        from paper_2301_07331_amd import build_lib
        build_lib.build()
    return hlc.load()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("hlc_xmatch", "hlc_partition", "hlc_part_free", "hlc_xmatch_part", "hlc_xmatch_batch",
              "hlc_xmatch_stream", "hlc_strerror", "hlc_last_stats", "hlc_shutdown"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2301_07331_amd as hlc
    out = subprocess.run(["nm", "-D", "--defined-only", hlc.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\S+)$", out, flags=re.M))
    for n in _declared_functions():
        assert n in exported, n
        assert hasattr(lib, n)


def test_strerror_strings(lib):
    import paper_2301_07331_amd as hlc
    for st in (hlc.HLC_OK, hlc.HLC_E_INVAL, hlc.HLC_E_NOMEM, hlc.HLC_E_OVERFLOW, hlc.HLC_E_DEVICE,
               hlc.HLC_E_UNSUPPORTED):
        s = lib.hlc_strerror(st).decode()
        assert s and s != "unknown status"
    assert lib.hlc_strerror(12345).decode() == "unknown status"


def test_argument_errors_are_caught_before_any_device_call(lib):
    """Bad scalar arguments return HLC_E_INVAL without touching a GPU."""
    import paper_2301_07331_amd as hlc
    n = C.c_int64(0)
    o = hlc.hlc_opts()
    o.precision = hlc.HLC_FP64
    o.capacity = 0
    o.n_pairs = C.pointer(n)
    fake = 0x1000  # never dereferenced: the checks fail first
    # NULL opts
    assert lib.hlc_xmatch(fake, fake, 1, fake, fake, 1, 1.0, fake, fake, None) == hlc.HLC_E_INVAL
    for r in (0.0, -1.0, float("nan"), 3600.001, float("inf")):
        assert lib.hlc_xmatch(fake, fake, 1, fake, fake, 1, r, fake, fake, C.byref(o)) == hlc.HLC_E_INVAL
    big = (1 << 31) - (1 << 16) + 1  # one above the largest catalogue
    for na, nb in ((-1, 1), (1, -1), (1 << 31, 1), (1, 1 << 31), (big, 1), (1, big)):
        assert lib.hlc_xmatch(fake, fake, na, fake, fake, nb, 1.0, fake, fake, C.byref(o)) == hlc.HLC_E_INVAL
    o.capacity = -5
    assert lib.hlc_xmatch(fake, fake, 1, fake, fake, 1, 1.0, fake, fake, C.byref(o)) == hlc.HLC_E_INVAL
    o.capacity = 10
    o.precision = 7
    assert lib.hlc_xmatch(fake, fake, 1, fake, fake, 1, 1.0, fake, fake, C.byref(o)) == hlc.HLC_E_INVAL
    o.precision = hlc.HLC_FP64
    # missing output buffers with capacity > 0
    assert lib.hlc_xmatch(fake, fake, 1, fake, fake, 1, 1.0, None, fake, C.byref(o)) == hlc.HLC_E_INVAL
    assert lib.hlc_xmatch(fake, fake, 1, fake, fake, 1, 1.0, fake, None, C.byref(o)) == hlc.HLC_E_INVAL
    # missing coordinates with n > 0
    assert lib.hlc_xmatch(None, fake, 1, fake, fake, 1, 1.0, fake, fake, C.byref(o)) == hlc.HLC_E_INVAL
    # a sorted order cannot be given for pairs that are handed over per chunk
    o.flags = hlc.HLC_SORTED
    sink = hlc.SINK(lambda p, s_, n, u: 0)
    assert lib.hlc_xmatch_stream(fake, fake, 1, fake, fake, 1, 1.0, sink, None, C.byref(o)) == hlc.HLC_E_UNSUPPORTED
    assert lib.hlc_last_stats(None) == hlc.HLC_E_INVAL


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2301_07331_amd as hlc
    x = torch.zeros(4, dtype=torch.float64)
    with pytest.raises(ValueError):
        hlc.hlc_xmatch(x, x, x, x, 1.0, None, None)


def test_job_table_layout_matches_hlc_job():
    """The numpy job table the batched binding passes is byte-for-byte hlc_job."""
    import numpy as np
    import paper_2301_07331_amd as hlc
    jobs = [(0, 10, 5, 20, 1.5), (10, 0, 25, 3, 0.25), ((1 << 31) - 2, 1, 0, 1, 3600.0)]
    t = hlc.job_table(jobs)
    assert t.dtype.itemsize == C.sizeof(hlc.hlc_job) and t.flags.c_contiguous and len(t) == 3
    for name, _ in hlc.hlc_job._fields_:
        assert t.dtype.fields[name][1] == getattr(hlc.hlc_job, name).offset
    arr = (hlc.hlc_job * 3).from_buffer_copy(t.tobytes())
    for k, (ao, na, bo, nb, r) in enumerate(jobs):
        assert (arr[k].a_off, arr[k].na, arr[k].b_off, arr[k].nb, arr[k].r_arcsec) == (ao, na, bo, nb, r)
    assert hlc.job_table(t) is t  # a prebuilt table is passed as is
    assert len(hlc.job_table([])) == 0
    assert np.array_equal(hlc.job_table(list(t)), t)
