"""Python binding of libhlc, the gfx950 positional cross-match library.

Argument marshalling only: every step of the cross-match runs in the HIP
kernels of ``libhlc.so`` (see ``include/hlc.h`` for the C ABI). PyTorch is
used for device memory and the current HIP stream. There is no CPU fallback:
if the library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhlc.so")

HLC_OK, HLC_E_INVAL, HLC_E_NOMEM, HLC_E_OVERFLOW, HLC_E_DEVICE, HLC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
HLC_FP32_RECHECK, HLC_FP64 = 0, 1
HLC_NO_SEP, HLC_PROFILE, HLC_SORTED, HLC_SELF, HLC_TIME_FILTER = 0x1, 0x2, 0x4, 0x8, 0x10

EXPORTS = ["hlc_xmatch", "hlc_xmatch_noalloc", "hlc_xmatch_radii", "hlc_xmatch_quad", "hlc_partition", "hlc_part_free", "hlc_xmatch_part", "hlc_xmatch_batch",
           "hlc_xmatch_stream", "hlc_transfer_model", "hlc_strerror", "hlc_last_stats", "hlc_shutdown"]


class hlc_tuning(C.Structure):
    _fields_ = [("zone_height_arcsec", C.c_double), ("ra_bins_log2", C.c_int32),
                ("filter_items", C.c_int32), ("zone_height_factor", C.c_double),
                ("fraction_sort", C.c_int32), ("batch_tile", C.c_int32), ("batch_blocks_per_cu", C.c_int32),
                ("reserved", C.c_int32 * 1)]


class hlc_opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("stream", C.c_void_p), ("capacity", C.c_int64),
                ("n_pairs", C.POINTER(C.c_int64)), ("flags", C.c_uint32),
                ("tuning", C.POINTER(hlc_tuning))]


class hlc_stats(C.Structure):
    _fields_ = [("na", C.c_int64), ("nb", C.c_int64), ("nb_halo", C.c_int64), ("n_pairs", C.c_int64),
                ("n_candidates", C.c_int64), ("n_band", C.c_int64), ("n_ties", C.c_int64),
                ("n_zones", C.c_int32), ("ra_bits", C.c_int32), ("zone_height_arcsec", C.c_double),
                ("t_keygen_ms", C.c_double), ("t_sort_ms", C.c_double), ("t_layout_ms", C.c_double),
                ("t_ranges_ms", C.c_double), ("t_match_ms", C.c_double), ("t_certify_ms", C.c_double),
                ("t_total_ms", C.c_double), ("batch_tile", C.c_double), ("batch_blocks_per_cu", C.c_double),
                ("reserved", C.c_double * 6)]


class hlc_job(C.Structure):
    _fields_ = [("a_off", C.c_int64), ("na", C.c_int64), ("b_off", C.c_int64), ("nb", C.c_int64),
                ("r_arcsec", C.c_double)]


class hlc_transfer(C.Structure):
    _fields_ = [("alpha_h2d", C.c_double), ("beta_h2d", C.c_double), ("alpha_d2h", C.c_double),
                ("beta_d2h", C.c_double), ("r2_h2d", C.c_double), ("r2_d2h", C.c_double)]


SINK = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p)

_lib = None


class HLCError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})" if what else f"{strerror(status)} ({status})")


def load() -> C.CDLL:
    """Load libhlc.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        lib.hlc_xmatch.restype = C.c_int
        lib.hlc_xmatch.argtypes = [vp, vp, i64, vp, vp, i64, C.c_double, vp, vp, C.POINTER(hlc_opts)]
        lib.hlc_xmatch_noalloc.restype = C.c_int
        lib.hlc_xmatch_noalloc.argtypes = [vp, vp, i64, vp, vp, i64, C.c_double, vp, vp, C.POINTER(hlc_opts)]
        lib.hlc_xmatch_radii.restype = C.c_int
        lib.hlc_xmatch_radii.argtypes = [vp, vp, vp, i64, vp, vp, vp, i64, C.c_double, vp, vp,
                                         C.POINTER(hlc_opts)]
        lib.hlc_xmatch_quad.restype = C.c_int
        lib.hlc_xmatch_quad.argtypes = [vp, vp, i64, vp, vp, i64, C.c_double, C.c_int32, vp, vp,
                                        C.POINTER(hlc_opts)]
        lib.hlc_partition.restype = C.c_int
        lib.hlc_partition.argtypes = [vp, vp, i64, C.c_double, C.POINTER(hlc_opts), C.POINTER(vp)]
        lib.hlc_part_free.restype = None
        lib.hlc_part_free.argtypes = [vp]
        lib.hlc_xmatch_part.restype = C.c_int
        lib.hlc_xmatch_part.argtypes = [vp, vp, C.c_double, vp, vp, C.POINTER(hlc_opts)]
        lib.hlc_xmatch_batch.restype = C.c_int
        lib.hlc_xmatch_batch.argtypes = [C.POINTER(hlc_job), C.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                         C.POINTER(hlc_opts)]
        lib.hlc_xmatch_stream.restype = C.c_int
        lib.hlc_xmatch_stream.argtypes = [vp, vp, i64, vp, vp, i64, C.c_double, SINK, vp,
                                          C.POINTER(hlc_opts)]
        lib.hlc_transfer_model.restype = C.c_int
        lib.hlc_transfer_model.argtypes = [C.POINTER(hlc_transfer)]
        lib.hlc_strerror.restype = C.c_char_p
        lib.hlc_strerror.argtypes = [C.c_int]
        lib.hlc_last_stats.restype = C.c_int
        lib.hlc_last_stats.argtypes = [C.POINTER(hlc_stats)]
        lib.hlc_shutdown.restype = None
        lib.hlc_shutdown.argtypes = []
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    try:
        return load().hlc_strerror(int(status)).decode()
    except Exception:  # library not built
        return f"status {status}"


def _ptr(t) -> int:
    if t is None:
        return 0
    return int(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _check_coords(*ts):
    import torch
    for t in ts:
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == 1):
            raise ValueError("coordinates must be contiguous 1-D float64 CUDA tensors")


def make_opts(precision=HLC_FP32_RECHECK, capacity=0, stream=None, flags=0, tuning=None):
    n = C.c_int64(0)
    o = hlc_opts()
    o.precision = int(precision)
    o.stream = _stream_handle(stream)
    o.capacity = int(capacity)
    o.n_pairs = C.pointer(n)
    o.flags = int(flags)
    tu = None
    if tuning:
        tu = hlc_tuning()
        tu.zone_height_arcsec = float(tuning.get("zone_height_arcsec", 0.0))
        tu.ra_bins_log2 = int(tuning.get("ra_bins_log2", 0))
        tu.filter_items = int(tuning.get("filter_items", 0))
        tu.zone_height_factor = float(tuning.get("zone_height_factor", 0.0))
        tu.fraction_sort = int(tuning.get("fraction_sort", 0))
        tu.batch_tile = int(tuning.get("batch_tile", 0))
        tu.batch_blocks_per_cu = int(tuning.get("batch_blocks_per_cu", 0))
        o.tuning = C.pointer(tu)
    return o, n, tu


def hlc_xmatch(a_ra, a_dec, b_ra, b_dec, r_arcsec, out_pairs, out_sep, *, precision=HLC_FP32_RECHECK,
               capacity=None, stream=None, flags=0, tuning=None):
    """Call hlc_xmatch on torch CUDA tensors. Returns (status, n_pairs).

    out_pairs: int32 tensor (capacity, 2); out_sep: float64 (capacity,) or None.
    """
    _check_coords(a_ra, a_dec, b_ra, b_dec)
    if capacity is None:
        capacity = 0 if out_pairs is None else out_pairs.shape[0]
    o, n, tu = make_opts(precision, capacity, stream, flags, tuning)
    st = load().hlc_xmatch(_ptr(a_ra), _ptr(a_dec), a_ra.numel(), _ptr(b_ra), _ptr(b_dec), b_ra.numel(),
                           float(r_arcsec), _ptr(out_pairs), _ptr(out_sep), C.byref(o))
    return st, n.value


def hlc_xmatch_noalloc(a_ra, a_dec, b_ra, b_dec, r_arcsec, out_pairs, out_sep, *, precision=HLC_FP32_RECHECK,
                       capacity=None, stream=None, flags=0, tuning=None):
    """Call hlc_xmatch_noalloc (no allocation inside the library) on torch CUDA
    tensors. Returns (status, n_pairs); arguments as hlc_xmatch."""
    _check_coords(a_ra, a_dec, b_ra, b_dec)
    if capacity is None:
        capacity = 0 if out_pairs is None else out_pairs.shape[0]
    o, n, tu = make_opts(precision, capacity, stream, flags, tuning)
    st = load().hlc_xmatch_noalloc(_ptr(a_ra), _ptr(a_dec), a_ra.numel(), _ptr(b_ra), _ptr(b_dec), b_ra.numel(),
                                   float(r_arcsec), _ptr(out_pairs), _ptr(out_sep), C.byref(o))
    return st, n.value


def xmatch(a_ra, a_dec, b_ra, b_dec, r_arcsec, *, precision=HLC_FP32_RECHECK, capacity=None,
           stream=None, flags=0, tuning=None, want_sep=True):
    """Allocate outputs, call hlc_xmatch, grow and retry once on overflow.

    Returns (pairs[n, 2] int32 CUDA tensor, sep[n] float64 CUDA tensor or None).
    """
    import torch
    dev = a_ra.device
    cap = capacity if capacity is not None else max(1024, (a_ra.numel() + b_ra.numel()) // 2)
    if not want_sep:
        flags |= HLC_NO_SEP
    for _ in range(2):
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        sep = torch.empty(cap, dtype=torch.float64, device=dev) if want_sep else None
        st, n = hlc_xmatch(a_ra, a_dec, b_ra, b_dec, r_arcsec, pairs, sep, precision=precision,
                           capacity=cap, stream=stream, flags=flags, tuning=tuning)
        if st == HLC_E_OVERFLOW:
            cap = int(n * 1.05) + 16
            continue
        if st != HLC_OK:
            raise HLCError(st, "hlc_xmatch")
        return pairs[:n], (sep[:n] if want_sep else None)
    raise HLCError(HLC_E_OVERFLOW, "hlc_xmatch")


def hlc_xmatch_radii(a_ra, a_dec, a_err, b_ra, b_dec, b_err, k_sigma, out_pairs, out_sep, *,
                     precision=HLC_FP32_RECHECK, capacity=None, stream=None, flags=0, tuning=None):
    """Eq. (4) per-source error radii (arcsec). Returns (status, n_pairs)."""
    _check_coords(a_ra, a_dec, a_err, b_ra, b_dec, b_err)
    if capacity is None:
        capacity = 0 if out_pairs is None else out_pairs.shape[0]
    o, n, tu = make_opts(precision, capacity, stream, flags, tuning)
    st = load().hlc_xmatch_radii(_ptr(a_ra), _ptr(a_dec), _ptr(a_err), a_ra.numel(), _ptr(b_ra),
                                 _ptr(b_dec), _ptr(b_err), b_ra.numel(), float(k_sigma), _ptr(out_pairs),
                                 _ptr(out_sep), C.byref(o))
    return st, n.value


def hlc_xmatch_quad(a_ra, a_dec, b_ra, b_dec, r_arcsec, order, out_pairs, out_sep, *, capacity=None,
                    stream=None, flags=0):
    """The paper's HEALPix + quad-direction partition, emulated. Returns (status, n_pairs)."""
    _check_coords(a_ra, a_dec, b_ra, b_dec)
    if capacity is None:
        capacity = 0 if out_pairs is None else out_pairs.shape[0]
    o, n, tu = make_opts(HLC_FP64, capacity, stream, flags, None)
    st = load().hlc_xmatch_quad(_ptr(a_ra), _ptr(a_dec), a_ra.numel(), _ptr(b_ra), _ptr(b_dec), b_ra.numel(),
                                float(r_arcsec), int(order), _ptr(out_pairs), _ptr(out_sep), C.byref(o))
    return st, n.value


class Part:
    """A catalogue partitioned on the device (hlc_partition); free with .free()."""

    def __init__(self, handle, n, r_arcsec):
        self.handle, self.n, self.r_arcsec = handle, n, r_arcsec

    def free(self):
        if self.handle:
            load().hlc_part_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hlc_partition(ra, dec, r_arcsec, *, stream=None, tuning=None):
    """Partition one catalogue for reuse; returns (status, Part or None)."""
    _check_coords(ra, dec)
    o, n, tu = make_opts(HLC_FP64, 0, stream, 0, tuning)
    h = C.c_void_p(0)
    st = load().hlc_partition(_ptr(ra), _ptr(dec), ra.numel(), float(r_arcsec), C.byref(o), C.byref(h))
    return st, (Part(h.value, ra.numel(), r_arcsec) if st == HLC_OK else None)


def hlc_xmatch_part(A: Part, B: Part, r_arcsec, out_pairs, out_sep, *, precision=HLC_FP32_RECHECK,
                    capacity=None, stream=None, flags=0):
    """Cross-match two partitioned catalogues. Returns (status, n_pairs)."""
    if capacity is None:
        capacity = 0 if out_pairs is None else out_pairs.shape[0]
    o, n, tu = make_opts(precision, capacity, stream, flags, None)
    st = load().hlc_xmatch_part(A.handle, B.handle, float(r_arcsec), _ptr(out_pairs), _ptr(out_sep),
                                C.byref(o))
    return st, n.value


def _check_host(*ts):
    import torch
    for t in ts:
        if not (t.device.type == "cpu" and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == 1):
            raise ValueError("streamed coordinates must be contiguous 1-D float64 host tensors (pinned)")


def hlc_xmatch_stream(a_ra, a_dec, b_ra, b_dec, r_arcsec, sink, *, precision=HLC_FP32_RECHECK,
                      ring_pairs=0, stream=None, flags=0):
    """Stream host catalogues (torch CPU tensors, ideally pinned) through the GPU.

    sink(pairs_ptr, sep_ptr, n) is called from the calling thread with host
    pointers to n (a, b) uint32 pairs and n FP64 separations (sep_ptr is None
    with HLC_NO_SEP); it returns 0 to continue. Returns (status, n_pairs).
    """
    _check_host(a_ra, a_dec, b_ra, b_dec)
    o, n, tu = make_opts(precision, ring_pairs, stream, flags, None)
    cb = SINK(lambda p, s_, k, u: int(sink(p, s_, k) or 0))
    st = load().hlc_xmatch_stream(_ptr(a_ra), _ptr(a_dec), a_ra.numel(), _ptr(b_ra), _ptr(b_dec),
                                  b_ra.numel(), float(r_arcsec), cb, None, C.byref(o))
    return st, n.value


def xmatch_stream(a_ra, a_dec, b_ra, b_dec, r_arcsec, **kw):
    """Collect the streamed result into numpy arrays: (pairs[n, 2] uint32, sep[n] float64)."""
    import numpy as np
    parts_p, parts_s = [], []

    def sink(p, s_, k):
        parts_p.append(np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint32)), shape=(k, 2)).copy())
        if s_:
            parts_s.append(np.ctypeslib.as_array(C.cast(s_, C.POINTER(C.c_double)), shape=(k,)).copy())
        return 0

    st, n = hlc_xmatch_stream(a_ra, a_dec, b_ra, b_dec, r_arcsec, sink, **kw)
    if st != HLC_OK:
        raise HLCError(st, "hlc_xmatch_stream")
    pairs = np.concatenate(parts_p) if parts_p else np.empty((0, 2), np.uint32)
    sep = np.concatenate(parts_s) if parts_s else np.empty(0)
    assert len(pairs) == n
    return pairs, sep


def hlc_xmatch_batch(jobs, a_ra, a_dec, b_ra, b_dec, out_pairs, out_sep, job_pair_count=None, *,
                     precision=HLC_FP32_RECHECK, capacity=None, stream=None, flags=0, tuning=None):
    """Batched cross-match. jobs: sequence of (a_off, na, b_off, nb, r_arcsec).

    Coordinates are device tensors holding all jobs; job_pair_count is an
    optional int64 device tensor of len(jobs). Returns (status, n_pairs).
    """
    _check_coords(a_ra, a_dec, b_ra, b_dec)
    tab = job_table(jobs)
    if capacity is None:
        capacity = 0 if out_pairs is None else out_pairs.shape[0]
    o, n, tu = make_opts(precision, capacity, stream, flags, tuning)
    st = load().hlc_xmatch_batch(tab.ctypes.data_as(C.POINTER(hlc_job)), len(tab), _ptr(a_ra), _ptr(a_dec),
                                 _ptr(b_ra), _ptr(b_dec), _ptr(out_pairs), _ptr(out_sep), _ptr(job_pair_count),
                                 C.byref(o))
    return st, n.value


# numpy layout of hlc_job (five 8-byte fields, no padding)
JOB_DTYPE = None


def job_table(jobs):
    """The jobs as a contiguous numpy array laid out as hlc_job.

    jobs: such an array (returned as is), or a sequence of
    (a_off, na, b_off, nb, r_arcsec). A caller that repeats a batch can build
    the table once and pass it on every call.
    """
    import numpy as np
    global JOB_DTYPE
    if JOB_DTYPE is None:
        JOB_DTYPE = np.dtype([(name, "<i8" if ct is C.c_int64 else "<f8") for name, ct in hlc_job._fields_])
        assert JOB_DTYPE.itemsize == C.sizeof(hlc_job)
    if isinstance(jobs, np.ndarray) and jobs.dtype == JOB_DTYPE and jobs.flags.c_contiguous:
        return jobs
    return np.array([tuple(j) for j in jobs], dtype=JOB_DTYPE) if len(jobs) else np.zeros(1, JOB_DTYPE)[:0]


def transfer_model() -> dict:
    """The eq. (5) host<->device model fitted on this device: alpha (s), beta (s/byte)."""
    t = hlc_transfer()
    st = load().hlc_transfer_model(C.byref(t))
    if st != HLC_OK:
        raise HLCError(st, "hlc_transfer_model")
    return {k: getattr(t, k) for k, _ in hlc_transfer._fields_}


def last_stats() -> dict:
    s = hlc_stats()
    st = load().hlc_last_stats(C.byref(s))
    if st != HLC_OK:
        raise HLCError(st, "hlc_last_stats")
    return {name: (getattr(s, name) if not isinstance(getattr(s, name), C.Array) else None)
            for name, _ in hlc_stats._fields_ if name != "reserved"}


def shutdown() -> None:
    load().hlc_shutdown()
