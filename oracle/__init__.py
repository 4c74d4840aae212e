"""CPU oracle for the positional cross-match (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never does, and this
package imports nothing from it: the two share no code.

The arithmetic lives in ``oracle.cpp`` (a plain FP64 zone join with a
binary128 certificate near the threshold, plus a brute-force all-pairs entry
point); this module only builds and loads it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OUT, IN_FP64, IN_QUAD, IN_TIE, OUT_QUAD = 0, 1, 2, 3, 4

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP, libquadmath)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["g++", "-O2", "-std=gnu++17", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lquadmath"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.oracle_pair.restype = C.c_int
        lib.oracle_pair.argtypes = [C.c_double] * 5 + [dp]
        lib.oracle_pair_q.restype = C.c_int
        lib.oracle_pair_q.argtypes = [C.c_double] * 5
        lib.oracle_sep_q.restype = C.c_double
        lib.oracle_sep_q.argtypes = [C.c_double] * 4
        for name in ("oracle_xmatch",):
            f = getattr(lib, name)
            f.restype = C.c_void_p
            f.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                          C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int)]
        lib.oracle_xmatch_radii.restype = C.c_void_p
        lib.oracle_xmatch_radii.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_int, C.c_int,
                                            C.POINTER(C.c_int)]
        lib.oracle_hp_nest.restype = C.c_int64
        lib.oracle_hp_nest.argtypes = [C.c_int, C.c_double, C.c_double]
        lib.oracle_quad_direction.restype = C.c_void_p
        lib.oracle_quad_direction.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                              C.c_int64, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int)]
        lib.oracle_brute.restype = C.c_void_p
        lib.oracle_brute.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_int64, C.c_double, C.c_int, C.POINTER(C.c_int)]
        lib.oracle_result_size.restype = C.c_int64
        lib.oracle_result_size.argtypes = [C.c_void_p]
        lib.oracle_result_copy.restype = None
        lib.oracle_result_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_result_stats.restype = None
        lib.oracle_result_stats.argtypes = [C.c_void_p, C.c_void_p]
        lib.oracle_result_free.restype = None
        lib.oracle_result_free.argtypes = [C.c_void_p]
        _lib = lib
    return _lib


class OracleError(ValueError):
    pass


class Result:
    """Pairs sorted by (a, b) unless the call asked otherwise."""

    def __init__(self, a, b, sep, stats, seconds):
        self.a, self.b, self.sep = a, b, sep
        self.candidates, self.band, self.ties = (int(x) for x in stats)
        self.seconds = seconds

    def __len__(self):
        return len(self.a)

    def keys(self) -> np.ndarray:
        """(a << 32) | b as uint64, the canonical pair identity."""
        return (self.a.astype(np.uint64) << np.uint64(32)) | self.b.astype(np.uint64)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _collect(lib, h, t0):
    n = lib.oracle_result_size(h)
    a = np.empty(n, np.uint32)
    b = np.empty(n, np.uint32)
    s = np.empty(n, np.float64)
    st = np.zeros(3, np.int64)
    lib.oracle_result_copy(h, a.ctypes.data, b.ctypes.data, s.ctypes.data)
    lib.oracle_result_stats(h, st.ctypes.data)
    lib.oracle_result_free(h)
    return Result(a, b, s, st, time.perf_counter() - t0)


def xmatch(a_ra, a_dec, b_ra, b_dec, r_arcsec: float, nthreads: int = 0, sort: bool = True) -> Result:
    """Zone-join oracle: every (i, j) with separation <= r_arcsec, FP64 seps in arcsec."""
    lib = _load()
    a_ra, a_dec, b_ra, b_dec = map(_f64, (a_ra, a_dec, b_ra, b_dec))
    st = C.c_int(0)
    t0 = time.perf_counter()
    h = lib.oracle_xmatch(a_ra.ctypes.data, a_dec.ctypes.data, len(a_ra), b_ra.ctypes.data,
                          b_dec.ctypes.data, len(b_ra), float(r_arcsec), int(nthreads),
                          1 if sort else 0, C.byref(st))
    if st.value != 0 or not h:
        raise OracleError("invalid input")
    return _collect(lib, h, t0)


def brute(a_ra, a_dec, b_ra, b_dec, r_arcsec: float, nthreads: int = 0) -> Result:
    """All m*n pairs through the same decision (small inputs only)."""
    lib = _load()
    a_ra, a_dec, b_ra, b_dec = map(_f64, (a_ra, a_dec, b_ra, b_dec))
    st = C.c_int(0)
    t0 = time.perf_counter()
    h = lib.oracle_brute(a_ra.ctypes.data, a_dec.ctypes.data, len(a_ra), b_ra.ctypes.data,
                         b_dec.ctypes.data, len(b_ra), float(r_arcsec), int(nthreads), C.byref(st))
    if st.value != 0 or not h:
        raise OracleError("invalid input")
    return _collect(lib, h, t0)


def xmatch_radii(a_ra, a_dec, a_err, b_ra, b_dec, b_err, k: float = 3.0, nthreads: int = 0,
                 brute: bool = False) -> Result:
    """Eq. (4) with per-source error radii: theta <= k sqrt(ea^2 + eb^2) arcsec."""
    lib = _load()
    a_ra, a_dec, a_err, b_ra, b_dec, b_err = map(_f64, (a_ra, a_dec, a_err, b_ra, b_dec, b_err))
    st = C.c_int(0)
    t0 = time.perf_counter()
    h = lib.oracle_xmatch_radii(a_ra.ctypes.data, a_dec.ctypes.data, a_err.ctypes.data, len(a_ra),
                                b_ra.ctypes.data, b_dec.ctypes.data, b_err.ctypes.data, len(b_ra), float(k),
                                int(nthreads), 1 if brute else 0, C.byref(st))
    if st.value != 0 or not h:
        raise OracleError("invalid input")
    return _collect(lib, h, t0)


def hp_nest(order: int, ra: float, dec: float) -> int:
    """HEALPix nested pixel index at Nside = 2**order."""
    return int(_load().oracle_hp_nest(int(order), float(ra), float(dec)))


def quad_direction(a_ra, a_dec, b_ra, b_dec, r_arcsec: float, order: int, nthreads: int = 0) -> Result:
    """Pairs found by the emulated paper partition (HEALPix + quad-direction copies)."""
    lib = _load()
    a_ra, a_dec, b_ra, b_dec = map(_f64, (a_ra, a_dec, b_ra, b_dec))
    st = C.c_int(0)
    t0 = time.perf_counter()
    h = lib.oracle_quad_direction(a_ra.ctypes.data, a_dec.ctypes.data, len(a_ra), b_ra.ctypes.data,
                                  b_dec.ctypes.data, len(b_ra), float(r_arcsec), int(order), int(nthreads),
                                  C.byref(st))
    if st.value != 0 or not h:
        raise OracleError("invalid input")
    return _collect(lib, h, t0)


def pair(ra1, dec1, ra2, dec2, r_arcsec):
    """(outcome code, separation arcsec or nan) for one pair."""
    lib = _load()
    s = C.c_double(float("nan"))
    k = lib.oracle_pair(float(ra1), float(dec1), float(ra2), float(dec2), float(r_arcsec), C.byref(s))
    if k < 0:
        raise OracleError("invalid input")
    return k, s.value


def pair_q(ra1, dec1, ra2, dec2, r_arcsec) -> bool:
    """Decision evaluated in binary128 only."""
    return bool(_load().oracle_pair_q(float(ra1), float(dec1), float(ra2), float(dec2), float(r_arcsec)))


def sep_q(ra1, dec1, ra2, dec2) -> float:
    """Separation in arcsec evaluated in binary128, rounded once."""
    return _load().oracle_sep_q(float(ra1), float(dec1), float(ra2), float(dec2))
