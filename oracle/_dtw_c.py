"""ctypes loader for the oracle's C DTW (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        lib = ctypes.CDLL(build_oracle.LIB)
        lib.oracle_dtw.restype = ctypes.c_double
        lib.oracle_dtw.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_int64]
        lib.oracle_num_threads.restype = ctypes.c_int32
        lib.oracle_num_threads.argtypes = []
        lib.oracle_dtw_pairs.restype = None
        lib.oracle_dtw_pairs.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] + \
            [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_float, ctypes.c_void_p]
        _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def dtw(q, x, r: int) -> float:
    q = _f32(q)
    x = _f32(x)
    return _load().oracle_dtw(q.ctypes.data, q.shape[0], x.ctypes.data, x.shape[0], int(r))


def dtw_pairs(q, q_off, db, db_off, cand, ncand, band_frac: float) -> np.ndarray:
    """float64 [nq, C] distances; entries past ncand[i] are left at +inf."""
    q = _f32(q)
    db = _f32(db)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    db_off = np.ascontiguousarray(db_off, dtype=np.int64)
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    ncand = np.ascontiguousarray(ncand, dtype=np.int32)
    nq, C = cand.shape
    out = np.full((nq, C), np.inf)
    _load().oracle_dtw_pairs(q.ctypes.data, q_off.ctypes.data, nq, db.ctypes.data,
                             db_off.ctypes.data, cand.ctypes.data, ncand.ctypes.data, C,
                             float(band_frac), out.ctypes.data)
    return out


def num_threads() -> int:
    """Threads the OpenMP pair loop runs on."""
    return int(_load().oracle_num_threads())
