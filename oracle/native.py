"""ctypes binding of the C part of the oracle (oracle/csrc/oracle.c)."""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        i64, p, dbl = C.c_int64, C.c_void_p, C.c_double
        L.orc_num_steps.argtypes = [i64, i64, i64]
        L.orc_num_steps.restype = i64
        L.orc_num_reflectors.argtypes = [i64, i64]
        L.orc_num_reflectors.restype = i64
        L.orc_larfg_d.argtypes = [i64, p, p, p]
        L.orc_larfg_z.argtypes = [i64, p, p, p]
        for nm in ("orc_band_to_tridiag_d", "orc_band_to_tridiag_z"):
            getattr(L, nm).argtypes = [i64, i64, p, i64, p, p, p, p]
            getattr(L, nm).restype = C.c_int
        for nm in ("orc_bt1_d", "orc_bt1_z"):
            getattr(L, nm).argtypes = [i64, i64, i64, p, p, p, i64, C.c_int]
            getattr(L, nm).restype = C.c_int
        L.orc_sturm_count.argtypes = [i64, p, p, dbl, dbl]
        L.orc_sturm_count.restype = i64
        L.orc_tridiag_bisect.argtypes = [i64, p, p, i64, i64, p, C.c_int]
        L.orc_tridiag_bisect.restype = C.c_int
        L.orc_tridiag_invit.argtypes = [i64, p, p, i64, p, p, i64, C.c_uint64, C.c_int]
        L.orc_tridiag_invit.restype = C.c_int
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)
