"""ctypes front end of the C oracle (test infrastructure only).

Inputs and outputs are canonical field elements as uint32[..][8]
little-endian limbs, the same byte layout as 4 x uint64.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.zco_degree.restype = ctypes.c_int
        lib.zco_degree.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.zco_prove.restype = ctypes.c_int
        lib.zco_prove.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.zco_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return load().zco_max_threads()


def degree(gate, m):
    d = load().zco_degree(gate, m)
    if d < 0:
        raise ValueError(f"unknown gate {gate}, m={m}")
    return d


def prove(mu, gate, m, tables: np.ndarray, r: np.ndarray, nthreads: int = 0):
    """tables uint32[k][2^mu][8], r uint32[mu][8] canonical -> dict of uint32 arrays."""
    lib = load()
    d = degree(gate, m)
    k = tables.shape[0]
    tables = np.ascontiguousarray(tables, dtype=np.uint32)
    r = np.ascontiguousarray(r, dtype=np.uint32)
    evals = np.zeros((mu, d + 2, 8), np.uint32)
    alphas = np.zeros((mu, 8), np.uint32)
    openings = np.zeros((k + 1, 8), np.uint32)
    rc = lib.zco_prove(mu, gate, m, tables.ctypes.data, r.ctypes.data, evals.ctypes.data,
                       alphas.ctypes.data, openings.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError(f"C oracle returned {rc}")
    return {"evals": evals, "alphas": alphas, "openings": openings}
