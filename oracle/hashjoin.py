"""ctypes wrapper of the oracle's C hash join (test infrastructure only).

``build()`` compiles ``hashjoin.c`` with gcc into ``liboracle_hashjoin.so``
next to it; the GPU product never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "hashjoin.c")
LIB = os.path.join(_HERE, "liboracle_hashjoin.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_hj_count.argtypes = [i32p, ctypes.c_int64, i32p, ctypes.c_int64, ctypes.c_int]
        lib.oracle_hj_count.restype = ctypes.c_int64
        lib.oracle_hj_pairs.argtypes = [i32p, ctypes.c_int64, i32p, ctypes.c_int64, i64p, i64p,
                                        ctypes.c_int64, ctypes.c_int]
        lib.oracle_hj_pairs.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def hj_count(probe_keys: np.ndarray, build_keys: np.ndarray, nthreads: int = 0) -> int:
    pk = np.ascontiguousarray(probe_keys, dtype=np.int32)
    bk = np.ascontiguousarray(build_keys, dtype=np.int32)
    r = _load().oracle_hj_count(_p32(pk), pk.size, _p32(bk), bk.size, nthreads)
    if r < 0:
        raise MemoryError("oracle hash join: allocation failed")
    return int(r)


def hj_pairs(probe_keys: np.ndarray, build_keys: np.ndarray, nthreads: int = 0):
    """All (probe row, build row) index pairs with equal keys."""
    pk = np.ascontiguousarray(probe_keys, dtype=np.int32)
    bk = np.ascontiguousarray(build_keys, dtype=np.int32)
    n = hj_count(pk, bk, nthreads)
    a = np.empty(max(n, 1), dtype=np.int64)
    b = np.empty(max(n, 1), dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    r = _load().oracle_hj_pairs(_p32(pk), pk.size, _p32(bk), bk.size, a.ctypes.data_as(i64p),
                                b.ctypes.data_as(i64p), n, nthreads)
    if r != n:
        raise RuntimeError(f"oracle hash join: {r} != {n}")
    return a[:n], b[:n]
