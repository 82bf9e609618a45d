"""Build and load the oracle's plain C arithmetic (ref_arith.c) with gcc.

Test infrastructure only.  The shared object is built next to the source the
first time it is needed (or by ``build()``) and loaded with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ref_arith.c")
_LIB = os.path.join(_HERE, "liboracle_ref.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ref_arith.c into liboracle_ref.so (gcc -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB)
            u64, sz, p = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p
            L.oracle_mulmod.restype = u64
            L.oracle_mulmod.argtypes = [u64, u64, u64]
            L.oracle_powmod.restype = u64
            L.oracle_powmod.argtypes = [u64, u64, u64]
            L.oracle_ntt_negacyclic.argtypes = [p, sz, u64, u64]
            L.oracle_intt_negacyclic.argtypes = [p, sz, u64, u64]
            L.oracle_polymul_batch.argtypes = [p, p, p, sz, sz, p, p]
            L.oracle_ntt_batch.argtypes = [p, sz, sz, p, p, ctypes.c_int]
            L.oracle_max_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"] and a.dtype == np.uint64
    return a.ctypes.data_as(ctypes.c_void_p)


def polymul_rows(a: np.ndarray, b: np.ndarray, qs, psis) -> np.ndarray:
    """Row-wise negacyclic products: a, b uint64[R][n]; row r modulo qs[r]."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    R, n = a.shape
    c = np.empty_like(a)
    q = np.ascontiguousarray(qs, dtype=np.uint64)
    ps = np.ascontiguousarray(psis, dtype=np.uint64)
    assert q.shape == (R,) and ps.shape == (R,) and b.shape == (R, n)
    lib().oracle_polymul_batch(_ptr(a), _ptr(b), _ptr(c), R, n, _ptr(q), _ptr(ps))
    return c


def ntt_rows(a: np.ndarray, qs, psis, inverse: bool = False) -> np.ndarray:
    """Row-wise negacyclic transforms (natural order), returns a new array."""
    a = np.array(a, dtype=np.uint64, copy=True, order="C")
    R, n = a.shape
    q = np.ascontiguousarray(qs, dtype=np.uint64)
    ps = np.ascontiguousarray(psis, dtype=np.uint64)
    lib().oracle_ntt_batch(_ptr(a), R, n, _ptr(q), _ptr(ps), 1 if inverse else 0)
    return a


def mulmod(a: int, b: int, q: int) -> int:
    return int(lib().oracle_mulmod(a, b, q))


def max_threads() -> int:
    return int(lib().oracle_max_threads())
