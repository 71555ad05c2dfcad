"""ctypes front end for the plain-C oracle (``ntt_ref.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring). Arrays are numpy
``uint64`` of shape ``(..., 4)``: canonical little-endian limbs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_transform.argtypes = [u64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_transform.restype = ctypes.c_int
        L.oracle_eval_output.argtypes = [u64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u64p]
        L.oracle_eval_output.restype = ctypes.c_int
        L.oracle_mul.argtypes = [u64p, u64p, u64p]
        L.oracle_mul.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def transform(x: np.ndarray, log_n: int, kind: int = 0, threads: int = 0) -> np.ndarray:
    """Transform of every length-2^log_n polynomial in ``x`` (copy returned)."""
    a = np.ascontiguousarray(np.array(x, dtype=np.uint64, copy=True))
    n = 1 << log_n
    if a.size % (4 * n):
        raise ValueError("array size is not a multiple of 2^log_n elements")
    batch = a.size // (4 * n)
    rc = lib().oracle_transform(_ptr(a), log_n, kind, batch, threads)
    if rc != 0:
        raise ValueError("oracle_transform rejected its input (bad argument or element >= r)")
    return a


def eval_output(x: np.ndarray, log_n: int, k: int, kind: int = 0) -> np.ndarray:
    """Output k of the transform of one polynomial, from the definition (O(N))."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    rc = lib().oracle_eval_output(_ptr(a), log_n, k, kind, _ptr(out))
    if rc != 0:
        raise ValueError("oracle_eval_output rejected its input")
    return out


def mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    if lib().oracle_mul(_ptr(a), _ptr(b), _ptr(out)) != 0:
        raise ValueError("operand >= r")
    return out


def max_threads() -> int:
    return int(lib().oracle_max_threads())
