"""ctypes loader for the plain C oracle -- TEST INFRASTRUCTURE ONLY.

The functions mirror ``hlf_oracle.c``; inputs are the Python oracle's stage-1
results (basis, shift), never anything produced by the HIP library.
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
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_mix13.restype = ctypes.c_uint64
        L.oracle_mix13.argtypes = [ctypes.c_uint64]
        L.oracle_enumerate.restype = ctypes.c_int
        L.oracle_enumerate.argtypes = [u64p, ctypes.c_int, ctypes.c_int, u64p,
                                       ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.oracle_enumerate_counter.restype = ctypes.c_int
        L.oracle_enumerate_counter.argtypes = [u64p, ctypes.c_int, ctypes.c_int, u64p,
                                               ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.oracle_reduce.restype = ctypes.c_int
        L.oracle_reduce.argtypes = [u64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p,
                                    ctypes.c_uint64, ctypes.c_uint64, u64p, u64p, u64p]
        L.oracle_identity_hash.restype = ctypes.c_uint64
        L.oracle_identity_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = L
    return _lib


def _words(F):
    W = F["words"]
    r = F["rank"]
    basis = np.zeros(max(r, 1) * W, dtype=np.uint64)
    for k, B in enumerate(F["basis"]):
        for w in range(W):
            basis[k * W + w] = (B >> (64 * w)) & ((1 << 64) - 1)
    shift = np.array([(F["shift"] >> (64 * w)) & ((1 << 64) - 1) for w in range(W)],
                     dtype=np.uint64)
    return basis, shift


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def threads() -> int:
    return int(lib().oracle_threads())


def enumerate_range(F, begin: int, count: int) -> np.ndarray:
    """uint64 array [count, W] of solutions begin .. begin+count-1 (Gray order)."""
    basis, shift = _words(F)
    W = F["words"]
    out = np.zeros((count, W), dtype=np.uint64)
    rc = lib().oracle_enumerate(_p(basis), F["rank"], W, _p(shift), begin, count,
                                _p(out) if count else _p(np.zeros(1, dtype=np.uint64)))
    if rc != 0:
        raise ValueError(f"oracle_enumerate failed ({rc})")
    return out


def enumerate_counter_range(F, begin: int, count: int) -> np.ndarray:
    """uint64 array [count, W] of solutions begin .. begin+count-1 in counter order."""
    basis, shift = _words(F)
    W = F["words"]
    out = np.zeros((count, W), dtype=np.uint64)
    rc = lib().oracle_enumerate_counter(_p(basis), F["rank"], W, _p(shift), begin, count,
                                        _p(out) if count else _p(np.zeros(1, dtype=np.uint64)))
    if rc != 0:
        raise ValueError(f"oracle_enumerate_counter failed ({rc})")
    return out


def reduce_range(F, begin: int, count: int):
    """(counts uint64[n], hash int, xorfold uint64[W])."""
    basis, shift = _words(F)
    W, n = F["words"], F["n"]
    counts = np.zeros(n, dtype=np.uint64)
    h = np.zeros(1, dtype=np.uint64)
    xf = np.zeros(W, dtype=np.uint64)
    rc = lib().oracle_reduce(_p(basis), F["rank"], W, n, _p(shift), begin, count,
                             _p(counts), _p(h), _p(xf))
    if rc != 0:
        raise ValueError(f"oracle_reduce failed ({rc})")
    return counts, int(h[0]), xf


def identity_hash(lo: int, hi: int) -> int:
    return int(lib().oracle_identity_hash(lo, hi))


def mix13(x: int) -> int:
    return int(lib().oracle_mix13(x))
