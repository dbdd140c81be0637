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
        L.oracle_sample.restype = ctypes.c_int
        L.oracle_sample.argtypes = [u64p, ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64,
                                    ctypes.c_uint64, u64p, u64p]
        L.oracle_membership.restype = ctypes.c_int
        L.oracle_membership.argtypes = [u64p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_int, u64p, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint8)]
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


def hash_range(F, begin: int, count: int) -> int:
    """Sum of h(z_i) mod 2^64 over solutions begin .. begin+count-1 (no counts)."""
    basis, shift = _words(F)
    W, n = F["words"], F["n"]
    h = np.zeros(1, dtype=np.uint64)
    rc = lib().oracle_reduce(_p(basis), F["rank"], W, n, _p(shift), begin, count,
                             None, _p(h), None)
    if rc != 0:
        raise ValueError(f"oracle_reduce failed ({rc})")
    return int(h[0])


def sample(F, seed: int, num: int, coeffs=None) -> np.ndarray:
    """uint64 array [num, W]: samples s = 0..num-1 (App. A), coefficient words
    from the SplitMix64 stream of ``seed`` or from ``coeffs`` (uint64
    [num, ceil(r/64)])."""
    basis, shift = _words(F)
    W, r = F["words"], F["rank"]
    out = np.zeros((max(num, 1), W), dtype=np.uint64)
    cp = None
    if coeffs is not None:
        c = np.ascontiguousarray(np.asarray(coeffs).view(np.uint64).reshape(num, -1))
        if c.shape[1] != (r + 63) // 64:
            raise ValueError("coefficients must have ceil(r/64) words per sample")
        cp = _p(c)
    rc = lib().oracle_sample(_p(basis), r, W, _p(shift), seed & ((1 << 64) - 1), num, cp, _p(out))
    if rc != 0:
        raise ValueError(f"oracle_sample failed ({rc})")
    return out[:num]


def membership(kernel, q, W: int, z) -> np.ndarray:
    """uint8 [num]: 1 iff q_f = 2 <z_s, k_f> (mod 4) for every kernel vector.

    ``kernel`` is the list of kernel basis vectors (ints), ``q`` their values
    of the quadratic form (ints), ``z`` a uint64 array [num, W]."""
    nk = len(kernel)
    kw = np.zeros((max(nk, 1), W), dtype=np.uint64)
    for f, k in enumerate(kernel):
        for w in range(W):
            kw[f, w] = (k >> (64 * w)) & ((1 << 64) - 1)
    qa = np.array(list(q) or [0], dtype=np.intc)
    zz = np.ascontiguousarray(np.asarray(z).view(np.uint64).reshape(-1, W))
    num = zz.shape[0]
    out = np.zeros(max(num, 1), dtype=np.uint8)
    rc = lib().oracle_membership(_p(kw), nk, qa.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), W,
                                 _p(zz) if num else _p(np.zeros(W, dtype=np.uint64)), num,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError(f"oracle_membership failed ({rc})")
    return out[:num]


def identity_hash(lo: int, hi: int) -> int:
    return int(lib().oracle_identity_hash(lo, hi))


def mix13(x: int) -> int:
    return int(lib().oracle_mix13(x))
