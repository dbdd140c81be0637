"""Serving: continuous admission of HLF requests onto one GPU, through the
native server of libhlf.so (hlf_server_*).

A request carries a dense matrix A (any n <= 1024) and a seed.  Its work is
the paper's two stages (Sections 1-2): stage 1 (pack + factor), then either
all 2^r solutions when r <= ``enum_max_rank`` and n <= 64, or
``num_samples`` uniform solutions (the quantum circuit's output distribution,
Appendix A).

The server (C++, one worker thread) owns ``slots`` HIP streams, one device
arena of ``hbm_budget`` bytes holding every device byte it uses (inputs,
packed rows, stage-1 records, outputs, the stage-1 cache) and a pinned host
arena for results.  A request is admitted when its arrival time has passed, a
slot is free and its stage-1 memory fits the arena; its phases then run on the
slot's stream (its output is carved at its exact size once r is known), so
requests arriving while others run are admitted as slots and memory free up
and their kernels overlap on the device.  Every result depends only on
(A, seed).

This module only marshals: it submits requests (with an xxh3 digest of A as
the stage-1 cache key) and wraps finished results as numpy views of the
server's pinned memory, returned to the server when the view is dropped.
"""

from __future__ import annotations

import ctypes
import hashlib
import time
from dataclasses import dataclass

import numpy as np

from . import hlf

try:  # a fast 128-bit digest for the stage-1 cache key; blake2b otherwise
    import xxhash

    def _digest(buf) -> bytes:
        return xxhash.xxh3_128_digest(buf)
except ImportError:  # pragma: no cover
    def _digest(buf) -> bytes:
        return hashlib.blake2b(buf, digest_size=16).digest()


@dataclass
class Request:
    rid: int
    A: np.ndarray
    seed: int
    arrival: float = 0.0  # seconds from the start of the run


@dataclass
class Result:
    rid: int
    status: int
    n: int
    rank: int
    kind: str                      # "enumerate" | "sample" | "error"
    data: np.ndarray | None        # pinned host memory of the server, or None
    admitted: float = 0.0          # seconds from the start of the run
    finished: float = 0.0
    latency: float = 0.0           # finished - arrival
    cache_hit: bool = False


class _Config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("hbm_bytes", ctypes.c_int64), ("host_bytes", ctypes.c_int64),
                ("num_samples", ctypes.c_int32), ("enum_max_rank", ctypes.c_int32),
                ("cache_entries", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n", ctypes.c_int32), ("A", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("key", ctypes.c_uint64 * 2), ("arrival_ns", ctypes.c_int64)]


class _Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("n", ctypes.c_int32),
                ("rank", ctypes.c_int32), ("kind", ctypes.c_int32), ("word_bytes", ctypes.c_int32),
                ("count", ctypes.c_int64), ("data", ctypes.c_void_p), ("arrival_ns", ctypes.c_int64),
                ("admitted_ns", ctypes.c_int64), ("finished_ns", ctypes.c_int64),
                ("cache_hit", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("admitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cache_hits", ctypes.c_int64),
                ("hbm_bytes", ctypes.c_int64), ("hbm_peak_bytes", ctypes.c_int64),
                ("host_peak_bytes", ctypes.c_int64), ("worker_status", ctypes.c_int32)]


_sigs = False


def _lib():
    global _sigs
    L = hlf.lib()
    if not _sigs:
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.hlf_server_create.restype = i32
        L.hlf_server_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(vp)]
        L.hlf_server_now.restype = i64
        L.hlf_server_now.argtypes = [vp]
        L.hlf_server_submit.restype = i32
        L.hlf_server_submit.argtypes = [vp, ctypes.POINTER(_Request), i32]
        L.hlf_server_poll.restype = i32
        L.hlf_server_poll.argtypes = [vp, ctypes.POINTER(_Result), i32, ctypes.POINTER(i32), i32]
        L.hlf_server_release.restype = i32
        L.hlf_server_release.argtypes = [vp, vp]
        L.hlf_server_get_stats.restype = i32
        L.hlf_server_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.hlf_server_destroy.restype = i32
        L.hlf_server_destroy.argtypes = [vp]
        _sigs = True
    return L


class _Lease:
    """Returns a result's pinned memory to the server when dropped."""

    def __init__(self, server: "Server", ptr: int):
        self.server = server
        self.ptr = ptr

    def __del__(self):
        h = getattr(self.server, "_h", None)
        if h:
            _lib().hlf_server_release(h, ctypes.c_void_p(self.ptr))


def _view(server: "Server", r: _Result) -> np.ndarray:
    nbytes = int(r.count) * int(r.word_bytes)
    buf = (ctypes.c_uint8 * nbytes).from_address(r.data)
    buf._lease = _Lease(server, r.data)  # the numpy view keeps buf, buf keeps the lease
    if r.kind == 1:
        dt = {2: np.int16, 4: np.int32, 8: np.int64}[int(r.word_bytes)]
        return np.frombuffer(buf, dtype=dt)
    W = int(r.word_bytes) // 8
    return np.frombuffer(buf, dtype=np.int64).reshape(int(r.count), W)


def _worst_output_bytes(n: int, num_samples: int, enum_max_rank: int) -> int:
    W = hlf.words_for(n)
    sample = num_samples * W * 8
    if n <= 64:
        width = 2 if n <= 16 else 4 if n <= 32 else 8
        return max(sample, (1 << enum_max_rank) * width)
    return sample


def _record_bytes(n: int) -> int:
    W = hlf.words_for(n)
    return (8 + 4 * n + 7) // 8 * 8 + 8 * (n * W + W)


class Server:
    def __init__(self, slots: int = 8, hbm_budget: int = 1 << 30, num_samples: int = 65536,
                 enum_max_rank: int = 24, cache_entries: int = 256, host_budget: int = 512 << 20):
        self.slots = slots
        self.budget = hbm_budget
        self.num_samples = num_samples
        self.enum_max_rank = enum_max_rank
        cfg = _Config(slots, hbm_budget, host_budget, num_samples, enum_max_rank, cache_entries)
        h = ctypes.c_void_p()
        hlf._check(_lib().hlf_server_create(ctypes.byref(cfg), ctypes.byref(h)), "hlf_server_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib().hlf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, n: int) -> int:
        """Most device bytes one request of size n can hold at once: input,
        packed rows and record in stage 1, then record and output (an upper
        bound; the arena rounds blocks to 256 bytes)."""
        return n * n + 8 * n * hlf.words_for(n) + _record_bytes(n) + _worst_output_bytes(
            n, self.num_samples, self.enum_max_rank)

    def stats(self) -> dict:
        st = _Stats()
        hlf._check(_lib().hlf_server_get_stats(self._h, ctypes.byref(st)), "hlf_server_get_stats")
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    @property
    def max_in_flight(self) -> int:
        """Most device arena bytes in use at once (inputs, records, outputs, cache)."""
        return int(self.stats()["hbm_peak_bytes"])

    def run(self, requests, realtime: bool = True, keep_data: bool = True,
            stall_s: float = 60.0) -> list[Result]:
        """Serve `requests` (arrival times in seconds from the start when
        `realtime`, else all present at the start) and return their results
        in completion order.  With keep_data=False each result's memory goes
        back to the server as soon as it is polled (data is None)."""
        L = _lib()
        reqs = sorted(requests, key=lambda q: (q.arrival, q.rid))
        mats = [np.ascontiguousarray(q.A, dtype=np.uint8) for q in reqs]
        arr = (_Request * max(len(reqs), 1))()
        for k, (q, A) in enumerate(zip(reqs, mats)):
            d = _digest(A.data)
            arr[k].id = q.rid
            arr[k].n = A.shape[0]
            arr[k].A = A.ctypes.data
            arr[k].seed = q.seed & ((1 << 64) - 1)
            arr[k].key[0] = int.from_bytes(d[:8], "little")
            arr[k].key[1] = int.from_bytes(d[8:16], "little")
        # the run's clock starts once everything is prepared (1 ms to submit)
        start = L.hlf_server_now(self._h) + 1_000_000
        arrival = {}
        for k, q in enumerate(reqs):
            t = start + (int(q.arrival * 1e9) if realtime else 0)
            arr[k].arrival_ns = t
            arrival[q.rid] = t
        if reqs:
            hlf._check(L.hlf_server_submit(self._h, arr, len(reqs)), "hlf_server_submit")
        out = (_Result * 64)()
        got = ctypes.c_int32()
        done: list[Result] = []
        last = time.perf_counter()
        while len(done) < len(reqs):
            hlf._check(L.hlf_server_poll(self._h, out, 64, ctypes.byref(got), 50), "hlf_server_poll")
            if got.value == 0:
                if time.perf_counter() - last > stall_s:
                    # the server reads each A at admission: stop it before `mats` goes away
                    msg = f"server made no progress for {stall_s} s ({len(done)}/{len(reqs)} done): {self.stats()}"
                    self.close()
                    raise hlf.HlfError(hlf.HLF_EDEVICE, msg)
                continue
            last = time.perf_counter()
            for i in range(got.value):
                r = out[i]
                data = None
                if r.data:
                    if keep_data:
                        data = _view(self, r)
                    else:
                        L.hlf_server_release(self._h, ctypes.c_void_p(r.data))
                kind = {1: "enumerate", 2: "sample"}.get(int(r.kind), "error")
                t_arr = arrival[int(r.id)]
                done.append(Result(rid=int(r.id), status=int(r.status), n=int(r.n), rank=int(r.rank),
                                   kind=kind, data=data, admitted=(r.admitted_ns - start) * 1e-9,
                                   finished=(r.finished_ns - start) * 1e-9,
                                   latency=(r.finished_ns - t_arr) * 1e-9, cache_hit=bool(r.cache_hit)))
        return done


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else float("nan")
