"""Serving loop: continuous admission of HLF requests onto one GPU.

A request carries a dense matrix A (any n <= 1024) and a seed.  Its work is
the paper's two stages (Sections 1-2): stage 1 (pack + factor), then either
the full enumeration of its 2^r solutions when r <= ``enum_max_rank`` and
n <= 64, or ``num_samples`` uniform solutions (the quantum circuit's output
distribution, Appendix A).  Results are copied to pinned host memory.

Scheduling.  The server owns ``slots`` HIP streams.  A request is admitted
when a slot is free and its worst-case device footprint fits the HBM budget;
admitted requests advance independently (phase 1 -> phase 2 -> copy-out),
each phase enqueued on the slot's stream as soon as the previous one has
finished, so requests that arrive while others run are admitted as slots and
memory free up and their kernels overlap on the device.  Every result depends
only on (A, seed): the sampling stream is keyed by (seed, sample index), never
by slot or timing, so a request's result is bit-identical alone and in a mix.

Stage-1 records are cached on the device, keyed by a digest of A (LRU, part
of the budget); a repeated matrix skips stage 1.

All device work goes through the C ABI of libhlf.so (``hlf``); this module only
schedules.
"""

from __future__ import annotations

import collections
import hashlib
import time

try:  # a fast 128-bit digest for the stage-1 cache key; blake2b otherwise
    import xxhash

    def _digest(buf: bytes) -> bytes:
        return xxhash.xxh3_128_digest(buf)
except ImportError:  # pragma: no cover
    def _digest(buf: bytes) -> bytes:
        return hashlib.blake2b(buf, digest_size=16).digest()
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hlf


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
    data: np.ndarray | None        # host result (pinned memory): uint64 (count, W) or narrow words
    admitted: float = 0.0
    finished: float = 0.0
    latency: float = 0.0           # finished - arrival
    cache_hit: bool = False


@dataclass
class _Entry:  # device-resident stage-1 record in the cache
    F: hlf.Factors
    rank: int
    status: int
    nbytes: int


@dataclass
class _Active:
    req: Request
    slot: int
    phase: int
    n: int
    footprint: int
    admitted: float
    F: hlf.Factors | None = None
    out: torch.Tensor | None = None
    host_out: torch.Tensor | None = None
    event: torch.cuda.Event | None = None
    key: bytes = b""
    cache_hit: bool = False
    kind: str = ""
    rank: int = -1
    status: int = 0
    extra: dict = field(default_factory=dict)


def _record_bytes(n: int) -> int:
    W = hlf.words_for(n)
    return 8 * (2 * n * W + W) + 4 * (n + 2)


def _worst_output_bytes(n: int, num_samples: int, enum_max_rank: int) -> int:
    W = hlf.words_for(n)
    sample = num_samples * W * 8
    if n <= 64:
        width = 2 if n <= 16 else 4 if n <= 32 else 8
        return max(sample, (1 << enum_max_rank) * width)
    return sample


class Server:
    def __init__(self, slots: int = 8, hbm_budget: int = 1 << 30, num_samples: int = 65536,
                 enum_max_rank: int = 24, cache_entries: int = 256, device: int = 0):
        self.device = torch.device("cuda", device)
        self.slots = slots
        self.budget = hbm_budget
        self.num_samples = num_samples
        self.enum_max_rank = enum_max_rank
        self.cache_entries = cache_entries
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # Per-slot buffers, grown on demand and reused: a slot takes its next
        # request only after every event of the previous one has fired.
        # Pinned staging of the dense input, its device copy, the packed rows,
        # the stage-2 output, and the pinned (status, rank) pair.
        self.staging: list[torch.Tensor | None] = [None] * slots
        self.dev_A: list[torch.Tensor | None] = [None] * slots
        self.dev_rows: list[torch.Tensor | None] = [None] * slots
        self.dev_out: list[torch.Tensor | None] = [None] * slots
        self.head_host = [torch.empty(2, dtype=torch.int32, pin_memory=True) for _ in range(slots)]
        self.cache: collections.OrderedDict[bytes, _Entry] = collections.OrderedDict()
        self.cache_bytes = 0
        self.in_flight = 0
        self.max_in_flight = 0
        self.stats = {"admitted": 0, "cache_hits": 0, "rejected": 0}

    # -- footprint / budget -------------------------------------------------
    def footprint(self, n: int) -> int:
        return n * n + 8 * n * hlf.words_for(n) + _record_bytes(n) + _worst_output_bytes(
            n, self.num_samples, self.enum_max_rank)

    def _fits(self, nbytes: int) -> bool:
        return self.in_flight + self.cache_bytes + nbytes <= self.budget

    def _evict_for(self, nbytes: int):
        while self.cache and not self._fits(nbytes):
            _, e = self.cache.popitem(last=False)
            self.cache_bytes -= e.nbytes

    # -- phases ---------------------------------------------------------------
    def _admit(self, req: Request, slot: int, now: float) -> _Active:
        n = req.A.shape[0]
        a = _Active(req=req, slot=slot, phase=1, n=n, footprint=self.footprint(n), admitted=now)
        A = np.ascontiguousarray(req.A, dtype=np.uint8)
        a.key = _digest(A.data) + n.to_bytes(2, "little")
        self.in_flight += a.footprint
        self.max_in_flight = max(self.max_in_flight, self.in_flight + self.cache_bytes)
        self.stats["admitted"] += 1
        s = self.streams[slot]
        hit = self.cache.get(a.key)
        if hit is not None:
            self.cache.move_to_end(a.key)
            a.cache_hit = True
            self.stats["cache_hits"] += 1
            a.F, a.rank, a.status = hit.F, hit.rank, hit.status
            a.F._buf.record_stream(s)  # keep the memory until this stream is done with it
            self._launch_phase2(a)
            return a
        with torch.cuda.stream(s):
            # H2D through the slot's pinned staging buffer.
            st = self._grow(self.staging, slot, n * n, torch.uint8, pinned=True)
            st[: n * n].numpy()[:] = A.reshape(-1)
            Ad = self._grow(self.dev_A, slot, n * n, torch.uint8)[: n * n]
            Ad.copy_(st[: n * n], non_blocking=True)
            W = hlf.words_for(n)
            rows = self._grow(self.dev_rows, slot, n * W, torch.int64)[: n * W].view(n, W)
            # The record outlives the request when it is cached: its own buffer.
            a.F = hlf.Factors.packed(n, device=self.device)
            # pack writes its verdict into the record's status; the factor
            # keeps a failed one (HLF_FACTOR_PACK_STATUS)
            hlf.pack_dense(Ad.view(n, n), rows, a.F.status, stream=s)
            hlf.factor(rows, n, a.F, stream=s, pack_status=True)
            self.head_host[slot].copy_(a.F.status_rank, non_blocking=True)
            a.event = torch.cuda.Event()
            a.event.record(s)
        return a

    def _grow(self, pool, slot: int, numel: int, dtype, pinned: bool = False) -> torch.Tensor:
        buf = pool[slot]
        if buf is None or buf.numel() < numel:
            size = max(numel, 1 << 16)
            if pinned:
                buf = torch.empty(size, dtype=dtype, pin_memory=True)
            else:
                buf = torch.empty(size, dtype=dtype, device=self.device)
            pool[slot] = buf
        return buf

    def _launch_phase2(self, a: _Active):
        a.phase = 2
        s = self.streams[a.slot]
        n, r = a.n, a.rank
        with torch.cuda.stream(s):
            if a.status != hlf.HLF_OK:
                a.kind = "error"
                a.out = None
            elif r <= self.enum_max_rank and n <= 64:
                a.kind = "enumerate"
                wb = 16 if n <= 16 else 32 if n <= 32 else 64
                dt = {16: torch.int16, 32: torch.int32, 64: torch.int64}[wb]
                nbytes = (1 << r) * wb // 8
                out = self._grow(self.dev_out, a.slot, (nbytes + 7) // 8, torch.int64)
                a.out = out.view(torch.uint8)[:nbytes].view(dt)
                hlf.enumerate_solutions(a.F, 0, 1 << r, wb, out=a.out, stream=s)
            else:
                a.kind = "sample"
                W = a.F.words
                out = self._grow(self.dev_out, a.slot, self.num_samples * W, torch.int64)
                a.out = out[: self.num_samples * W].view(self.num_samples, W)
                hlf.sample(a.F, a.req.seed, self.num_samples, out=a.out, stream=s)
            if a.out is not None:
                a.host_out = torch.empty(a.out.shape, dtype=a.out.dtype, pin_memory=True)
                a.host_out.copy_(a.out, non_blocking=True)
            a.event = torch.cuda.Event()
            a.event.record(s)

    def _finish(self, a: _Active, now: float) -> Result:
        self.in_flight -= a.footprint
        if not a.cache_hit and a.status == hlf.HLF_OK and self.cache_entries > 0:
            nb = _record_bytes(a.n)
            self._evict_for(nb)
            if self._fits(nb):
                self.cache[a.key] = _Entry(a.F, a.rank, a.status, nb)
                self.cache_bytes += nb
                while len(self.cache) > self.cache_entries:
                    _, e = self.cache.popitem(last=False)
                    self.cache_bytes -= e.nbytes
        # The pinned buffer itself is handed over (numpy keeps it alive).
        data = a.host_out.numpy() if a.host_out is not None else None
        arrival = a.req.arrival if self._realtime else 0.0
        return Result(rid=a.req.rid, status=a.status, n=a.n, rank=a.rank, kind=a.kind, data=data,
                      admitted=a.admitted, finished=now, latency=now - arrival,
                      cache_hit=a.cache_hit)

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, realtime: bool = True) -> list[Result]:
        """Serve `requests` (arrival times in seconds from the start when
        `realtime`, else all present at time 0) and return their results in
        completion order."""
        pending = collections.deque(sorted(requests, key=lambda q: (q.arrival, q.rid)))
        for q in pending:
            if self.footprint(q.A.shape[0]) > self.budget:
                raise hlf.HlfError(hlf.HLF_ENOMEM, f"request {q.rid} exceeds the HBM budget")
        self._realtime = realtime  # without it every request counts as arrived at t = 0
        active: dict[int, _Active] = {}
        free = list(range(self.slots))
        done: list[Result] = []
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            progressed = False
            # admission: arrived requests, free slots, budget (with cache eviction)
            while pending and free and (not realtime or pending[0].arrival <= now):
                fp = self.footprint(pending[0].A.shape[0])
                if not self._fits(fp):
                    self._evict_for(fp)
                    if not self._fits(fp):
                        break
                req = pending.popleft()
                slot = free.pop()
                active[slot] = self._admit(req, slot, now)
                progressed = True
            # advance admitted requests whose last phase finished
            for slot in list(active):
                a = active[slot]
                if a.event is not None and not a.event.query():
                    continue
                now = time.perf_counter() - t0
                if a.phase == 1:
                    head = self.head_host[slot]
                    a.status, a.rank = int(head[0]), int(head[1])
                    self._launch_phase2(a)
                else:
                    done.append(self._finish(a, now))
                    del active[slot]
                    free.append(slot)
                progressed = True
            if not progressed:
                if active:
                    time.sleep(0)
                elif pending and realtime:
                    time.sleep(max(0.0, min(1e-3, pending[0].arrival - now)))
        return done


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else float("nan")
