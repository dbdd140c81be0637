"""Thin ctypes binding of libhlf.so (the C ABI declared in include/hlf.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libhlf.so.  PyTorch provides device memory and the current stream.
uint64 data lives in int64 tensors (same bits); ``as_uint64`` reinterprets a
host copy.  If libhlf.so is missing, every call raises ``HlfError``: there is
no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlf.so")

HLF_OK = 0
HLF_EINVAL = -1
HLF_ENOTSYM = -2
HLF_ERANGE = -3
HLF_ENOMEM = -4
HLF_EDEVICE = -5
HLF_EINTERNAL = -7
HLF_MAX_N = 1024
HLF_MAX_ENUM_RANK = 62
HLF_ORDER_COUNTER = 1
HLF_ACCUMULATE = 1
HLF_FACTOR_WORKGROUP = 1
HLF_FACTOR_PACK_STATUS = 2

EXPORTED = (
    "hlf_version", "hlf_status_string", "hlf_words_for", "hlf_pack_dense", "hlf_factor",
    "hlf_factor_ex", "hlf_solve_dense", "hlf_enumerate", "hlf_enumerate_ex", "hlf_enumerate_circuit",
    "hlf_enumerate_reduce", "hlf_sample", "hlf_pair_stats", "hlf_membership",
    "hlf_batch_create", "hlf_batch_destroy", "hlf_batch_get_layout", "hlf_batch_factor_dense",
    "hlf_batch_enumerate", "hlf_batch_enumerate_overlap", "hlf_batch_solve", "hlf_batch_reduce", "hlf_batch_tune", "hlf_batch_graph_capture",
    "hlf_batch_graph_launch", "hlf_batch_reduce_noalloc",
    "hlf_server_create", "hlf_server_now", "hlf_server_submit", "hlf_server_poll", "hlf_server_release",
    "hlf_server_get_stats", "hlf_server_destroy",
)


class HlfError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        msg = status_string(code) if _lib is not None else str(code)
        super().__init__(f"{where}: {msg}" if where else msg)


class _Factors(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("words", ctypes.c_int32),
        ("status", ctypes.c_void_p),
        ("rank", ctypes.c_void_p),
        ("pivots", ctypes.c_void_p),
        ("basis", ctypes.c_void_p),
        ("shift", ctypes.c_void_p),
        ("kernel", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libhlf.so (raises HlfError if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HlfError(HLF_EDEVICE, f"{LIB_PATH} is missing; build it with "
                                        "`python -m paper_2103_00693_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        fp = ctypes.POINTER(_Factors)
        L.hlf_version.restype = i32
        L.hlf_status_string.restype = ctypes.c_char_p
        L.hlf_status_string.argtypes = [i32]
        L.hlf_words_for.restype = i32
        L.hlf_words_for.argtypes = [i32]
        L.hlf_pack_dense.restype = i32
        L.hlf_pack_dense.argtypes = [vp, i32, vp, vp, vp]
        L.hlf_factor.restype = i32
        L.hlf_factor.argtypes = [vp, fp, vp]
        L.hlf_factor_ex.restype = i32
        L.hlf_factor_ex.argtypes = [vp, fp, u32, vp]
        L.hlf_enumerate.restype = i32
        L.hlf_enumerate.argtypes = [fp, u64, u64, i32, vp, vp]
        L.hlf_enumerate_ex.restype = i32
        L.hlf_enumerate_ex.argtypes = [fp, u64, u64, i32, u32, vp, vp]
        L.hlf_pair_stats.restype = i32
        L.hlf_pair_stats.argtypes = [fp, vp, vp, vp]
        L.hlf_membership.restype = i32
        L.hlf_membership.argtypes = [fp, vp, u64, vp, vp]
        L.hlf_enumerate_circuit.restype = i32
        L.hlf_enumerate_circuit.argtypes = [fp, vp, i32, u64, u64, i32, vp, vp]
        L.hlf_solve_dense.restype = i32
        L.hlf_solve_dense.argtypes = [vp, fp, u64, u64, i32, vp, vp]
        L.hlf_enumerate_reduce.restype = i32
        L.hlf_enumerate_reduce.argtypes = [fp, u64, u64, u32, vp, vp, vp, vp]
        L.hlf_sample.restype = i32
        L.hlf_sample.argtypes = [fp, u64, u64, vp, vp, vp]
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().hlf_status_string(int(code)).decode()


def words_for(n: int) -> int:
    return (n + 63) // 64


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(code: int, where: str):
    if code != HLF_OK:
        raise HlfError(code, where)


def as_uint64(t: torch.Tensor) -> np.ndarray:
    """Host copy of an int64 tensor viewed as uint64."""
    return t.detach().cpu().numpy().view(np.uint64)


class Factors:
    """A device-resident factor record (hlf_factors) whose buffers are tensors."""

    def __init__(self, n: int, device=None, kernel: bool = True):
        if not 1 <= n <= HLF_MAX_N:
            raise HlfError(HLF_EINVAL, f"n={n} outside [1, {HLF_MAX_N}]")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        W = words_for(n)
        self.n, self.words, self.device = n, W, dev
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.rank = torch.zeros(1, dtype=torch.int32, device=dev)
        self.pivots = torch.full((n,), -1, dtype=torch.int32, device=dev)
        self.basis = torch.zeros((n, W), dtype=torch.int64, device=dev)
        self.shift = torch.zeros(W, dtype=torch.int64, device=dev)
        self.kernel = torch.zeros((n, W), dtype=torch.int64, device=dev) if kernel else None
        self._c = _Factors(n, W, self.status.data_ptr(), self.rank.data_ptr(),
                           self.pivots.data_ptr(), self.basis.data_ptr(), self.shift.data_ptr(),
                           self.kernel.data_ptr() if kernel else 0)

    @classmethod
    def packed(cls, n: int, device=None, kernel: bool = False) -> "Factors":
        """A record in ONE uninitialised device buffer: status and rank
        adjacent (one 8-byte copy reads both), then pivots, shift, basis and
        the optional kernel vectors.  hlf_factor writes every field that a
        later call reads (the basis rows past r are not read)."""
        if not 1 <= n <= HLF_MAX_N:
            raise HlfError(HLF_EINVAL, f"n={n} outside [1, {HLF_MAX_N}]")
        self = cls.__new__(cls)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        W = words_for(n)
        self.n, self.words, self.device = n, W, dev
        piv_words = (n + 1) // 2                       # int32 pivots in int64 units
        total = 1 + piv_words + W + n * W + (n * W if kernel else 0)
        buf = torch.empty(total, dtype=torch.int64, device=dev)
        self._buf = buf
        head = buf[:1].view(torch.int32)               # [status, rank]
        self.status, self.rank = head[0:1], head[1:2]
        self.status_rank = head
        self.pivots = buf[1:1 + piv_words].view(torch.int32)[:n]
        o = 1 + piv_words
        self.shift = buf[o:o + W]
        self.basis = buf[o + W:o + W + n * W].view(n, W)
        o += W + n * W
        self.kernel = buf[o:o + n * W].view(n, W) if kernel else None
        self._c = _Factors(n, W, self.status.data_ptr(), self.rank.data_ptr(),
                           self.pivots.data_ptr(), self.basis.data_ptr(), self.shift.data_ptr(),
                           self.kernel.data_ptr() if kernel else 0)
        return self

    @property
    def c(self):
        return ctypes.byref(self._c)

    def check(self):
        """Synchronise and raise HlfError if the device status is not HLF_OK."""
        code = int(self.status.item())
        if code != HLF_OK:
            raise HlfError(code, "device status")
        return self

    def read(self) -> dict:
        """Synchronise and return the record as Python ints (bit j of an int is z_{j+1})."""
        status = int(self.status.item())
        r = int(self.rank.item())
        W = self.words
        basis = as_uint64(self.basis)
        shift = as_uint64(self.shift)

        def to_int(row):
            return sum(int(row[w]) << (64 * w) for w in range(W))

        out = {
            "status": status,
            "n": self.n,
            "words": W,
            "rank": r,
            "pivots": [int(p) for p in self.pivots.cpu().tolist()],
            "basis": [to_int(basis[k]) for k in range(r)],
            "shift": to_int(shift),
        }
        if self.kernel is not None:
            kern = as_uint64(self.kernel)
            out["kernel"] = [to_int(kern[j]) for j in range(self.n - r)]
        return out


def pack_dense(A: torch.Tensor, rows: torch.Tensor | None = None,
               status: torch.Tensor | None = None, stream=None):
    """A0: hlf_pack_dense on a uint8 (n, n) device tensor -> (rows, status)."""
    if A.dtype != torch.uint8 or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise HlfError(HLF_EINVAL, "A must be a square uint8 tensor")
    A = A.contiguous()
    n = A.shape[0]
    W = words_for(n)
    if rows is None:
        rows = torch.empty((n, W), dtype=torch.int64, device=A.device)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib().hlf_pack_dense(_ptr(A), n, _ptr(rows), _ptr(status), _stream(stream)),
           "hlf_pack_dense")
    return rows, status


def factor(rows: torch.Tensor, n: int, F: Factors | None = None, workgroup: bool = False,
           stream=None, pack_status: bool = False) -> Factors:
    """A1-A4: hlf_factor(_ex) of packed rows into a device record.  With
    pack_status, F.status must have been the status output of the
    pack_dense of these rows on the same stream (HLF_FACTOR_PACK_STATUS)."""
    if F is None:
        F = Factors(n, device=rows.device)
    flags = (HLF_FACTOR_WORKGROUP if workgroup else 0) | (HLF_FACTOR_PACK_STATUS if pack_status else 0)
    _check(lib().hlf_factor_ex(_ptr(rows), F.c, flags, _stream(stream)), "hlf_factor")
    return F


_DTYPES = {16: torch.int16, 32: torch.int32, 64: torch.int64}


def enumerate_solutions(F: Factors, begin: int, count: int, word_bits: int,
                        out: torch.Tensor | None = None, stream=None,
                        order: str = "gray") -> torch.Tensor:
    """E1: hlf_enumerate (order "gray") or hlf_enumerate_ex with
    HLF_ORDER_COUNTER (order "counter") into ``out`` (allocated when None)."""
    if order not in ("gray", "counter"):
        raise HlfError(HLF_EINVAL, f"order {order!r}")
    if out is None:
        if word_bits in _DTYPES and F.n <= word_bits:
            out = torch.empty(count, dtype=_DTYPES[word_bits], device=F.device)
        else:
            out = torch.empty((count, word_bits // 64), dtype=torch.int64, device=F.device)
    if order == "gray":
        _check(lib().hlf_enumerate(F.c, begin, count, word_bits, _ptr(out) if count else None,
                                   _stream(stream)), "hlf_enumerate")
    else:
        _check(lib().hlf_enumerate_ex(F.c, begin, count, word_bits, HLF_ORDER_COUNTER,
                                      _ptr(out) if count else None, _stream(stream)),
               "hlf_enumerate_ex")
    return out


def solve_dense(A: torch.Tensor, F: Factors, begin: int, count: int, word_bits: int,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """A0-A4 + E1 of one instance with n <= 64 in one launch (hlf_solve_dense):
    the record F is written as by factor(), out[i - begin] = z_i."""
    if A.dtype != torch.uint8 or A.dim() != 2 or A.shape[0] != A.shape[1] or A.shape[0] != F.n:
        raise HlfError(HLF_EINVAL, "A must be a square uint8 tensor of the record's n")
    A = A.contiguous()
    if out is None and count:
        out = torch.empty(count, dtype=_DTYPES[word_bits], device=F.device)
    _check(lib().hlf_solve_dense(_ptr(A), F.c, begin, count, word_bits,
                                 _ptr(out) if count else None, _stream(stream)),
           "hlf_solve_dense")
    return out


def enumerate_circuit(F: Factors, rows: torch.Tensor, grid_N: int, begin: int, count: int,
                      word_bits: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """f1: hlf_enumerate_circuit -- the paper's circuit in binary-counter order
    (word_bits 16/32/64 for n <= 64, else 64*W: out is int64 (count, W))."""
    if out is None:
        if word_bits in _DTYPES and F.n <= word_bits:
            out = torch.empty(count, dtype=_DTYPES[word_bits], device=F.device)
        else:
            out = torch.empty((count, word_bits // 64), dtype=torch.int64, device=F.device)
    _check(lib().hlf_enumerate_circuit(F.c, _ptr(rows), grid_N, begin, count, word_bits,
                                       _ptr(out) if count else None, _stream(stream)),
           "hlf_enumerate_circuit")
    return out


def enumerate_reduce(F: Factors, begin: int, count: int, accumulate: bool = False,
                     counts: torch.Tensor | None = None, hash_out: torch.Tensor | None = None,
                     xorfold: torch.Tensor | None = None, want_xorfold: bool = True,
                     stream=None):
    """E2: hlf_enumerate_reduce -> (counts int64[n], hash int64[1], xorfold int64[W] or None)."""
    dev = F.device
    if counts is None:
        counts = torch.zeros(F.n, dtype=torch.int64, device=dev)
    if hash_out is None:
        hash_out = torch.zeros(1, dtype=torch.int64, device=dev)
    if xorfold is None and want_xorfold:
        xorfold = torch.zeros(F.words, dtype=torch.int64, device=dev)
    flags = HLF_ACCUMULATE if accumulate else 0
    _check(lib().hlf_enumerate_reduce(F.c, begin, count, flags, _ptr(counts), _ptr(hash_out),
                                      _ptr(xorfold), _stream(stream)), "hlf_enumerate_reduce")
    return counts, hash_out, xorfold


def sample(F: Factors, seed: int, num: int, coeffs: torch.Tensor | None = None,
           out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """S1: hlf_sample -> int64 (num, W)."""
    if out is None:
        out = torch.empty((num, F.words), dtype=torch.int64, device=F.device)
    _check(lib().hlf_sample(F.c, seed & ((1 << 64) - 1), num, _ptr(coeffs),
                            _ptr(out) if num else None, _stream(stream)), "hlf_sample")
    return out


def pair_stats(F: Factors, rows: torch.Tensor, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """hlf_pair_stats -> uint8 (n, n): 4 * P(z_i = 1 and z_j = 1)."""
    if out is None:
        out = torch.empty((F.n, F.n), dtype=torch.uint8, device=F.device)
    _check(lib().hlf_pair_stats(F.c, _ptr(rows), _ptr(out), _stream(stream)), "hlf_pair_stats")
    return out


def membership(F: Factors, z: torch.Tensor, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """hlf_membership -> uint8 (num,): 1 where z[s] (int64 (num, W)) is a solution."""
    num = z.shape[0]
    if out is None:
        out = torch.empty(num, dtype=torch.uint8, device=F.device)
    _check(lib().hlf_membership(F.c, _ptr(z) if num else None, num, _ptr(out) if num else None,
                                _stream(stream)), "hlf_membership")
    return out


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------

class _BatchLayout(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int32),
        ("max_n", ctypes.c_int32),
        ("dense_bytes", ctypes.c_int64),
        ("mat_words", ctypes.c_int64),
        ("vec_words", ctypes.c_int64),
        ("piv_entries", ctypes.c_int64),
        ("dense_off", ctypes.POINTER(ctypes.c_int64)),
        ("mat_off", ctypes.POINTER(ctypes.c_int64)),
        ("vec_off", ctypes.POINTER(ctypes.c_int64)),
        ("piv_off", ctypes.POINTER(ctypes.c_int64)),
        ("status", ctypes.c_void_p),
        ("rank", ctypes.c_void_p),
        ("pivots", ctypes.c_void_p),
        ("basis", ctypes.c_void_p),
        ("shift", ctypes.c_void_p),
        ("kernel", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
        ("hash", ctypes.c_void_p),
    ]


class BatchParams(ctypes.Structure):
    _fields_ = [("chunk_log2", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32)]

    def __repr__(self):
        return f"BatchParams(chunk_log2={self.chunk_log2}, waves_per_cu={self.waves_per_cu})"


_batch_sigs_done = False
_hip = None


def _batch_lib():
    global _batch_sigs_done
    L = lib()
    if not _batch_sigs_done:
        vp, i32, u64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)
        L.hlf_batch_create.restype = i32
        L.hlf_batch_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vp)]
        L.hlf_batch_destroy.restype = i32
        L.hlf_batch_destroy.argtypes = [vp]
        L.hlf_batch_get_layout.restype = i32
        L.hlf_batch_get_layout.argtypes = [vp, ctypes.POINTER(_BatchLayout)]
        L.hlf_batch_factor_dense.restype = i32
        L.hlf_batch_factor_dense.argtypes = [vp, vp, vp]
        L.hlf_batch_enumerate.restype = i32
        L.hlf_batch_enumerate.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), u64p, u64p,
                                          ctypes.POINTER(vp), i32, vp]
        L.hlf_batch_enumerate_overlap.restype = i32
        L.hlf_batch_enumerate_overlap.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), u64p,
                                                  u64p, ctypes.POINTER(vp), i32, vp, vp, vp]
        L.hlf_batch_solve.restype = i32
        L.hlf_batch_solve.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_int32), u64p, u64p,
                                      ctypes.POINTER(vp), i32, vp]
        L.hlf_batch_reduce.restype = i32
        L.hlf_batch_reduce.argtypes = [vp, vp, i32, ctypes.POINTER(BatchParams), vp]
        L.hlf_batch_tune.restype = i32
        L.hlf_batch_tune.argtypes = [vp, vp, i32, ctypes.POINTER(BatchParams),
                                     ctypes.POINTER(ctypes.c_float), vp]
        L.hlf_batch_graph_capture.restype = i32
        L.hlf_batch_graph_capture.argtypes = [vp, vp, i32, ctypes.POINTER(BatchParams)]
        L.hlf_batch_graph_launch.restype = i32
        L.hlf_batch_graph_launch.argtypes = [vp, vp]
        L.hlf_batch_reduce_noalloc.restype = i32
        L.hlf_batch_reduce_noalloc.argtypes = [i32, i32, vp, vp, i32, vp] + [vp] * 8 + [vp]
        _batch_sigs_done = True
    return L


def _device_to_host(ptr: int, nbytes: int, dtype) -> np.ndarray:
    """Copy nbytes from a device pointer owned by the library (after a sync)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(nbytes // np.dtype(dtype).itemsize, dtype=dtype)
    if nbytes:
        rc = _hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), nbytes, 2)  # device to host
        if rc != 0:
            raise HlfError(HLF_EDEVICE, f"hipMemcpy failed ({rc})")
    return out


class Batch:
    """hlf_batch: many instances, one launch per stage (device arrays owned by the library)."""

    def __init__(self, ns):
        L = _batch_lib()
        ns = [int(x) for x in ns]
        arr = (ctypes.c_int32 * len(ns))(*ns)
        h = ctypes.c_void_p()
        _check(L.hlf_batch_create(len(ns), arr, ctypes.byref(h)), "hlf_batch_create")
        self._h = h
        self.ns = ns
        lay = _BatchLayout()
        _check(L.hlf_batch_get_layout(h, ctypes.byref(lay)), "hlf_batch_get_layout")
        I = lay.count
        self.count = I
        self.max_n = lay.max_n
        self.dense_bytes = lay.dense_bytes
        self.mat_words, self.vec_words, self.piv_entries = lay.mat_words, lay.vec_words, lay.piv_entries
        self.dense_off = np.ctypeslib.as_array(lay.dense_off, shape=(I,)).copy()
        self.mat_off = np.ctypeslib.as_array(lay.mat_off, shape=(I,)).copy()
        self.vec_off = np.ctypeslib.as_array(lay.vec_off, shape=(I,)).copy()
        self.piv_off = np.ctypeslib.as_array(lay.piv_off, shape=(I,)).copy()
        self.ptr = {k: getattr(lay, k) for k in ("status", "rank", "pivots", "basis", "shift",
                                                  "kernel", "counts", "hash")}

    def close(self):
        if getattr(self, "_h", None):
            _batch_lib().hlf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dense_input(self, mats, device=None) -> torch.Tensor:
        """Concatenate dense uint8 matrices in the batch's input layout, on the device."""
        host = np.zeros(self.dense_bytes, dtype=np.uint8)
        for i, A in enumerate(mats):
            n = self.ns[i]
            a = np.ascontiguousarray(A, dtype=np.uint8)
            if a.shape != (n, n):
                raise HlfError(HLF_EINVAL, f"instance {i} must be {n}x{n}")
            host[self.dense_off[i]:self.dense_off[i] + n * n] = a.reshape(-1)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        return torch.from_numpy(host).to(dev)

    def factor_dense(self, A_dev: torch.Tensor, stream=None):
        _check(_batch_lib().hlf_batch_factor_dense(self._h, _ptr(A_dev), _stream(stream)),
               "hlf_batch_factor_dense")

    def enumerate(self, inst, begin, count, outs, word_bits: int, stream=None):
        num = len(inst)
        ia = (ctypes.c_int32 * num)(*[int(x) for x in inst])
        ba = (ctypes.c_uint64 * num)(*[int(x) for x in begin])
        ca = (ctypes.c_uint64 * num)(*[int(x) for x in count])
        oa = (ctypes.c_void_p * num)(*[o.data_ptr() for o in outs])
        _check(_batch_lib().hlf_batch_enumerate(self._h, num, ia, ba, ca, oa, word_bits,
                                                _stream(stream)), "hlf_batch_enumerate")

    def enumerate_overlap(self, inst, begin, count, outs, word_bits: int, next_batch: "Batch",
                          A_next: torch.Tensor, stream=None):
        """Materialise this batch's tasks and factor `next_batch` in the same launch."""
        num = len(inst)
        ia = (ctypes.c_int32 * num)(*[int(x) for x in inst])
        ba = (ctypes.c_uint64 * num)(*[int(x) for x in begin])
        ca = (ctypes.c_uint64 * num)(*[int(x) for x in count])
        oa = (ctypes.c_void_p * num)(*[o.data_ptr() for o in outs])
        _check(_batch_lib().hlf_batch_enumerate_overlap(self._h, num, ia, ba, ca, oa, word_bits,
                                                        next_batch._h, _ptr(A_next),
                                                        _stream(stream)),
               "hlf_batch_enumerate_overlap")

    def solve(self, A_dev: torch.Tensor, inst, begin, count, outs, word_bits: int, stream=None):
        """Stage 1 + materialise of the listed instances in one launch."""
        num = len(inst)
        ia = (ctypes.c_int32 * num)(*[int(x) for x in inst])
        ba = (ctypes.c_uint64 * num)(*[int(x) for x in begin])
        ca = (ctypes.c_uint64 * num)(*[int(x) for x in count])
        oa = (ctypes.c_void_p * num)(*[o.data_ptr() for o in outs])
        _check(_batch_lib().hlf_batch_solve(self._h, _ptr(A_dev), num, ia, ba, ca, oa, word_bits,
                                            _stream(stream)), "hlf_batch_solve")

    def reduce(self, A_dev: torch.Tensor, max_rank: int, params: BatchParams | None = None,
               stream=None):
        p = ctypes.byref(params) if params is not None else None
        _check(_batch_lib().hlf_batch_reduce(self._h, _ptr(A_dev), max_rank, p, _stream(stream)),
               "hlf_batch_reduce")

    def tune(self, A_dev: torch.Tensor, max_rank: int, stream=None):
        best = BatchParams()
        ms = ctypes.c_float()
        _check(_batch_lib().hlf_batch_tune(self._h, _ptr(A_dev), max_rank, ctypes.byref(best),
                                           ctypes.byref(ms), _stream(stream)), "hlf_batch_tune")
        return best, float(ms.value)

    def graph_capture(self, A_dev: torch.Tensor, max_rank: int, params: BatchParams | None = None):
        p = ctypes.byref(params) if params is not None else None
        _check(_batch_lib().hlf_batch_graph_capture(self._h, _ptr(A_dev), max_rank, p),
               "hlf_batch_graph_capture")

    def graph_launch(self, stream=None):
        _check(_batch_lib().hlf_batch_graph_launch(self._h, _stream(stream)), "hlf_batch_graph_launch")

    # -- reading results (synchronise first) --
    def _read(self, key, nbytes, dtype):
        return _device_to_host(self.ptr[key], nbytes, dtype)

    def statuses(self) -> np.ndarray:
        torch.cuda.synchronize()
        return self._read("status", 4 * self.count, np.int32)

    def ranks(self) -> np.ndarray:
        torch.cuda.synchronize()
        return self._read("rank", 4 * self.count, np.int32)

    def records(self) -> list[dict]:
        """Every instance's record as Python ints (same layout as Factors.read)."""
        torch.cuda.synchronize()
        status = self._read("status", 4 * self.count, np.int32)
        rank = self._read("rank", 4 * self.count, np.int32)
        piv = self._read("pivots", 4 * self.piv_entries, np.int32)
        basis = self._read("basis", 8 * self.mat_words, np.uint64)
        shift = self._read("shift", 8 * self.vec_words, np.uint64)
        kern = self._read("kernel", 8 * self.mat_words, np.uint64)
        out = []
        for i, n in enumerate(self.ns):
            W = words_for(n)
            r = int(rank[i])
            mo, vo, po = int(self.mat_off[i]), int(self.vec_off[i]), int(self.piv_off[i])

            def vec(arr, off):
                return sum(int(arr[off + w]) << (64 * w) for w in range(W))

            rec = {"status": int(status[i]), "n": n, "words": W, "rank": r,
                   "pivots": [int(p) for p in piv[po:po + n]]}
            if rec["status"] == HLF_OK:
                rec["basis"] = [vec(basis, mo + k * W) for k in range(r)]
                rec["shift"] = vec(shift, vo)
                rec["kernel"] = [vec(kern, mo + j * W) for j in range(n - r)]
            out.append(rec)
        return out

    def reduce_results(self):
        """(counts per instance as uint64 arrays, hashes as Python ints)."""
        torch.cuda.synchronize()
        counts = self._read("counts", 8 * self.piv_entries, np.uint64)
        hashes = self._read("hash", 8 * self.count, np.uint64)
        return ([counts[int(self.piv_off[i]):int(self.piv_off[i]) + n] for i, n in enumerate(self.ns)],
                [int(h) for h in hashes])


def batch_reduce_noalloc(n_dev: torch.Tensor, max_n: int, A_dev: torch.Tensor, max_rank: int,
                         out: dict, params: BatchParams | None = None, stream=None):
    """hlf_batch_reduce_noalloc: factor + reduce of len(n_dev) instances into the
    caller's arrays ``out`` (keys status, rank, pivots, basis, shift, kernel
    (may be None), counts, hash; the layout of hlf_batch_get_layout)."""
    p = ctypes.byref(params) if params is not None else None
    k = out.get("kernel")
    _check(_batch_lib().hlf_batch_reduce_noalloc(
        int(n_dev.numel()), int(max_n), _ptr(n_dev), _ptr(A_dev), int(max_rank), p,
        _ptr(out["status"]), _ptr(out["rank"]), _ptr(out["pivots"]), _ptr(out["basis"]),
        _ptr(out["shift"]), _ptr(k) if k is not None else None, _ptr(out["counts"]),
        _ptr(out["hash"]), _stream(stream)), "hlf_batch_reduce_noalloc")
