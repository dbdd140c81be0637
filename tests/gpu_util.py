"""Helpers for the GPU parity tests: run the HIP path, convert results."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2103_00693_amd import hlf


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    hlf.lib()  # raises if libhlf.so is missing


def device_matrix(A: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.uint8)).cuda()


def gpu_factor(A: np.ndarray, workgroup: bool = False, kernel: bool = True):
    """pack + factor on the GPU; returns (Factors, pack status)."""
    n = A.shape[0]
    Ad = device_matrix(A)
    rows, st = hlf.pack_dense(Ad)
    F = hlf.Factors(n, kernel=kernel)
    hlf.factor(rows, n, F, workgroup=workgroup)
    torch.cuda.synchronize()
    return F, int(st.item())


def oracle_rows(A: np.ndarray) -> np.ndarray:
    """Expected packed rows, written out from the definition of the layout."""
    n = A.shape[0]
    W = (n + 63) // 64
    out = np.zeros((n, W), dtype=np.uint64)
    for i in range(n):
        for j in range(n):
            if A[i, j]:
                out[i, j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return out


def words_to_ints(arr: np.ndarray) -> list[int]:
    """uint64 array [m, W] (or [m]) -> list of Python ints."""
    a = np.asarray(arr).view(np.uint64)
    if a.ndim == 1:
        return [int(x) for x in a]
    W = a.shape[1]
    return [sum(int(a[k, w]) << (64 * w) for w in range(W)) for k in range(a.shape[0])]


def narrow_to_u64(t: torch.Tensor) -> np.ndarray:
    """Materialised solutions (int16/int32/int64 tensor) -> uint64 numpy."""
    a = t.cpu().numpy()
    if a.dtype == np.int16:
        return a.view(np.uint16).astype(np.uint64)
    if a.dtype == np.int32:
        return a.view(np.uint32).astype(np.uint64)
    return a.view(np.uint64)
