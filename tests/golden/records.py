"""Canonical digest of a stage-1 record, used to store and compare the
records of many instances compactly.  Formatting only: no method arithmetic."""

from __future__ import annotations

import hashlib


def record_digest(rank: int, pivots, basis, shift: int, kernel) -> str:
    """First 16 hex digits of the sha256 of the record's canonical text:
    rank, the r pivots, the r basis vectors, the shift and the n - r kernel
    vectors, each vector as a hexadecimal integer."""
    parts = [str(int(rank)), ",".join(str(int(p)) for p in list(pivots)[:rank]),
             ",".join(format(int(b), "x") for b in basis), format(int(shift), "x"),
             ",".join(format(int(k), "x") for k in kernel)]
    return hashlib.sha256(";".join(parts).encode()).hexdigest()[:16]


def dense_digest(mats) -> str:
    """sha256 (16 hex digits) of the concatenated dense matrices and their sizes."""
    h = hashlib.sha256()
    for m in mats:
        h.update(int(m.shape[0]).to_bytes(4, "little"))
        h.update(m.astype("uint8").tobytes())
    return h.hexdigest()[:16]
