"""MI355X (gfx950) implementation of the FS2D HLF two-stage scheme.

The computation runs in the HIP kernels of ``libhlf.so`` (C ABI:
``include/hlf.h``); ``hlf`` is its ctypes binding.
"""

from .hlf import (  # noqa: F401
    EXPORTED,
    Batch,
    BatchParams,
    Factors,
    HlfError,
    as_uint64,
    enumerate_circuit,
    enumerate_reduce,
    enumerate_solutions,
    factor,
    lib,
    pack_dense,
    sample,
    status_string,
    words_for,
)
