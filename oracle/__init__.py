"""CPU oracle for the FS2D HLF hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import, call, link or execute anything in this package.  The product path
(the HIP library and its Python binding) never touches it and shares no code
with it: no kernels, headers, helpers, tables or constants.

Contents
--------
``hlf_oracle``  plain Python/numpy definitions: GF(2) factorisation, the
                canonical shift, enumeration by direct definition and by the
                paper's literal stage-2 circuit, reduction, sampling, brute force
                over the problem definition and a dense state-vector simulation
                of the quantum circuit.
``c_oracle``    ctypes loader for ``hlf_oracle.c``: the same per-index
                definitions in plain C (OpenMP over indices), for ranges too
                long for Python and for the CPU baseline timing.
``build``       compiles ``hlf_oracle.c`` with gcc.

Parity status of each function is listed in the header of ``hlf_oracle``.
"""
