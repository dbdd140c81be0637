"""Writes the stored expected values that are too slow to recompute per test.

Calls only the oracle (test infrastructure).  Run from the repository root:
    python tests/golden/make_golden.py
"""

from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import c_oracle  # noqa: E402


def main():
    # A full-rank instance has every bit string as a solution (Section 3), so
    # the order-independent hash of its solution set is the plain sum of h(z)
    # over all z < 2^n, whatever basis and order an implementation uses.
    out = {"_source": "sum of h(z) mod 2^64 over all z in [0, 2^n), written by "
                      "tests/golden/make_golden.py through oracle.c_oracle.identity_hash"}
    for n in (16, 24, 36):
        out[f"identity_hash_n{n}"] = hex(c_oracle.identity_hash(0, 1 << n))
    with open(os.path.join(HERE, "identity_hash.json"), "w") as fh:
        json.dump(out, fh, indent=2)
        fh.write("\n")
    print(out)


if __name__ == "__main__":
    main()
