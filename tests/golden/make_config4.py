"""Writes the oracle's results for the 4096-instance batch workload
(grid side N ~ U{3..12}, edge probability p ~ U{0.3, 0.5, 1.0}, diagonal
Bernoulli(0.5), master seed 0): every instance's rank and stage-1 record
digest, and the hash of the full solution set of every instance with
r <= 28.  The per-qubit counts of those instances have a closed form
(2^(r-1) per nonzero row of A) that the tests check directly.

Calls only the oracle (test infrastructure) and the input generator.  Takes
several minutes on 8 cores.  Run from the repository root:
    python tests/golden/make_config4.py
"""

from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from hlf_inputs import batch_instances  # noqa: E402
from oracle import c_oracle, hlf_oracle  # noqa: E402
from records import dense_digest, record_digest  # noqa: E402

COUNT = 4096
MASTER_SEED = 0
MAX_RANK = 28


def _factor(A):
    F = hlf_oracle.factor(A)
    return F


def main():
    t0 = time.time()
    insts = batch_instances(COUNT, master_seed=MASTER_SEED)
    mats = [a for (_, _, _, a) in insts]
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        Fs = pool.map(_factor, mats, chunksize=16)
    print(f"factored {len(Fs)} instances in {time.time() - t0:.1f} s", flush=True)
    ranks = [F["rank"] for F in Fs]
    digests = [record_digest(F["rank"], F["pivots"], F["basis"], F["shift"], F["kernel"]) for F in Fs]
    hashes = {}
    small = [i for i, r in enumerate(ranks) if r <= MAX_RANK]
    total = sum(1 << ranks[i] for i in small)
    for k, i in enumerate(small):
        hashes[str(i)] = format(c_oracle.hash_range(Fs[i], 0, 1 << ranks[i]), "016x")
        if k % 100 == 0:
            print(f"hashed {k}/{len(small)} ({time.time() - t0:.1f} s)", flush=True)
    out = {
        "_source": "oracle results for batch_instances(4096, master_seed=0): hlf_oracle.factor "
                   "(rank, record digest of tests/golden/records.py) for every instance, "
                   "c_oracle.hash_range over all 2^r solutions for every r <= 28; written by "
                   "tests/golden/make_config4.py",
        "count": COUNT, "master_seed": MASTER_SEED, "max_rank": MAX_RANK,
        "dense_sha16": dense_digest(mats),
        "Ns": [int(N) for (N, _, _, _) in insts],
        "ranks": ranks,
        "record_sha16": digests,
        "reduced": len(small),
        "solutions": total,
        "hash": hashes,
    }
    with open(os.path.join(HERE, "config4_oracle.json"), "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
        fh.write("\n")
    print(f"wrote {len(small)} hashes ({total} solutions) in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
