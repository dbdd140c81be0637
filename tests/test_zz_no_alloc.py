"""GPU test of hlf_batch_reduce_noalloc, the allocation-free batched reduce:
its outputs equal hlf_batch_reduce's (records, counts, hashes) bit for bit, on
two calls in a row that share the library's scratch, the second with fewer
and smaller instances."""

import numpy as np
import pytest
import torch

from hlf_inputs import batch_instances
from paper_2103_00693_amd import hlf

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _outputs(ns):
    Ws = [hlf.words_for(n) for n in ns]
    piv = sum(ns)
    mat = sum(n * w for n, w in zip(ns, Ws))
    vec = sum(Ws)
    d = "cuda"
    return {"status": torch.full((len(ns),), 99, dtype=torch.int32, device=d),
            "rank": torch.full((len(ns),), -9, dtype=torch.int32, device=d),
            "pivots": torch.full((piv,), 7, dtype=torch.int32, device=d),
            "basis": torch.zeros(mat, dtype=torch.int64, device=d),
            "shift": torch.full((vec,), 5, dtype=torch.int64, device=d),
            "kernel": torch.zeros(mat, dtype=torch.int64, device=d),
            "counts": torch.full((piv,), -1, dtype=torch.int64, device=d),
            "hash": torch.full((len(ns),), -1, dtype=torch.int64, device=d)}


def _check_against_batch(mats, max_rank, params, label):
    ns = [m.shape[0] for m in mats]
    B = hlf.Batch(ns)
    A = B.dense_input(mats)
    B.reduce(A, max_rank, params)
    recs = B.records()
    counts_b, hashes_b = B.reduce_results()
    out = _outputs(ns)
    n_dev = torch.tensor(ns, dtype=torch.int32, device="cuda")
    print(f"[noalloc] {label}: {len(ns)} instances, max_n={max(ns)}", flush=True)
    hlf.batch_reduce_noalloc(n_dev, max(ns), A, max_rank, out, params)
    torch.cuda.synchronize()
    h = {k: v.cpu().numpy() for k, v in out.items()}
    for i, rec in enumerate(recs):
        n, W, r = ns[i], hlf.words_for(ns[i]), rec["rank"]
        po, mo, vo = int(B.piv_off[i]), int(B.mat_off[i]), int(B.vec_off[i])
        assert int(h["status"][i]) == rec["status"] == hlf.HLF_OK, (label, i)
        assert int(h["rank"][i]) == r, (label, i)
        assert [int(p) for p in h["pivots"][po:po + n]] == rec["pivots"], (label, i)

        def vec(arr, off):
            return sum(int(arr[off + w]) << (64 * w) for w in range(W))

        assert [vec(h["basis"].view(np.uint64), mo + k * W) for k in range(r)] == rec["basis"], (label, i)
        assert vec(h["shift"].view(np.uint64), vo) == rec["shift"], (label, i)
        assert [vec(h["kernel"].view(np.uint64), mo + j * W) for j in range(n - r)] == rec["kernel"], (label, i)
        assert np.array_equal(h["counts"][po:po + n].view(np.uint64), counts_b[i]), (label, i)
        assert int(h["hash"].view(np.uint64)[i]) == hashes_b[i], (label, i)
    B.close()
    return sum(1 for r in recs if r["rank"] <= max_rank)


def test_noalloc_equals_batch_reduce_twice_second_smaller():
    first = [a for (_, _, _, a) in batch_instances(600, master_seed=3)]
    reduced = _check_against_batch(first, 22, hlf.BatchParams(14, 4), "first call")
    assert reduced > 50
    second = [a for (N, _, _, a) in batch_instances(400, master_seed=4) if N <= 7][:150]
    assert max(m.shape[0] for m in second) <= 64 < max(m.shape[0] for m in first)
    _check_against_batch(second, 20, None, "second call")


def test_noalloc_host_errors():
    n_dev = torch.full((4,), 16, dtype=torch.int32, device="cuda")
    A = torch.zeros(4 * 256, dtype=torch.uint8, device="cuda")
    out = _outputs([16] * 4)
    for count_ok, max_n, max_rank, params in ((True, 193, 20, None), (True, 0, 20, None),
                                             (True, 16, 63, None), (True, 16, 20, hlf.BatchParams(9, 4))):
        with pytest.raises(hlf.HlfError):
            hlf.batch_reduce_noalloc(n_dev, max_n, A, max_rank, out, params)
    big = torch.full((16385,), 16, dtype=torch.int32, device="cuda")
    with pytest.raises(hlf.HlfError):
        hlf.batch_reduce_noalloc(big, 16, A, 20, out)
    torch.cuda.synchronize()
    assert bool((out["status"] == 99).all())  # nothing ran
