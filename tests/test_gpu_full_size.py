"""GPU parity at the measured sizes, in the launch configurations the
benchmark times, element by element against the oracle.

* Sampling (App. A): 65536 samples at n = 1024 (r = 953 and r = 1024), every
  word of every sample against the C oracle's sampler, for the SplitMix64
  stream and for explicit coefficients.  At this size each wave of the
  matrix-core kernel takes several 32-sample blocks.
* Membership (Section 1's definition, the ideal probabilities of Section 5):
  2^20 strings at n = 1024 -- exact samples, samples with one and with two
  flipped bits, and uniform strings, shuffled -- against the C oracle's check
  of q(k_f) = 2 <z, k_f> (mod 4) on the Ker(A) basis; plus 2^16 strings on the
  per-string kernel (n - r above 128).
* The headline step: 8 N=5 instances materialised as uint32 by the
  two-stream overlap launches (stage 1 of step k+2 carried by launch k),
  several steps, every word of both output sets against the C oracle.
* The 4096-instance batch: the tuned persistent factor + reduce kernel
  replayed from a HIP graph; every rank and stage-1 record, and the hash of
  every instance with r <= 28, against stored oracle results
  (tests/golden/config4_oracle.json, written by make_config4.py through the
  oracle only); counts against their closed form.
"""

import json
import os
import sys

import numpy as np
import pytest
import torch

from hlf_inputs import batch_instances, grid_instance, random_symmetric
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import gpu_factor, require_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "golden"))
sys.path.insert(0, ROOT)
from records import dense_digest, record_digest  # noqa: E402

MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _say(msg):
    print(msg, flush=True)


SAMPLE_CASES = {
    "grid N=32 p=0.5 seed 17 (r=953)": lambda: grid_instance(32, p=0.5, seed=17),
    "random n=1024 (r=1024)": lambda: random_symmetric(1024, 8, 0.5),
}


@pytest.mark.parametrize("name", list(SAMPLE_CASES))
def test_sample_65536_n1024_every_word(name):
    A = SAMPLE_CASES[name]()
    Fo = O.factor(A)
    r = Fo["rank"]
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK and int(F.rank.item()) == r
    num = 65536
    out = torch.empty((num, 16), dtype=torch.int64, device="cuda")
    for seed in (1, 0xFEEDFACE12345678):
        _say(f"[full] sample {name} seed={seed:#x} num={num}")
        out.fill_(-1)
        hlf.sample(F, seed, num, out=out)
        torch.cuda.synchronize()
        got = hlf.as_uint64(out)
        want = C.sample(Fo, seed, num)
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, f"{bad.size} samples differ, first {bad[:8].tolist()}"
    R64 = (r + 63) // 64
    rng = np.random.default_rng(r)
    coeffs = rng.integers(-(2**63), 2**63 - 1, size=(num, R64), dtype=np.int64)
    _say(f"[full] sample {name} explicit coefficients num={num}")
    out.fill_(-1)
    hlf.sample(F, 0, num, coeffs=torch.from_numpy(coeffs).cuda(), out=out)
    torch.cuda.synchronize()
    want = C.sample(Fo, 0, num, coeffs=coeffs.view(np.uint64))
    assert np.array_equal(hlf.as_uint64(out), want)


def test_sample_long_runs_of_blocks():
    """2^22 samples, so that every wave of the n > 192 sampler takes many
    32-sample blocks: the sparse path on the N=17 grid (n = 289, about 85
    blocks per wave), every word for the SplitMix64 stream; the matrix cores
    on a dense random n = 1024 matrix (about 170 blocks per wave), 4096 rows
    spread over the range for explicit coefficients; against the C oracle."""
    num = 1 << 22
    A = grid_instance(17, p=0.5, seed=4)
    Fo = O.factor(A)
    F, st = gpu_factor(A)
    W = Fo["words"]
    assert st == hlf.HLF_OK and int(F.rank.item()) == Fo["rank"]
    _say(f"[full] sample n=289 r={Fo['rank']} num={num}")
    out = hlf.sample(F, 0xC0FFEE, num)
    torch.cuda.synchronize()
    got = hlf.as_uint64(out).reshape(num, W)
    want = C.sample(Fo, 0xC0FFEE, num)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} samples differ, first {bad[:8].tolist()}"
    del out, got, want

    A = random_symmetric(1024, 8, 0.5)
    Fo = O.factor(A)
    F, st = gpu_factor(A)
    r = Fo["rank"]
    R64 = (r + 63) // 64
    rng = np.random.default_rng(29)
    coeffs = rng.integers(-(2**63), 2**63 - 1, size=(num, R64), dtype=np.int64)
    _say(f"[full] sample n=1024 r={r} explicit coefficients num={num}")
    out = torch.empty((num, 16), dtype=torch.int64, device="cuda")
    out.fill_(-1)
    hlf.sample(F, 0, num, coeffs=torch.from_numpy(coeffs).cuda(), out=out)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([np.arange(0, num, 1024), rng.integers(0, num, 2048), np.arange(num - 64, num)]))
    got = hlf.as_uint64(out)[rows]
    want = C.sample(Fo, 0, rows.size, coeffs=coeffs[rows].view(np.uint64))
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} of {rows.size} rows differ, first rows {rows[bad[:8]].tolist()}"


def _mixed_strings(Fo, n, num, seed):
    """num strings: a quarter exact samples, a quarter samples with one
    flipped bit, a quarter with two (possibly equal) flipped bits, the rest
    uniform; shuffled."""
    W = (n + 63) // 64
    q = num // 4
    rng = np.random.default_rng(seed)
    Z = np.zeros((num, W), dtype=np.uint64)
    Z[:3 * q] = C.sample(Fo, seed, 3 * q)
    for lo, hi in ((q, 2 * q), (2 * q, 3 * q), (2 * q, 3 * q)):
        bit = rng.integers(0, n, size=hi - lo)
        Z[np.arange(lo, hi), bit // 64] ^= np.left_shift(np.uint64(1), (bit % 64).astype(np.uint64))
    m = num - 3 * q
    U = rng.integers(0, 2**32, size=(m, 2 * W), dtype=np.uint64)
    Z[3 * q:] = (U[:, 0::2] << np.uint64(32)) | U[:, 1::2]
    if n % 64:
        Z[3 * q:, W - 1] &= np.uint64((1 << (n % 64)) - 1)
    return Z[rng.permutation(num)]


MEMBERSHIP_CASES = {
    # n - r = 71 kernel vectors: the matrix-core kernel (the benchmark's case)
    "grid N=32 p=0.5 seed 17, 2^20 strings": (lambda: grid_instance(32, p=0.5, seed=17), 1 << 20),
    # n - r above 128: the per-string kernel
    "random n=1024 rank <= 800, 2^16 strings": (
        lambda: _embedded_sym(1024, 800, 21), 1 << 16),
}


def _embedded_sym(n, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    A = np.zeros((n, n), dtype=np.uint8)
    A[np.ix_(idx, idx)] = random_symmetric(m, seed, density=0.5)
    return A


@pytest.mark.parametrize("name", list(MEMBERSHIP_CASES))
def test_membership_mixed_strings_n1024_every_flag(name):
    make, num = MEMBERSHIP_CASES[name]
    A = make()
    n = A.shape[0]
    Fo = O.factor(A)
    q = [O.q_form(A, O.bits_to_array(k, n)) for k in Fo["kernel"]]
    Z = _mixed_strings(Fo, n, num, seed=len(q))
    want = C.membership(Fo["kernel"], q, 16, Z)
    frac = float(want.mean())
    _say(f"[full] membership {name}: n-r={len(q)} members={frac:.3f}")
    assert 0.3 < frac < 0.9  # a genuine mix of members and non-members
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    out = torch.full((num,), 7, dtype=torch.uint8, device="cuda")
    hlf.membership(F, torch.from_numpy(Z.view(np.int64)).cuda(), out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} flags differ, first {bad[:8].tolist()}"


def test_headline_two_stream_overlap_steps_every_word():
    import bench

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    P = bench.headline_pipeline(hlf, torch, torch.device("cuda", 0), stream)
    Fos = [O.factor(m) for m in P.mats]
    assert P.ranks == [F["rank"] for F in Fos]
    for outs in P.out_sets:
        for o in outs:
            o.fill_(-1)
    torch.cuda.synchronize()
    steps = 2 * P.n_streams + 3  # warm-up launches + several steps on each stream
    for k in range(steps):
        _say(f"[full] headline step {k} stream {k % P.n_streams}")
        P.step(k)
    torch.cuda.synchronize()
    for Bk in P.Bs:
        assert all(st == hlf.HLF_OK for st in Bk.statuses())
        assert [int(r) for r in Bk.ranks()] == P.ranks
    for s, F in enumerate(Fos):
        want = C.enumerate_range(F, 0, 1 << F["rank"])[:, 0]
        for k, outs in enumerate(P.out_sets):
            got = outs[s].cpu().numpy().view(np.uint32).astype(np.uint64)
            assert np.array_equal(got, want), (s, k)


def test_config4_graph_replay_every_instance_against_oracle():
    with open(os.path.join(HERE, "golden", "config4_oracle.json")) as fh:
        gold = json.load(fh)
    insts = batch_instances(gold["count"], master_seed=gold["master_seed"])
    mats = [a for (_, _, _, a) in insts]
    assert dense_digest(mats) == gold["dense_sha16"]
    max_rank = gold["max_rank"]
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    stream = torch.cuda.Stream()
    _say("[full] config4 tune")
    params, _ = B.tune(A, max_rank, stream=stream)
    B.graph_capture(A, max_rank, params)
    for rep in range(2):
        _say(f"[full] config4 graph replay {rep} chunk_log2={params.chunk_log2} "
             f"waves_per_cu={params.waves_per_cu}")
        B.graph_launch(stream=stream)
        stream.synchronize()
        ranks = [int(r) for r in B.ranks()]
        assert ranks == gold["ranks"]
        counts, hashes = B.reduce_results()
        for i, r in enumerate(ranks):
            if r <= max_rank:
                assert format(hashes[i], "016x") == gold["hash"][str(i)], i
                want = [(1 << (r - 1)) if mats[i][j].any() else 0 for j in range(mats[i].shape[0])]
                assert [int(v) for v in counts[i]] == want, i
            else:
                assert hashes[i] == 0 and not counts[i].any(), i
    recs = B.records()
    for i, rec in enumerate(recs):
        assert rec["status"] == hlf.HLF_OK, i
        assert record_digest(rec["rank"], rec["pivots"], rec["basis"], rec["shift"],
                             rec["kernel"]) == gold["record_sha16"][i], i
    B.close()
