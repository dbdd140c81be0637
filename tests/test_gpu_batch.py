"""GPU parity of the batch layer: fused pack+factor for many instances, the
multi-instance materialise launch, and the persistent factor+reduce kernel
(plain, tuned, every launch shape, and replayed from a HIP graph) against the
oracle and against the single-instance entry points."""

import numpy as np
import pytest
import torch

from hlf_inputs import CONFIG2_SEEDS, batch_instances, grid_instance, random_symmetric
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import gpu_factor, narrow_to_u64, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def mixed_batch(seed=0, count=48, Ns=range(3, 13)):
    rng = np.random.default_rng(seed)
    mats = []
    for k in range(count):
        N = int(rng.choice(list(Ns)))
        p = float(rng.choice([0.3, 0.5, 1.0]))
        mats.append(grid_instance(N, p=p, seed=int(rng.integers(0, 2**31))))
    return mats


def check_record(got, ref, name):
    assert got["status"] == hlf.HLF_OK, name
    r = ref["rank"]
    assert got["rank"] == r, name
    assert got["pivots"][:r] == ref["pivots"] and all(p == -1 for p in got["pivots"][r:]), name
    assert got["basis"] == ref["basis"], name
    assert got["shift"] == ref["shift"], name
    assert got["kernel"] == ref["kernel"], name


def test_batch_factor_mixed_sizes_and_invalid():
    mats = [grid_instance(5, seed=1), np.zeros((1, 1), np.uint8), random_symmetric(64, 3),
            random_symmetric(65, 4), grid_instance(12, p=0.5, seed=2), random_symmetric(192, 5),
            random_symmetric(193, 6), random_symmetric(300, 7, 0.1), grid_instance(3, b="101010101")]
    bad = grid_instance(4, seed=9)
    bad[0, 7] = 1  # not symmetric
    mats.append(bad)
    bad2 = random_symmetric(250, 8)
    bad2[3, 3] = 2  # not 0/1 (a large instance: pack + workgroup factor path)
    mats.append(bad2)
    bad3 = random_symmetric(40, 9)
    bad3[5, 5] = 3  # not 0/1 (wave path)
    mats.append(bad3)
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    print("[batch] factor_dense mixed", flush=True)
    B.factor_dense(A)
    recs = B.records()
    for i, m in enumerate(mats[:-3]):
        check_record(recs[i], O.factor(m), f"instance {i} n={m.shape[0]}")
    for i in (len(mats) - 3, len(mats) - 2, len(mats) - 1):
        assert recs[i]["status"] == hlf.HLF_ENOTSYM, i
    B.close()


@pytest.mark.parametrize("word_bits", [32, 64])
def test_batch_enumerate_config2(word_bits):
    mats = [grid_instance(5, seed=s) for s in CONFIG2_SEEDS]
    B = hlf.Batch([25] * len(mats))
    A = B.dense_input(mats)
    B.factor_dense(A)
    ranks = B.ranks()
    dt = torch.int32 if word_bits == 32 else torch.int64
    outs = [torch.empty(1 << int(r), dtype=dt, device="cuda") for r in ranks]
    print(f"[batch] enumerate config2 wb={word_bits}", flush=True)
    B.enumerate(list(range(8)), [0] * 8, [1 << int(r) for r in ranks], outs, word_bits)
    torch.cuda.synchronize()
    for s, (m, o, r) in enumerate(zip(mats, outs, ranks)):
        Fo = O.factor(m)
        assert Fo["rank"] == r
        ref = C.enumerate_range(Fo, 0, 1 << int(r))[:, 0]
        assert np.array_equal(narrow_to_u64(o), ref), s


def test_batch_enumerate_mixed_tasks_and_fallbacks():
    mats = [grid_instance(4, seed=0), grid_instance(5, seed=3), grid_instance(3, p=0.5, seed=1)]
    B = hlf.Batch([16, 25, 9])
    A = B.dense_input(mats)
    B.factor_dense(A)
    ranks = [int(r) for r in B.ranks()]
    Fs = [O.factor(m) for m in mats]
    # instance 1 twice: an aligned chunk and an unaligned chunk (general path)
    inst = [0, 1, 1, 2]
    begin = [4, 1 << 10, 3, 0]
    count = [(1 << ranks[0]) - 4, 12345, 1000, 1 << ranks[2]]
    outs = [torch.empty(c, dtype=torch.int32, device="cuda") for c in count]
    print("[batch] enumerate mixed tasks", flush=True)
    B.enumerate(inst, begin, count, outs, 32)
    torch.cuda.synchronize()
    for k in range(4):
        ref = C.enumerate_range(Fs[inst[k]], begin[k], count[k])[:, 0]
        assert np.array_equal(narrow_to_u64(outs[k]), ref), k
    # a bad range poisons only its own instance
    o = torch.full((8,), -5, dtype=torch.int32, device="cuda")
    B.enumerate([2], [(1 << ranks[2]) - 4], [8], [o], 32)
    st = B.statuses()
    assert st[2] == hlf.HLF_ERANGE and st[0] == hlf.HLF_OK and st[1] == hlf.HLF_OK
    assert bool((o == -5).all())


def reduce_reference(mats, max_rank):
    refs = []
    for m in mats:
        Fo = O.factor(m)
        if Fo["rank"] <= max_rank:
            c, h, _ = C.reduce_range(Fo, 0, 1 << Fo["rank"])
            refs.append((Fo["rank"], [int(v) for v in c], h))
        else:
            refs.append((Fo["rank"], [0] * m.shape[0], 0))
    return refs


def check_reduce(B, refs, name):
    counts, hashes = B.reduce_results()
    ranks = B.ranks()
    for i, (r, c, h) in enumerate(refs):
        assert ranks[i] == r, (name, i)
        assert [int(v) for v in counts[i]] == c, (name, i)
        assert hashes[i] == h, (name, i)


def test_batch_reduce_all_launch_shapes_agree():
    mats = mixed_batch(seed=1, count=40)
    max_rank = 22
    refs = reduce_reference(mats, max_rank)
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    for chunk in (10, 14, 20):
        for waves in (1, 4, 16):
            print(f"[batch] reduce chunk_log2={chunk} waves={waves}", flush=True)
            B.reduce(A, max_rank, hlf.BatchParams(chunk, waves))
            check_reduce(B, refs, f"chunk={chunk} waves={waves}")
    recs = B.records()
    for i, m in enumerate(mats[:10]):
        check_record(recs[i], O.factor(m), f"instance {i}")
    best, ms = B.tune(A, max_rank)
    print(f"[batch] tuned {best} {ms:.3f} ms", flush=True)
    B.reduce(A, max_rank)
    check_reduce(B, refs, "tuned")
    B.close()


def test_batch_reduce_rejects_chunk_totals_beyond_the_queue_word():
    # the queue counts chunks in 40 bits: count * 2^(max_rank - chunk_log2) must stay below 2^40
    mats = mixed_batch(seed=5, count=300, Ns=range(3, 6))
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    for max_rank, chunk in ((62, 10), (50, 10), (62, 30)):
        with pytest.raises(hlf.HlfError):
            B.reduce(A, max_rank, hlf.BatchParams(chunk, 4))
        with pytest.raises(hlf.HlfError):
            B.graph_capture(A, max_rank, hlf.BatchParams(chunk, 4))
    print("[batch] claim limit: accepted shape", flush=True)
    B.reduce(A, 20, hlf.BatchParams(10, 4))  # 300 * 2^10 chunks fit
    torch.cuda.synchronize()
    assert all(s == hlf.HLF_OK for s in B.statuses())
    B.close()


def test_batch_reduce_w1_only_batch():
    mats = [grid_instance(N, p=p, seed=s) for N, p, s in
            [(3, 1.0, 0), (4, 0.5, 1), (5, 1.0, 2), (6, 0.3, 3), (2, 1.0, 4), (1, 1.0, 5)]]
    mats.append(np.zeros((8, 8), np.uint8))
    refs = reduce_reference(mats, 26)
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    print("[batch] reduce W=1 batch", flush=True)
    B.reduce(A, 26, hlf.BatchParams(16, 8))
    check_reduce(B, refs, "w1")


def test_batch_graph_replays_match_eager():
    mats = mixed_batch(seed=2, count=24, Ns=range(3, 9))
    max_rank = 20
    refs = reduce_reference(mats, max_rank)
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    B.reduce(A, max_rank, hlf.BatchParams(14, 4))
    check_reduce(B, refs, "eager")
    B.graph_capture(A, max_rank, hlf.BatchParams(14, 4))
    for rep in range(4):
        print(f"[batch] graph replay {rep}", flush=True)
        x = torch.arange(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert int(x.item()) == 499500
        B.graph_launch()
        torch.cuda.synchronize()
        check_reduce(B, refs, f"replay {rep}")
    B.close()


def test_batch_config4_matches_plain_launches():
    insts = batch_instances(4096, master_seed=0)
    mats = [a for (_, _, _, a) in insts]
    max_rank = 28
    B = hlf.Batch([m.shape[0] for m in mats])
    A = B.dense_input(mats)
    print("[batch] config4 batched reduce", flush=True)
    B.reduce(A, max_rank)
    counts_b, hashes_b = B.reduce_results()
    ranks_b = [int(r) for r in B.ranks()]
    assert all(s == hlf.HLF_OK for s in B.statuses())
    # per-instance plain launches: factor every instance, then reduce the small-rank ones
    print("[batch] config4 plain launches", flush=True)
    Fs = []
    for m in mats:
        n = m.shape[0]
        rows, _ = hlf.pack_dense(torch.from_numpy(m).cuda())
        Fs.append(hlf.factor(rows, n, hlf.Factors(n, kernel=False)))
    torch.cuda.synchronize()
    ranks_p = [int(F.rank.item()) for F in Fs]
    assert ranks_p == ranks_b
    outs = {}
    for i, F in enumerate(Fs):
        if ranks_p[i] <= max_rank:
            outs[i] = hlf.enumerate_reduce(F, 0, 1 << ranks_p[i], want_xorfold=False)
    torch.cuda.synchronize()
    for i, (c, h, _) in outs.items():
        assert np.array_equal(hlf.as_uint64(c), counts_b[i]), i
        assert int(hlf.as_uint64(h)[0]) == hashes_b[i], i
    for i in range(len(mats)):
        if ranks_b[i] > max_rank:
            assert hashes_b[i] == 0 and not counts_b[i].any()
    # the oracle on a sample: closed-form counts for every reduced instance, exact
    # records and hashes for a few
    for i in outs:
        r = ranks_b[i]
        want = [(1 << (r - 1)) if mats[i][j].any() else 0 for j in range(mats[i].shape[0])]
        assert [int(v) for v in counts_b[i]] == want, i
    small = [i for i in outs if ranks_b[i] <= 18][:30]
    recs = B.records()
    for i in small:
        Fo = O.factor(mats[i])
        check_record(recs[i], Fo, f"config4 instance {i}")
        _, h, _ = C.reduce_range(Fo, 0, 1 << Fo["rank"])
        assert hashes_b[i] == h, i
    B.close()


@pytest.mark.parametrize("word_bits", [32, 64])
def test_batch_solve_one_launch(word_bits):
    mats = [grid_instance(5, seed=s) for s in CONFIG2_SEEDS]
    Fs = [O.factor(m) for m in mats]
    B = hlf.Batch([25] * len(mats))
    A = B.dense_input(mats)
    dt = torch.int32 if word_bits == 32 else torch.int64
    counts = [1 << F["rank"] for F in Fs]
    outs = [torch.empty(c, dtype=dt, device="cuda") for c in counts]
    for rep in range(3):
        for o in outs:
            o.fill_(-1)
        print(f"[batch] solve wb={word_bits} rep={rep}", flush=True)
        B.solve(A, list(range(8)), [0] * 8, counts, outs, word_bits)
        torch.cuda.synchronize()
        for s, (F, o) in enumerate(zip(Fs, outs)):
            assert np.array_equal(narrow_to_u64(o), C.enumerate_range(F, 0, counts[s])[:, 0]), (rep, s)
    recs = B.records()
    for s, F in enumerate(Fs):
        check_record(recs[s], F, f"solve record {s}")
    # new matrices in the same input buffer: the next launch factors them again
    mats2 = [mats[(s + 1) % 8] for s in range(8)]
    A2 = B.dense_input(mats2)
    A.copy_(A2)
    counts2 = [counts[(s + 1) % 8] for s in range(8)]
    outs2 = [torch.empty(c, dtype=dt, device="cuda") for c in counts2]
    B.solve(A, list(range(8)), [0] * 8, counts2, outs2, word_bits)
    torch.cuda.synchronize()
    for s in range(8):
        F = Fs[(s + 1) % 8]
        assert np.array_equal(narrow_to_u64(outs2[s]), C.enumerate_range(F, 0, counts2[s])[:, 0]), s


def test_batch_solve_single_tiny_instance_u16():
    # the one-launch form of the N=4 workload: a batch of one n = 16 instance
    A0 = grid_instance(4, seed=0)
    F = O.factor(A0)
    total = 1 << F["rank"]
    B = hlf.Batch([16])
    A = B.dense_input([A0])
    out = torch.full((total,), -1, dtype=torch.int16, device="cuda")
    for rep in range(3):
        print(f"[batch] solve u16 single rep={rep}", flush=True)
        B.solve(A, [0], [0], [total], [out], 16)
        torch.cuda.synchronize()
        assert B.statuses()[0] == hlf.HLF_OK
        assert np.array_equal(narrow_to_u64(out), C.enumerate_range(F, 0, total)[:, 0]), rep
    check_record(B.records()[0], F, "solve u16 record")


def test_batch_solve_partial_ranges_and_errors():
    mats = [grid_instance(4, seed=0), grid_instance(5, seed=2), grid_instance(3, p=0.5, seed=4)]
    Fs = [O.factor(m) for m in mats]
    B = hlf.Batch([16, 25, 9])
    A = B.dense_input(mats)
    inst = [1, 0, 1, 2]
    begin = [0, 8, 1 << 20, 0]
    count = [1 << 20, (1 << Fs[0]["rank"]) - 8, 777, 1 << Fs[2]["rank"]]
    outs = [torch.empty(c, dtype=torch.int32, device="cuda") for c in count]
    print("[batch] solve partial", flush=True)
    B.solve(A, inst, begin, count, outs, 32)
    torch.cuda.synchronize()
    for k in range(4):
        ref = C.enumerate_range(Fs[inst[k]], begin[k], count[k])[:, 0]
        assert np.array_equal(narrow_to_u64(outs[k]), ref), k
    # out-of-range task: its instance gets HLF_ERANGE, the other instance is intact
    o1 = torch.full((64,), -9, dtype=torch.int32, device="cuda")
    o2 = torch.empty(1 << Fs[0]["rank"], dtype=torch.int32, device="cuda")
    B.solve(A, [2, 0], [(1 << Fs[2]["rank"]) - 8, 0], [64, 1 << Fs[0]["rank"]], [o1, o2], 32)
    st = B.statuses()
    assert st[2] == hlf.HLF_ERANGE and st[0] == hlf.HLF_OK
    assert bool((o1 == -9).all())
    assert np.array_equal(narrow_to_u64(o2), C.enumerate_range(Fs[0], 0, 1 << Fs[0]["rank"])[:, 0])
    # host-detected: n > word_bits, misaligned begin
    with pytest.raises(hlf.HlfError):
        B.solve(A, [1], [0], [16], [torch.empty(16, dtype=torch.int16, device="cuda")], 16)
    with pytest.raises(hlf.HlfError):
        B.solve(A, [0], [3], [16], [torch.empty(16, dtype=torch.int32, device="cuda")], 32)


def test_batch_enumerate_overlap_pipeline():
    mats = [grid_instance(5, seed=s) for s in CONFIG2_SEEDS[:4]] + [grid_instance(4, seed=1)]
    Fs = [O.factor(m) for m in mats]
    ns = [m.shape[0] for m in mats]
    Bs = [hlf.Batch(ns), hlf.Batch(ns)]
    A = Bs[0].dense_input(mats)
    Bs[0].factor_dense(A)
    counts = [1 << F["rank"] for F in Fs]
    outs = [torch.empty(c, dtype=torch.int32, device="cuda") for c in counts]
    refs = [C.enumerate_range(F, 0, c)[:, 0] for F, c in zip(Fs, counts)]
    for k in range(4):
        j = k % 2
        for o in outs:
            o.fill_(-1)
        print(f"[batch] overlap step {k}", flush=True)
        Bs[j].enumerate_overlap(list(range(5)), [0] * 5, counts, outs, 32, Bs[1 - j], A)
        torch.cuda.synchronize()
        for s, o in enumerate(outs):
            assert np.array_equal(narrow_to_u64(o), refs[s]), (k, s)
        recs = Bs[1 - j].records()  # factored by this launch
        for s, F in enumerate(Fs):
            check_record(recs[s], F, f"overlap step {k} instance {s}")
    with pytest.raises(hlf.HlfError):
        Bs[0].enumerate_overlap([0], [0], [16], [outs[0]], 32, Bs[0], A)


@pytest.mark.parametrize("S", [2, 3])
def test_batch_enumerate_overlap_several_streams(S):
    # S streams take the steps in turn; launch k materialises record set
    # k % 2S and factors record set (k + S) % 2S for the next launch on its
    # own stream, writing output set k % S.  S launches run at once and every
    # one of them must still produce the full solution sets and records.
    mats = [grid_instance(5, seed=s) for s in CONFIG2_SEEDS[:3]] + [grid_instance(4, seed=2)]
    Fs = [O.factor(m) for m in mats]
    ns = [m.shape[0] for m in mats]
    Bs = [hlf.Batch(ns) for _ in range(2 * S)]
    A = Bs[0].dense_input(mats)
    for Bk in Bs[:S]:
        Bk.factor_dense(A)
    torch.cuda.synchronize()
    counts = [1 << F["rank"] for F in Fs]
    refs = [C.enumerate_range(F, 0, c)[:, 0] for F, c in zip(Fs, counts)]
    out_sets = [[torch.full((c,), -1, dtype=torch.int32, device="cuda") for c in counts]
                for _ in range(S)]
    streams = [torch.cuda.Stream() for _ in range(S)]
    steps = 5 * S
    print(f"[batch] {S}-stream overlap, {steps} steps", flush=True)
    for k in range(steps):
        Bs[k % (2 * S)].enumerate_overlap(list(range(len(mats))), [0] * len(mats), counts,
                                          out_sets[k % S], 32, Bs[(k + S) % (2 * S)], A,
                                          stream=streams[k % S])
    torch.cuda.synchronize()
    for outs in out_sets:
        for s, o in enumerate(outs):
            assert np.array_equal(narrow_to_u64(o), refs[s]), s
    for j, Bk in enumerate(Bs):
        recs = Bk.records()
        for s, F in enumerate(Fs):
            check_record(recs[s], F, f"{S}-stream record set {j} instance {s}")
