"""GPU parity of reduce mode (hlf_enumerate_reduce) and sampling (hlf_sample).

Reduce: per-qubit counts, the order-independent hash and the XOR-fold equal the
oracle's plain loops on small ranges and on random 2^20-index chunks of the
N=6 p=0.5 instances; full ranges meet the closed-form counts; the full-rank
36-qubit instance (2^36 solutions) meets the stored identity hash.
Sampling: exact bits against the oracle's independent SplitMix64 stream, kernel
equations for every sample at n = 1024, and uniformity.
"""

import json
import os

import numpy as np
import pytest
import torch

from hlf_inputs import CONFIG3_SEEDS, grid_instance, paper_diagonal, random_symmetric
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import gpu_factor, require_gpu, words_to_ints

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _embedded(n, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    A = np.zeros((n, n), dtype=np.uint8)
    A[np.ix_(idx, idx)] = random_symmetric(m, seed, density=0.3)
    return A


def gpu_reduce(F, begin, count, accumulate=False, outs=None):
    counts, h, xf = outs if outs else (None, None, None)
    counts, h, xf = hlf.enumerate_reduce(F, begin, count, accumulate=accumulate,
                                         counts=counts, hash_out=h, xorfold=xf)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_OK
    return counts, h, xf


def as_ints(counts, h, xf):
    return ([int(c) for c in hlf.as_uint64(counts)], int(hlf.as_uint64(h)[0]),
            words_to_ints(hlf.as_uint64(xf).reshape(1, -1))[0])


def test_reduce_small_ranges_vs_python_oracle():
    for name, A in [("2x2 b=1011", grid_instance(2, b="1011")), ("config1", grid_instance(4, seed=0)),
                    ("3x3 m=2", grid_instance(3, b=paper_diagonal(9, 2))), ("zero n=3", np.zeros((3, 3), np.uint8))]:
        Fo = O.factor(A)
        r = Fo["rank"]
        F, _ = gpu_factor(A)
        for begin, count in [(0, 1 << r), (1, (1 << r) - 1), ((1 << r) // 3, (1 << r) // 3)]:
            if count <= 0:
                continue
            print(f"[reduce] {name} r={r} begin={begin} count={count}", flush=True)
            got = as_ints(*gpu_reduce(F, begin, count))
            c2, h2, x2 = O.reduce_range(Fo, begin, count)
            assert got == (c2, h2, x2)


@pytest.mark.parametrize("seed", CONFIG3_SEEDS)
def test_config3_random_chunks_and_closed_form(seed):
    A = grid_instance(6, p=0.5, seed=seed)
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    rng = np.random.default_rng(1000 + seed)
    for _ in range(16):
        begin = int(rng.integers(0, (1 << r) - (1 << 20)))
        print(f"[reduce] config3 seed={seed} r={r} chunk begin={begin}", flush=True)
        got = as_ints(*gpu_reduce(F, begin, 1 << 20))
        c, h, xf = C.reduce_range(Fo, begin, 1 << 20)
        assert got == ([int(v) for v in c], h, int(xf[0]))
    print(f"[reduce] config3 seed={seed} full 2^{r}", flush=True)
    counts, h, xf = as_ints(*gpu_reduce(F, 0, 1 << r))
    for j in range(36):
        assert counts[j] == ((1 << (r - 1)) if A[j].any() else 0), j
    assert xf == 0
    # additivity: uneven pieces accumulated == one call
    cuts = sorted(set([0, 1 << r] + [int(x) for x in rng.integers(1, 1 << r, size=6)]))
    outs = hlf.enumerate_reduce(F, 0, 0)  # zeroed outputs
    for a, b in zip(cuts[:-1], cuts[1:]):
        gpu_reduce(F, a, b - a, accumulate=True, outs=outs)
    assert as_ints(*outs) == (counts, h, xf)


def test_full_rank_36_identity_hash():
    with open(os.path.join(ROOT, "tests", "golden", "identity_hash.json")) as fh:
        gold = json.load(fh)
    A = grid_instance(6, b="1" * 36)
    F, _ = gpu_factor(A)
    assert int(F.rank.item()) == 36
    print("[reduce] full rank n=36, 2^36 solutions", flush=True)
    counts, h, xf = as_ints(*gpu_reduce(F, 0, 1 << 36))
    assert h == int(gold["identity_hash_n36"], 16)
    assert counts == [1 << 35] * 36
    assert xf == 0


def test_zero_count_overwrite_and_erange():
    A = grid_instance(4, seed=0)
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    counts = torch.full((16,), 5, dtype=torch.int64, device="cuda")
    h = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    xf = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    hlf.enumerate_reduce(F, 0, 0, counts=counts, hash_out=h, xorfold=xf)
    torch.cuda.synchronize()
    assert int(counts.abs().sum().item()) == 0 and int(h.item()) == 0 and int(xf.item()) == 0
    counts.fill_(9)
    print("[reduce] erange", flush=True)
    hlf.enumerate_reduce(F, 1, 1 << Fo["rank"], counts=counts, hash_out=h, xorfold=xf)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_ERANGE
    assert bool((counts == 9).all())


@pytest.mark.parametrize("n,m,seed", [(65, 30, 1), (130, 24, 2), (1024, 22, 3)])
def test_reduce_multiword(n, m, seed):
    A = _embedded(n, m, seed)
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    for begin, count in [(0, 1 << r), (7, min((1 << r) - 7, 100000))]:
        print(f"[reduce] multiword n={n} r={r} begin={begin} count={count}", flush=True)
        counts, h, xf = gpu_reduce(F, begin, count)
        c2, h2, x2 = C.reduce_range(Fo, begin, count)
        assert [int(v) for v in hlf.as_uint64(counts)] == [int(v) for v in c2]
        assert int(hlf.as_uint64(h)[0]) == h2
        assert np.array_equal(hlf.as_uint64(xf), x2)


# -- sampling -------------------------------------------------------------------

@pytest.mark.parametrize("name,A", [
    ("config1", grid_instance(4, seed=0)),
    ("config3 seed0", grid_instance(6, p=0.5, seed=0)),
    ("n=100 random", random_symmetric(100, 5, 0.5)),
    ("grid N=20", grid_instance(20, p=0.5, seed=3)),
    ("grid N=32", grid_instance(32, p=0.5, seed=4)),
    ("zero n=7", np.zeros((7, 7), dtype=np.uint8)),
])
def test_sample_matches_oracle_stream(name, A):
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    seed = 0xDEADBEEF12345
    num = 257
    print(f"[sample] {name} r={Fo['rank']} num={num}", flush=True)
    out = hlf.sample(F, seed, num)
    torch.cuda.synchronize()
    got = words_to_ints(hlf.as_uint64(out).reshape(num, F.words))
    assert got == O.sample(Fo, seed, num)


def test_sample_explicit_coefficients():
    A = grid_instance(10, p=0.5, seed=9)
    Fo = O.factor(A)
    r = Fo["rank"]
    R64 = (r + 63) // 64
    F, _ = gpu_factor(A)
    rng = np.random.default_rng(3)
    coeffs = rng.integers(0, 2**63, size=(100, R64), dtype=np.int64)
    coeffs[:, 0] ^= rng.integers(0, 2, size=100, dtype=np.int64) << 63
    out = hlf.sample(F, 0, 100, coeffs=torch.from_numpy(coeffs).cuda())
    torch.cuda.synchronize()
    cints = words_to_ints(coeffs.view(np.uint64))
    assert words_to_ints(hlf.as_uint64(out).reshape(100, F.words)) == O.sample(Fo, 0, 100, coeffs=cints)


def test_sample_65536_at_n1024_satisfy_kernel_equations():
    A = grid_instance(32, p=0.5, seed=17)
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    num = 65536
    print(f"[sample] n=1024 r={Fo['rank']} num={num}", flush=True)
    out = hlf.sample(F, 42, num)
    torch.cuda.synchronize()
    Z = hlf.as_uint64(out).reshape(num, 16)
    W = 16
    free = [c for c in range(1024) if c not in set(Fo["pivots"])]
    for f, kf in zip(free, Fo["kernel"]):
        kw = np.array([(kf >> (64 * w)) & MASK64 for w in range(W)], dtype=np.uint64)
        parity = np.bitwise_count(Z & kw).sum(axis=1) & 1
        assert np.all(parity == ((Fo["shift"] >> f) & 1)), f
    # exact bits of the first samples against the oracle stream
    assert words_to_ints(Z[:4]) == O.sample(Fo, 42, 4)


def test_sample_uniformity():
    A = grid_instance(3, b=paper_diagonal(9, 0))  # r = 6
    F, _ = gpu_factor(A)
    num = 64 * 1000
    out = hlf.sample(F, 7, num)
    torch.cuda.synchronize()
    vals, cnts = np.unique(hlf.as_uint64(out)[:, 0], return_counts=True)
    assert vals.size == 64
    chi2 = float(((cnts - 1000.0) ** 2 / 1000.0).sum())
    assert chi2 < 130


@pytest.mark.parametrize("name,A,num", [
    ("grid N=12 (W=3)", grid_instance(12, p=0.5, seed=5), 777),
    ("random n=100 (W=2)", random_symmetric(100, 11, 0.3), 500),
    ("grid N=25 (W=10)", grid_instance(25, p=0.5, seed=12), 1000),
    ("random n=1024 (r=1024)", random_symmetric(1024, 8, 0.5), 333),
    ("grid N=32 all edges", grid_instance(32, p=1.0, seed=2), 129),
])
def test_sample_large_n_matrix_core_path(name, A, num):
    """n > 64 runs on sample_mfma_kernel: the grids take its sparse path, the
    random matrices its matrix cores (fp4 products, parities in bits 0 and 11
    of the fp32 sums): exact words against the oracle for the SplitMix64
    stream and for explicit coefficients, with sample counts that leave
    ragged blocks."""
    Fo = O.factor(A)
    F, st = gpu_factor(A)
    r, W = Fo["rank"], Fo["words"]
    print(f"[sample] {name} r={r} num={num}", flush=True)
    out = hlf.sample(F, 0x5EED, num)
    torch.cuda.synchronize()
    assert words_to_ints(hlf.as_uint64(out).reshape(num, W)) == O.sample(Fo, 0x5EED, num)
    R64 = (r + 63) // 64
    rng = np.random.default_rng(r)
    coeffs = rng.integers(-(2**63), 2**63 - 1, size=(num, R64), dtype=np.int64)
    out = hlf.sample(F, 0, num, coeffs=torch.from_numpy(coeffs).cuda())
    torch.cuda.synchronize()
    cints = words_to_ints(coeffs.view(np.uint64))
    assert words_to_ints(hlf.as_uint64(out).reshape(num, W)) == O.sample(Fo, 0, num, coeffs=cints)


def _one_edge(n, i, j, diag=()):
    A = np.zeros((n, n), dtype=np.uint8)
    A[i, j] = A[j, i] = 1
    for d in diag:
        A[d, d] = 1
    return A


@pytest.mark.parametrize("name,A", [
    ("zero n=100 (r=0)", np.zeros((100, 100), dtype=np.uint8)),
    ("one edge n=129 (r=2)", _one_edge(129, 3, 128)),
    ("zero n=300 (r=0)", np.zeros((300, 300), dtype=np.uint8)),
    ("one edge n=300 (r=2)", _one_edge(300, 5, 290)),
    ("one loop n=257 (r=1)", _one_edge(257, 256, 256)),
    ("edge + loops n=640 (r=3)", _one_edge(640, 0, 639, diag=(100,))),
])
def test_sample_matrix_core_path_small_ranks(name, A):
    Fo = O.factor(A)
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    num = 300
    print(f"[sample] {name} r={Fo['rank']}", flush=True)
    out = hlf.sample(F, 77, num)
    torch.cuda.synchronize()
    assert words_to_ints(hlf.as_uint64(out).reshape(num, Fo["words"])) == O.sample(Fo, 77, num)


def test_sample_matrix_core_path_gated_on_status():
    A = np.zeros((300, 300), dtype=np.uint8)
    A[3, 4] = 1  # not symmetric
    F, st = gpu_factor(A)
    assert st == hlf.HLF_ENOTSYM
    out = torch.full((50, F.words), 0x5A5A, dtype=torch.int64, device="cuda")
    hlf.sample(F, 1, 50, out=out)
    torch.cuda.synchronize()
    assert bool((out == 0x5A5A).all())


# --- sparse bases: the per-group choice between the sparse path and the matrix cores
def _group_weights(Fo, words_per_group=4):
    """Per group of 64 * words_per_group columns (the unit in which the
    sampler picks its path: four words for W >= 4, two below): the largest
    number of set bits in one 64-column word of a basis row, and the largest
    column weight."""
    n, W, r = Fo["n"], Fo["words"], Fo["rank"]
    bits = np.zeros((r, n), dtype=np.uint8)
    for k, b in enumerate(Fo["basis"]):
        for j in range(n):
            bits[k, j] = (b >> j) & 1
    out = []
    for g0 in range(0, W, words_per_group):
        blk = bits[:, 64 * g0: min(n, 64 * (g0 + words_per_group))]
        word = max(int(blk[:, 64 * w: 64 * (w + 1)].sum(axis=1).max(initial=0))
                   for w in range((blk.shape[1] + 63) // 64))
        out.append((word, int(blk.sum(axis=0).max(initial=0))))
    return out


def _bounded_degree(n, deg, seed):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.uint8)
    d = np.zeros(n, dtype=int)
    for _ in range(n * deg):
        i, j = rng.integers(0, n, 2)
        if i != j and not A[i, j] and d[i] < deg and d[j] < deg:
            A[i, j] = A[j, i] = 1
            d[i] += 1
            d[j] += 1
    A[np.arange(n), np.arange(n)] = rng.integers(0, 2, n)
    return A


def _mixed_sparse_dense():
    A = np.zeros((512, 512), dtype=np.uint8)
    A[:256, :256] = grid_instance(16, p=0.5, seed=21)
    A[256:, 256:] = random_symmetric(256, 22, 0.5)
    return A


def _heavy_column(n=300, seed=23):
    """Rows of weight <= 16 everywhere, but a column of weight about 20: the
    last vertex is joined to the XOR of two other vertices' neighbourhoods
    (its column depends on theirs, so it is no pivot, and the pivots next to
    it give its basis column many set bits)."""
    rng = np.random.default_rng(seed)
    A = _bounded_degree(n - 1, 10, seed)
    deg = A.sum(axis=1) - A.diagonal()
    u, v = [int(x) for x in np.argsort(-deg)[:2]]
    for cand in np.argsort(-deg)[1:]:
        if not np.any(A[u, :] & A[int(cand), :]):
            v = int(cand)
            break
    a = (A[:, u] ^ A[:, v]).astype(np.uint8)
    B = np.zeros((n, n), dtype=np.uint8)
    B[:n - 1, :n - 1] = A
    B[n - 1, :n - 1] = a
    B[:n - 1, n - 1] = a
    B[n - 1, n - 1] = (a[u] ^ a[v]) & 1
    del rng
    return B


@pytest.mark.parametrize("name,make,expect", [
    ("grid 16x16 + dense 256 (sparse and heavy-word groups)", _mixed_sparse_dense, "mixed"),
    ("degree <= 6 random, n=600 (lists of 6-8)", lambda: _bounded_degree(600, 6, 26), "sparse 8"),
    ("degree <= 15 random, n=600 (lists of 9-16)", lambda: _bounded_degree(600, 15, 24), "sparse 16"),
    ("degree <= 22 random, n=600 (long lists)", lambda: _bounded_degree(600, 22, 25), "column"),
    ("light rows, one heavy column, n=300", _heavy_column, "column"),
])
def test_sample_sparse_path_choice(name, make, expect):
    """Each outcome of the sampler's per-group path choice against the
    oracle: the sparse path when no 64-column word of a basis row has more
    than 16 set bits and no column more than 16 rows (row lists of at most 5,
    8 or 16 entries), the matrix cores at once for a heavy word, and after
    the lists for a heavy column.  The weights check that each case is built
    as intended."""
    A = make()
    Fo = O.factor(A)
    gw = _group_weights(Fo)
    if expect == "mixed":
        assert gw[0][0] <= 16 and gw[0][1] <= 5 and gw[1][0] > 16, gw
    elif expect == "sparse 8":
        assert all(ww <= 16 and cw <= 8 for ww, cw in gw) and any(cw > 5 for _, cw in gw), gw
    elif expect == "sparse 16":
        assert all(ww <= 16 and cw <= 16 for ww, cw in gw) and any(cw > 8 for _, cw in gw), gw
    else:
        assert all(ww <= 16 for ww, _ in gw) and any(cw > 16 for _, cw in gw), gw
    _sample_stream_and_coeffs(A, Fo, f"{name} weights={gw}")


def _sample_stream_and_coeffs(A, Fo, label, num=3000):
    """3000 samples (ragged last block) for the SplitMix64 stream and for
    explicit coefficients, word for word against the oracle."""
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK and int(F.rank.item()) == Fo["rank"]
    print(f"[sample] {label} r={Fo['rank']}", flush=True)
    out = hlf.sample(F, 0xABC, num)
    torch.cuda.synchronize()
    assert words_to_ints(hlf.as_uint64(out).reshape(num, Fo["words"])) == O.sample(Fo, 0xABC, num)
    R64 = (Fo["rank"] + 63) // 64
    rng = np.random.default_rng(Fo["rank"])
    coeffs = rng.integers(-(2**63), 2**63 - 1, size=(num, R64), dtype=np.int64)
    out = hlf.sample(F, 0, num, coeffs=torch.from_numpy(coeffs).cuda())
    torch.cuda.synchronize()
    cints = words_to_ints(coeffs.view(np.uint64))
    assert words_to_ints(hlf.as_uint64(out).reshape(num, Fo["words"])) == O.sample(Fo, 0, num, coeffs=cints)


@pytest.mark.parametrize("name,make,lo,hi", [
    ("degree <= 4 random, n=190 (lists of 5)", lambda: _bounded_degree(190, 4, 34), 0, 5),
    ("degree <= 6 random, n=150 (lists of 6-8)", lambda: _bounded_degree(150, 6, 31), 5, 8),
    ("degree <= 15 random, n=150 (lists of 9-16)", lambda: _bounded_degree(150, 15, 32), 8, 16),
    ("degree <= 22 random, n=100 (heavy words)", lambda: _bounded_degree(100, 22, 33), 16, None),
])
def test_sample_path_choice_two_word_groups(name, make, lo, hi):
    """The same choice in the kernel for 65 <= n <= 192 (groups of two words,
    16 waves): each list length and a heavy word, against the oracle."""
    A = make()
    Fo = O.factor(A)
    assert 2 <= Fo["words"] <= 3
    gw = _group_weights(Fo, words_per_group=2)
    if hi is None:
        assert any(ww > 16 for ww, _ in gw), gw
    else:
        assert all(ww <= 16 and cw <= hi for ww, cw in gw) and any(cw > lo for _, cw in gw), gw
    _sample_stream_and_coeffs(A, Fo, f"{name} weights={gw}")
