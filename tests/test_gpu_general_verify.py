"""GPU parity of the arbitrary-graph workload (Section 5: the scheme applies to
any symmetric A) and of the verification data (pair statistics, membership,
linear XEB) against the oracle.

* hlf_enumerate_ex with HLF_ORDER_COUNTER: element by element against the C
  counter-order oracle (pinned to the paper's circuit evaluated layer by
  layer) on grids, random graphs with self-loops and low-rank graphs up to
  n = 1024, one-word (tile and general paths, ragged and unaligned ranges)
  and multi-word; against hlf_enumerate_circuit on grids; the same set as
  Gray order.
* Multi-word Gray order after the word-per-lane stores: against the C oracle.
* hlf_pair_stats: against the oracle's plain counting over all solutions
  (small r) and its closed form; at n = 1024 on sampled pairs.
* hlf_membership: against the oracle's definition on every string (small n)
  and on random strings (n = 64); samples are members and flipping a free
  coordinate makes a non-member (n = 1024); linear XEB of exact samples.
"""

import numpy as np
import pytest
import torch

from hlf_inputs import grid_instance, low_rank_symmetric, random_symmetric
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import device_matrix, gpu_factor, narrow_to_u64, require_gpu, words_to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _ints_from_c(arr):
    a = np.asarray(arr)
    if a.ndim == 1:
        return [int(x) for x in a.view(np.uint64)]
    return words_to_ints(a)


def _gpu_counter(F, begin, count, word_bits):
    out = hlf.enumerate_solutions(F, begin, count, word_bits, order="counter")
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_OK
    if out.dim() == 1:
        return [int(x) for x in narrow_to_u64(out)]
    return words_to_ints(out.cpu().numpy())


@pytest.mark.parametrize("seed", range(8))
def test_counter_order_config2_full_equals_oracle_and_circuit(seed):
    A = grid_instance(5, seed=seed)
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    Fo = O.factor(A)
    total = 1 << Fo["rank"]
    got = hlf.enumerate_solutions(F, 0, total, 32, order="counter")
    circ = hlf.enumerate_circuit(F, hlf.pack_dense(device_matrix(A))[0], 5, 0, total, 32)
    torch.cuda.synchronize()
    want = C.enumerate_counter_range(Fo, 0, total)[:, 0]
    g = narrow_to_u64(got)
    assert np.array_equal(g, want.view(np.uint64))
    assert np.array_equal(g, narrow_to_u64(circ))


@pytest.mark.parametrize("word_bits", [16, 32, 64])
def test_counter_order_ragged_and_unaligned_ranges(word_bits):
    A = random_symmetric(16, seed=5, density=0.4)
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    total = 1 << Fo["rank"]
    for begin, count in [(0, total), (3, 5000), (total - 1027, 1027), (8, 16 * 1024 + 3), (1, 1)]:
        if begin + count > total:
            continue
        got = _gpu_counter(F, begin, count, word_bits)
        want = _ints_from_c(C.enumerate_counter_range(Fo, begin, count)[:, 0])
        assert got == want, (begin, count)


@pytest.mark.parametrize("n,k,seed", [(64, 14, 1), (100, 12, 2), (200, 11, 3), (600, 10, 4),
                                      (1024, 13, 5)])
def test_counter_and_gray_multiword_low_rank(n, k, seed):
    A = low_rank_symmetric(n, k, seed)
    Fo = O.factor(A)
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    r = Fo["rank"]
    W = Fo["words"]
    total = 1 << r
    word_bits = 64 * W if n > 64 else 64
    got_c = _gpu_counter(F, 0, total, word_bits)
    want_c = _ints_from_c(C.enumerate_counter_range(Fo, 0, total))
    assert got_c == want_c
    got_g = hlf.enumerate_solutions(F, 0, total, word_bits)
    torch.cuda.synchronize()
    got_g = words_to_ints(got_g.cpu().numpy()) if got_g.dim() == 2 else [int(x) for x in narrow_to_u64(got_g)]
    assert got_g == _ints_from_c(C.enumerate_range(Fo, 0, total))
    assert sorted(got_c) == sorted(got_g)
    # ragged sub-range in counter order
    b, c = total // 3 + 1, min(777, total - total // 3 - 1)
    assert _gpu_counter(F, b, c, word_bits) == want_c[b:b + c]


def test_counter_order_on_a_random_graph_matches_literal_python_circuit():
    A = random_symmetric(10, seed=11, density=0.5)
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    total = 1 << Fo["rank"]
    assert _gpu_counter(F, 0, total, 16) == O.enumerate_counter_order(A, Fo, 0, total)


def _pair_cases():
    cases = [random_symmetric(n, seed=70 + n, density=d) for n, d in [(3, 0.6), (6, 0.5), (9, 0.3), (11, 0.5)]]
    cases.append(grid_instance(3, p=0.5, seed=4))
    A = np.zeros((7, 7), dtype=np.uint8)
    for i, j in [(0, 2), (1, 2), (0, 3), (1, 3), (0, 1), (2, 4), (5, 5)]:
        A[i, j] = A[j, i] = 1
    cases.append(A)  # rows 0 and 1 equal, row 6 zero
    cases.append(np.zeros((5, 5), dtype=np.uint8))
    return cases


@pytest.mark.parametrize("A", _pair_cases())
def test_pair_stats_equal_plain_counting(A):
    Fo = O.factor(A)
    F, st = gpu_factor(A)
    rows, _ = hlf.pack_dense(device_matrix(A))
    q = hlf.pair_stats(F, rows)
    torch.cuda.synchronize()
    Q = q.cpu().numpy().astype(np.int64)
    Cnt = O.pair_counts(Fo)
    r = Fo["rank"]
    n = A.shape[0]
    for i in range(n):
        for j in range(n):
            assert 4 * Cnt[i][j] == Q[i, j] * (1 << r), (i, j)
    assert np.array_equal(Q, O.pair_quarters(A))


@pytest.mark.parametrize("A", [grid_instance(32, p=0.5, seed=17), random_symmetric(700, seed=3, density=0.5),
                               low_rank_symmetric(1024, 20, 6)])
def test_pair_stats_large_sampled_pairs(A):
    n = A.shape[0]
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    rows, _ = hlf.pack_dense(device_matrix(A))
    Q = hlf.pair_stats(F, rows).cpu().numpy()
    rng = np.random.default_rng(n)
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, n, size=(3000, 2))] + [(i, i) for i in range(0, n, 7)]
    for i, j in pairs:
        if not A[i].any() or not A[j].any():
            want = 0
        elif np.array_equal(A[i], A[j]):
            want = 2
        else:
            want = 1
        assert Q[i, j] == want, (i, j)
    # row-class property over the whole matrix: Q[i, j] == 2 exactly for equal nonzero rows
    _, inv = np.unique(A, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nz = A.any(axis=1)
    same = (inv[:, None] == inv[None, :]) & nz[:, None] & nz[None, :]
    assert np.array_equal(Q == 2, same)
    assert np.array_equal(Q == 0, ~(nz[:, None] & nz[None, :]))


def test_pair_stats_gated_on_status():
    A = np.zeros((6, 6), dtype=np.uint8)
    A[0, 1] = 1  # not symmetric
    F, st = gpu_factor(A)
    assert st == hlf.HLF_ENOTSYM
    rows, _ = hlf.pack_dense(device_matrix(A))
    out = torch.full((6, 6), 0xEE, dtype=torch.uint8, device="cuda")
    hlf.pair_stats(F, rows, out=out)
    torch.cuda.synchronize()
    assert int(out.min().item()) == 0xEE and int(out.max().item()) == 0xEE


@pytest.mark.parametrize("A", [random_symmetric(n, seed=80 + n, density=0.4) for n in (1, 4, 8, 12)]
                         + [grid_instance(3, p=1.0, seed=0), np.zeros((6, 6), dtype=np.uint8)])
def test_membership_every_string_small_n(A):
    n = A.shape[0]
    F, _ = gpu_factor(A)
    allz = torch.arange(1 << n, dtype=torch.int64, device="cuda").reshape(-1, 1)
    m = hlf.membership(F, allz).cpu().numpy()
    S = O.brute_force_solutions(A)
    assert [z for z in range(1 << n) if m[z]] == sorted(S)


def test_membership_random_strings_n64():
    A = random_symmetric(64, seed=9, density=0.1)
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    rng = np.random.default_rng(1)
    zs = [int(x) for x in rng.integers(0, 2**63, size=300, dtype=np.int64)]
    # half of them made into solutions by the oracle's own shift + basis
    zs += O.sample(Fo, 5, 300)
    z = torch.tensor([[x - (1 << 64) if x >= (1 << 63) else x] for x in zs], dtype=torch.int64,
                     device="cuda")
    m = hlf.membership(F, z).cpu().numpy()
    ker = Fo["kernel"]
    want = [O.is_solution(A, x, kernel=ker) for x in zs]
    assert [bool(v) for v in m] == want
    assert all(want[300:])


def test_membership_n1024_samples_flips_and_xeb():
    A = grid_instance(32, p=0.5, seed=17)
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    n = 1024
    r = int(F.rank.item())
    z = hlf.sample(F, 7, 20000)
    m = hlf.membership(F, z)
    torch.cuda.synchronize()
    assert int(m.sum().item()) == 20000
    assert O.linear_xeb(n, r, m.cpu().numpy().tolist()) == 2.0 ** (n - r) - 1.0
    # flip one free coordinate f of every sample: <k_f, z> changes, so no sample stays a solution
    piv = set(int(p) for p in F.pivots.cpu().numpy()[:r])
    free = [c for c in range(n) if c not in piv]
    f = free[len(free) // 2]
    flipped = z.clone()
    flipped[:, f // 64] ^= torch.tensor(np.array([1 << (f % 64)], dtype=np.uint64).view(np.int64)[0],
                                        device="cuda")
    m2 = hlf.membership(F, flipped)
    torch.cuda.synchronize()
    assert int(m2.sum().item()) == 0
    # flipping a coordinate in Col(A) direction (adding basis vector 0) keeps membership
    moved = z ^ F.basis[0].unsqueeze(0)
    assert int(hlf.membership(F, moved).sum().item()) == 20000



def _embedded_sym(n, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    A = np.zeros((n, n), dtype=np.uint8)
    A[np.ix_(idx, idx)] = random_symmetric(m, seed, density=0.3)
    return A


MEMBERSHIP_CASES = {  # n - r of each instance: one to four 32-vector chunks, beyond 128, none
    "nk21": lambda: _embedded_sym(256, 236, 1),
    "nk51": lambda: _embedded_sym(256, 206, 2),
    "nk80": lambda: _embedded_sym(320, 240, 3),
    "nk120": lambda: _embedded_sym(256, 136, 4),
    "nk157": lambda: _embedded_sym(256, 100, 5),
    "nk2": lambda: random_symmetric(256, 6, density=0.5),
    "nk0": lambda: random_symmetric(200, 8, density=0.5),
}


@pytest.mark.parametrize("name", list(MEMBERSHIP_CASES))
def test_membership_n_above_192_against_definition(name):
    # n > 192: the matrix-core kernel for 1 <= n - r <= 128, the per-string
    # kernel otherwise.  Exact samples, samples with one or two flipped bits
    # and uniform strings, each compared with the definition: z is a solution
    # iff <k_f, z> = q(k_f)/2 (mod 2) for every kernel vector k_f.
    A = MEMBERSHIP_CASES[name]()
    n = A.shape[0]
    Fo = O.factor(A)
    ker = Fo["kernel"]
    print(f"[verify] membership {name}: n={n} n-r={len(ker)}", flush=True)
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    rng = np.random.default_rng(len(ker) + 7)
    members = O.sample(Fo, 3, 200)
    flipped = [z ^ (1 << int(rng.integers(n))) for z in members[:100]]
    flipped += [z ^ (1 << int(rng.integers(n))) ^ (1 << int(rng.integers(n))) for z in members[100:]]
    uniform = [int.from_bytes(rng.bytes((n + 7) // 8), "little") & ((1 << n) - 1) for _ in range(100)]
    zs = members + flipped + uniform + members[:37]  # 637 strings: a ragged last block
    qhalf = [(O.q_form(A, O.bits_to_array(k, n)) // 2) & 1 for k in ker]
    want = [all(bin(z & k).count("1") % 2 == q for k, q in zip(ker, qhalf)) for z in zs]
    for z, w in list(zip(zs, want))[::97]:  # the restated definition agrees with the oracle's own
        assert O.is_solution(A, z, kernel=ker) == w
    W = (n + 63) // 64
    words = np.array([[(z >> (64 * w)) & ((1 << 64) - 1) for w in range(W)] for z in zs],
                     dtype=np.uint64).view(np.int64)
    m = hlf.membership(F, torch.from_numpy(words).to("cuda")).cpu().numpy()
    assert [bool(v) for v in m] == want
    assert all(want[:200])

def test_membership_requires_kernel_buffer():
    A = grid_instance(3, seed=1)
    F, _ = gpu_factor(A, kernel=False)
    with pytest.raises(hlf.HlfError):
        hlf.membership(F, torch.zeros((4, 1), dtype=torch.int64, device="cuda"))
