"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped term
of q, a wrong index in the kernel basis, a transposed basis, a wrong sign of
the S gate, an off-by-one in the Gray walk) fails at least one of them.
"""

import json
import os

import numpy as np
import pytest

from hlf_inputs import grid_instance, paper_diagonal, random_symmetric
from oracle import hlf_oracle as O
from oracle import c_oracle as C


def bits(z, n):
    return "".join(str((z >> j) & 1) for j in range(n))


def from_bits(s):
    return sum(int(ch) << j for j, ch in enumerate(s))


@pytest.fixture(scope="module")
def paper(golden_dir):
    with open(os.path.join(golden_dir, "paper_instances.json")) as fh:
        return json.load(fh)


# -- Values the paper prints -------------------------------------------------

@pytest.mark.parametrize("b", ["0000", "1011", "1111"])
def test_fig3_2x2_solution_lists(paper, b):
    """Fig. 3(a)-(c): the printed solution sets of the 2x2 grid."""
    entry = paper["lists_2x2"][b]
    A = grid_instance(2, b=b)
    F = O.factor(A)
    assert F["rank"] == entry["rank"]
    got = sorted(bits(z, 4) for z in O.enumerate_range(F, 0, 1 << F["rank"]))
    want = [bits(v, 4) for v in range(16)] if entry["solutions"] == "all" else entry["solutions"]
    assert got == sorted(want)
    assert sorted(bits(z, 4) for z in O.brute_force_solutions(A)) == sorted(want)


def test_paper_counts_and_ranks(paper):
    """Fig. 3(d)-(f), Fig. 6, Fig. 7: rank r and 2^r solutions of 0^(n-m)1^(m)."""
    for e in paper["counts"]:
        n = e["N"] ** 2
        A = grid_instance(e["N"], b=paper_diagonal(n, e["ones_at_end"]))
        F = O.factor(A)
        assert F["rank"] == e["rank"], e
        assert (1 << F["rank"]) == e["solutions"]
        assert O.independent_columns_greedy(A) == F["pivots"]


def test_3x3_paper_sets_match_brute_force():
    """The 3x3 instances of Fig. 6 (n = 9): full set vs the problem definition."""
    for m in (0, 1, 2):
        A = grid_instance(3, b=paper_diagonal(9, m))
        F = O.factor(A)
        got = set(O.enumerate_range(F, 0, 1 << F["rank"]))
        assert got == O.brute_force_solutions(A)


# -- Appendix B rank interval --------------------------------------------------

def test_appendix_b_rank_zero_diagonal():
    """All-connected N x N grid with b = 0: r = n - N (App. B)."""
    for N in range(2, 11):
        A = grid_instance(N, b=np.zeros(N * N, dtype=np.uint8))
        assert O.factor(A)["rank"] == N * N - N


def test_appendix_b_rank_interval_random_diagonal():
    """All-connected grids, any b: n - N <= r <= n (App. B)."""
    rng = np.random.default_rng(12345)
    for N in range(2, 9):
        for _ in range(25):
            b = rng.integers(0, 2, size=N * N)
            r = O.factor(grid_instance(N, b=b))["rank"]
            assert N * N - N <= r <= N * N


# -- Structure theorem against the problem definition (Section 2) -------------

def _span(vectors):
    s = {0}
    for v in vectors:
        s |= {x ^ v for x in s}
    return s


def test_solution_set_is_shift_plus_column_space_random_symmetric():
    """Brute force (definition, Section 1) == l + Col(A), |set| = 2^r (Section 2)."""
    for seed in range(60):
        n = 1 + seed % 8
        A = random_symmetric(n, seed, density=0.3 + 0.1 * (seed % 5))
        F = O.factor(A)
        col_space = {int(sum(int(A[i, :] @ np.array([(x >> j) & 1 for j in range(n)])) % 2 << i
                             for i in range(n))) for x in range(1 << n)}
        assert _span(F["basis"]) == col_space
        sols = O.brute_force_solutions(A)
        assert len(sols) == 1 << F["rank"]
        assert {F["shift"] ^ y for y in col_space} == sols


def test_solution_set_random_grid_subgraphs():
    for seed in range(30):
        N = 2 + seed % 2
        A = grid_instance(N, p=0.5, seed=seed)
        F = O.factor(A)
        assert set(O.enumerate_range(F, 0, 1 << F["rank"])) == O.brute_force_solutions(A)


def test_kernel_basis_properties():
    """Task (2): A k_f = 0, n - r vectors, unit at f, zero at other free columns;
    |Ker| = 2^(n-r) by exhaustive count."""
    for seed in range(40):
        n = 2 + seed % 7
        A = random_symmetric(n, 100 + seed, density=0.4)
        F = O.factor(A)
        K = F["kernel"]
        free = [c for c in range(n) if c not in F["pivots"]]
        assert len(K) == n - F["rank"]
        for f, kf in zip(free, K):
            x = O.bits_to_array(kf, n)
            assert not np.any((A.astype(np.int64) @ x) % 2)
            for g in free:
                assert ((kf >> g) & 1) == (1 if g == f else 0)
        assert len(O.kernel_vectors_all(A)) == 1 << (n - F["rank"])
        assert _span(K) == {O.array_to_bits(x) for x in O.kernel_vectors_all(A)}


def test_shift_is_the_unique_solution_zero_on_pivots():
    """Task (4) with the canonical choice: l solves the problem, l_p = 0 on P,
    and no other solution is zero on P."""
    for seed in range(40):
        n = 1 + seed % 8
        A = random_symmetric(n, 200 + seed, density=0.5)
        F = O.factor(A)
        sols = O.brute_force_solutions(A)
        assert F["shift"] in sols
        zero_on_p = [z for z in sols if all(((z >> p) & 1) == 0 for p in F["pivots"])]
        assert zero_on_p == [F["shift"]]


def test_q_is_even_and_linear_on_kernel():
    """q takes values {0, 2} on Ker(A) and is additive there (Section 2)."""
    for seed in range(30):
        n = 2 + seed % 7
        A = random_symmetric(n, 300 + seed)
        ker = [O.array_to_bits(x) for x in O.kernel_vectors_all(A)]
        for x in ker:
            assert O.q_form(A, O.bits_to_array(x, n)) in (0, 2)
        for x in ker[:8]:
            for y in ker[:8]:
                qx = O.q_form(A, O.bits_to_array(x, n))
                qy = O.q_form(A, O.bits_to_array(y, n))
                assert O.q_form(A, O.bits_to_array(x ^ y, n)) == (qx + qy) % 4


def test_q_form_hand_values():
    """q counts the diagonal once and each off-diagonal pair twice."""
    A = np.array([[1, 1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.uint8)
    assert O.q_form(A, [1, 0, 0]) == 1
    assert O.q_form(A, [1, 1, 0]) == (1 + 0 + 2) % 4
    assert O.q_form(A, [1, 1, 1]) == (1 + 0 + 1 + 2 + 2) % 4
    assert O.q_form(A, [0, 1, 0]) == 0


# -- Appendix A: the quantum circuit's output ---------------------------------

@pytest.mark.parametrize("N,p,seed", [(2, 1.0, 0), (2, 0.5, 3), (3, 1.0, 1), (3, 0.5, 7), (4, 1.0, 2), (4, 0.5, 5)])
def test_statevector_support_is_uniform_on_solutions(N, p, seed):
    """Eqs. (A1)-(A2): the support of the output distribution is the solution
    set and it is uniform, each outcome with probability 2^-r."""
    A = grid_instance(N, p=p, seed=seed)
    n = N * N
    F = O.factor(A)
    prob = O.statevector_probabilities(A)
    support = {int(v) for v in np.nonzero(prob > 0.5 * 2.0 ** (-n))[0]}
    assert support == set(O.enumerate_range(F, 0, 1 << F["rank"]))
    assert np.allclose(prob[sorted(support)], 2.0 ** (-F["rank"]), atol=1e-12)
    assert abs(prob.sum() - 1.0) < 1e-9


def test_statevector_paper_4x4():
    A = grid_instance(4, b=paper_diagonal(16, 1))
    F = O.factor(A)
    prob = O.statevector_probabilities(A)
    assert int(np.count_nonzero(prob > 0.5 * 2.0 ** -16)) == 8192 == 1 << F["rank"]


# -- Enumeration invariants ---------------------------------------------------

def test_gray_walk_distinct_and_successive_difference():
    A = grid_instance(4, seed=0)
    F = O.factor(A)
    zs = O.enumerate_range(F, 0, 1 << F["rank"])
    assert len(set(zs)) == len(zs) == 1 << F["rank"]
    assert zs[0] == F["shift"]
    for i in range(1, len(zs)):
        ctz = (i & -i).bit_length() - 1
        assert zs[i] ^ zs[i - 1] == F["basis"][ctz]


def test_literal_circuit_equals_direct_definition():
    """Eqs. (1)-(3): the ROU + Toffoli layers compute A R on the pivot inputs."""
    for seed in range(6):
        A = grid_instance(3 + seed % 2, p=0.7, seed=seed)
        F = O.factor(A)
        for R in range(min(1 << F["rank"], 200)):
            y = 0
            for k, Bk in enumerate(F["basis"]):
                if (R >> k) & 1:
                    y ^= Bk
            assert O.cpc_output(A, F["pivots"], R, F["shift"]) == y ^ F["shift"]
        full = O.enumerate_counter_order(A, F, 0, 1 << F["rank"]) if F["rank"] <= 12 else None
        if full is not None:
            assert set(full) == set(O.enumerate_range(F, 0, 1 << F["rank"]))


def test_counts_closed_form_and_xorfold():
    """Full enumeration: counts_j = 2^(r-1) if row j of A is nonzero else 0;
    XOR of all solutions is 0 for r >= 2."""
    for seed in range(8):
        A = grid_instance(3, p=0.5, seed=seed)
        F = O.factor(A)
        r = F["rank"]
        counts, h, xf = O.reduce_range(F, 0, 1 << r)
        for j in range(9):
            want = (1 << (r - 1)) if A[j].any() else 0
            assert counts[j] == want
        if r >= 2:
            assert xf == 0


def test_reduce_hash_full_rank_equals_identity_sum(golden_dir):
    """Full rank: the solution set is {0,1}^n (Section 3), so the set hash is the
    plain sum over all z; the C oracle's identity sum is stored."""
    with open(os.path.join(golden_dir, "identity_hash.json")) as fh:
        gold = json.load(fh)
    A = grid_instance(4, b="0110011101111110")
    F = O.factor(A)
    assert F["rank"] == 16
    _, h, _ = O.reduce_range(F, 0, 1 << 16)
    direct = sum(O.hash_solution(z, 1) for z in range(1 << 16)) & O.MASK64
    assert h == direct == int(gold["identity_hash_n16"], 16)


def test_hash_chain_multiword_hand_value():
    z = (5 << 64) | 7
    h1 = O.mix13(0 ^ 7 ^ O.GAMMA)
    assert O.hash_solution(z, 2) == O.mix13(h1 ^ 5 ^ O.GAMMA)


def test_splitmix64_known_answers():
    """SplitMix64 from state 0: first outputs of the published reference
    implementation (Vigna's splitmix64.c)."""
    assert O.splitmix64_output(0, 0) == 0xE220A8397B1DCDAF
    assert O.splitmix64_output(0, 1) == 0x6E789E6AA1B965F4
    assert O.splitmix64_output(0, 2) == 0x06C45D188009454F
    assert C.mix13(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_samples_are_solutions_and_follow_coefficients():
    for seed in range(5):
        A = grid_instance(3, p=0.6, seed=seed)
        F = O.factor(A)
        sols = O.brute_force_solutions(A)
        zs = O.sample(F, seed=99 + seed, num=64)
        assert all(z in sols for z in zs)
        # explicit coefficients reproduce the generator's draw
        cs = [O.sample_coefficients(99 + seed, F["rank"], s) for s in range(64)]
        assert O.sample(F, 0, 64, coeffs=cs) == zs


def test_samples_uniform_chi_square():
    A = grid_instance(3, b=paper_diagonal(9, 0))
    F = O.factor(A)  # r = 6: 64 solutions
    zs = O.sample(F, seed=2024, num=64 * 200)
    hist = {}
    for z in zs:
        hist[z] = hist.get(z, 0) + 1
    assert len(hist) == 64
    exp = 200.0
    chi2 = sum((c - exp) ** 2 / exp for c in hist.values())
    assert chi2 < 130  # 63 dof; p ~ 1e-6 above this


def test_edge_cases():
    A0 = np.zeros((5, 5), dtype=np.uint8)
    F = O.factor(A0)
    assert F["rank"] == 0 and F["shift"] == 0 and O.enumerate_range(F, 0, 1) == [0]
    A1 = np.ones((1, 1), dtype=np.uint8)
    F1 = O.factor(A1)
    assert F1["rank"] == 1 and set(O.enumerate_range(F1, 0, 2)) == {0, 1}
    with pytest.raises(ValueError):
        O.validate(np.array([[0, 1], [0, 0]]))
    with pytest.raises(ValueError):
        O.validate(np.array([[2, 0], [0, 0]]))


# -- The C oracle agrees with the Python one ------------------------------------

def test_c_oracle_matches_python_oracle():
    for seed in range(4):
        A = grid_instance(5, seed=seed)
        F = O.factor(A)
        for begin, count in [(0, 300), (12345, 1000), ((1 << F["rank"]) - 257, 257)]:
            zs = C.enumerate_range(F, begin, count)
            assert [int(z[0]) for z in zs] == O.enumerate_range(F, begin, count)
            c, h, xf = C.reduce_range(F, begin, count)
            c2, h2, xf2 = O.reduce_range(F, begin, count)
            assert list(map(int, c)) == c2 and h == h2 and int(xf[0]) == xf2


def _embedded(n, m, seed):
    """An n x n symmetric matrix whose support is m scattered vertices (r <= m)."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    A = np.zeros((n, n), dtype=np.uint8)
    A[np.ix_(idx, idx)] = random_symmetric(m, seed, density=0.3)
    return A


def test_c_oracle_multiword_matches_python():
    A = _embedded(100, 40, 7)
    F = O.factor(A)
    assert F["rank"] <= 40
    zs = C.enumerate_range(F, 5, 200)
    ref = O.enumerate_range(F, 5, 200)
    for row, z in zip(zs, ref):
        assert sum(int(row[w]) << (64 * w) for w in range(2)) == z
    c, h, _ = C.reduce_range(F, 5, 200)
    c2, h2, _ = O.reduce_range(F, 5, 200)
    assert list(map(int, c)) == c2 and h == h2


def test_c_oracle_counts_closed_form_at_scale():
    A = grid_instance(5, seed=3)
    F = O.factor(A)
    r = F["rank"]
    counts, h, xf = C.reduce_range(F, 0, 1 << r)
    for j in range(25):
        assert int(counts[j]) == ((1 << (r - 1)) if A[j].any() else 0)
    assert int(xf[0]) == 0


def test_c_oracle_counter_order_equals_literal_circuit():
    """The C counter-order enumerator equals the paper's circuit (Eqs. (1)-(2)
    evaluated layer by layer, Fig. 1(c)) fed by the binary counter (Section 4)."""
    for seed, (N, p) in enumerate([(3, 1.0), (4, 0.5), (5, 1.0), (4, 1.0)]):
        A = grid_instance(N, p=p, seed=seed)
        F = O.factor(A)
        total = 1 << F["rank"]
        for begin, count in [(0, min(total, 300)), (max(0, total - 77), min(total, 77))]:
            got = [int(z[0]) for z in C.enumerate_counter_range(F, begin, count)]
            assert got == O.enumerate_counter_order(A, F, begin, count)
        assert set(int(z[0]) for z in C.enumerate_counter_range(F, 0, min(total, 1 << 12))) <= \
            set(int(z[0]) for z in C.enumerate_range(F, 0, total))


def test_c_oracle_counter_order_equals_literal_circuit_any_graph():
    """Section 5: the same circuit, one ROU per edge of G(A) plus the Toffoli
    layer, serves any symmetric A.  The C counter-order enumerator (basis
    form) equals it on random graphs with self-loops and on low-rank graphs,
    multi-word included."""
    from hlf_inputs import low_rank_symmetric
    cases = [random_symmetric(n, seed=60 + n, density=d) for n, d in [(6, 0.5), (9, 0.3), (12, 0.6)]]
    cases += [low_rank_symmetric(70, 9, 1), low_rank_symmetric(130, 7, 2)]
    for A in cases:
        F = O.factor(A)
        total = 1 << F["rank"]
        for begin, count in [(0, min(total, 200)), (max(0, total - 33), min(total, 33))]:
            got = C.enumerate_counter_range(F, begin, count)
            want = O.enumerate_counter_order(A, F, begin, count)
            W = F["words"]
            assert [sum(int(zw) << (64 * w) for w, zw in enumerate(z)) for z in got] == want
