"""Pins of the oracle's distribution statistics and membership test
(verification data for a cross-entropy benchmark, Section 5; the ideal output
distribution of App. A), and of the low-rank instance generator."""
import itertools

import numpy as np
import pytest

from hlf_inputs import grid_instance, low_rank_symmetric, random_symmetric
from oracle import hlf_oracle as O


def _instances():
    out = []
    for n, seed, dens in [(1, 0, 0.5), (2, 1, 0.5), (3, 2, 0.9), (5, 3, 0.3), (6, 4, 0.5),
                          (7, 5, 0.2), (8, 6, 0.5), (9, 7, 0.7)]:
        out.append(random_symmetric(n, seed=seed, density=dens))
    out.append(np.zeros((4, 4), dtype=np.uint8))           # r = 0: S = {0}
    for N, p, seed in [(2, 1.0, 0), (3, 0.5, 1), (3, 1.0, 2)]:
        out.append(grid_instance(N, p=p, seed=seed))
    # equal rows on purpose: vertices 0 and 1 with identical neighbourhoods
    A = np.zeros((5, 5), dtype=np.uint8)
    for i, j in [(0, 2), (1, 2), (0, 3), (1, 3), (0, 0), (1, 1), (0, 1), (2, 4)]:
        A[i, j] = A[j, i] = 1
    out.append(A)
    return out


@pytest.mark.parametrize("A", _instances())
def test_pair_quarters_closed_form_equals_counting(A):
    F = O.factor(A)
    C = O.pair_counts(F)
    Q = O.pair_quarters(A)
    r = F["rank"]
    n = A.shape[0]
    for i in range(n):
        for j in range(n):
            assert 4 * C[i][j] == int(Q[i, j]) * (1 << r), (i, j, C[i][j], Q[i, j], r)


@pytest.mark.parametrize("A", _instances())
def test_pair_counts_diagonal_is_reduce_counts(A):
    F = O.factor(A)
    counts, _, _ = O.reduce_range(F, 0, 1 << F["rank"])
    C = O.pair_counts(F)
    assert [C[j][j] for j in range(A.shape[0])] == counts


def test_equal_rows_force_equal_bits():
    A = _instances()[-1]
    assert np.array_equal(A[0], A[1]) and A[0].any()
    F = O.factor(A)
    for z in O.enumerate_range(F, 0, 1 << F["rank"]):
        assert (z & 1) == ((z >> 1) & 1)


@pytest.mark.parametrize("A", [a for a in _instances() if a.shape[0] <= 9])
def test_is_solution_matches_brute_force(A):
    n = A.shape[0]
    S = O.brute_force_solutions(A)
    members = {z for z in range(1 << n) if O.is_solution(A, z)}
    assert members == S
    assert len(members) == 1 << O.factor(A)["rank"]


def test_is_solution_basis_equals_full_kernel_span():
    # checking a basis of Ker(A) decides the same as every x in Ker(A)
    for seed in range(6):
        A = random_symmetric(7, seed=40 + seed, density=0.4)
        n = A.shape[0]
        ker = O.kernel_vectors_all(A)
        for z in range(1 << n):
            full = all((O.q_form(A, x) - 2 * int(sum(((z >> j) & 1) * int(x[j]) for j in range(n)))) % 4 == 0
                       for x in ker)
            assert full == O.is_solution(A, z)


def test_linear_xeb_exact_and_uniform_samples():
    A = grid_instance(3, p=1.0, seed=0)
    F = O.factor(A)
    n, r = A.shape[0], F["rank"]
    exact = O.sample(F, 3, 64)
    assert O.linear_xeb(n, r, [O.is_solution(A, z) for z in exact]) == 2.0 ** (n - r) - 1.0
    # all 2^n strings once: the fraction in S is 2^(r-n), so the estimate is 0
    every = [O.is_solution(A, z) for z in range(1 << n)]
    assert O.linear_xeb(n, r, every) == 0.0


@pytest.mark.parametrize("n,k,seed", [(12, 3, 0), (20, 5, 1), (40, 8, 2), (70, 10, 3)])
def test_low_rank_symmetric_generator(n, k, seed):
    A = low_rank_symmetric(n, k, seed)
    assert A.shape == (n, n) and A.dtype == np.uint8
    assert np.array_equal(A, A.T)
    r = len(O.rref_gf2(A)[1])
    assert r <= k
