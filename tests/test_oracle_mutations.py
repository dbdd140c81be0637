"""The pins catch plausible mistakes: each test plants one mistake in the
oracle (on the CPU, by monkeypatching) and checks that a pin fails."""

import numpy as np
import pytest

from hlf_inputs import grid_instance
from oracle import hlf_oracle as O

import test_oracle_pins as P


def fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def pins_for_factor():
    """A bundle of pins that exercise every stage-1 quantity."""
    for b in ("0000", "1011", "1111"):
        P.test_fig3_2x2_solution_lists(P_paper(), b)
    P.test_solution_set_is_shift_plus_column_space_random_symmetric()
    P.test_kernel_basis_properties()
    P.test_shift_is_the_unique_solution_zero_on_pivots()


_PAPER = None


def P_paper():
    global _PAPER
    if _PAPER is None:
        import json, os
        with open(os.path.join(os.path.dirname(__file__), "golden", "paper_instances.json")) as fh:
            _PAPER = json.load(fh)
    return _PAPER


def test_unmutated_pins_pass():
    pins_for_factor()


def test_dropping_the_diagonal_of_q_is_caught(monkeypatch):
    def q_no_diag(A, x):
        A = np.asarray(A, dtype=np.int64).copy()
        np.fill_diagonal(A, 0)
        xv = np.asarray(x, dtype=np.int64)
        return int(xv @ A @ xv) % 4
    monkeypatch.setattr(O, "q_form", q_no_diag)
    assert fails(pins_for_factor)


def test_q_mod_2_instead_of_mod_4_is_caught(monkeypatch):
    orig = O.q_form
    monkeypatch.setattr(O, "q_form", lambda A, x: orig(A, x) % 2)
    assert fails(pins_for_factor)


def test_row_echelon_without_back_substitution_is_caught(monkeypatch):
    def rref_forward_only(A):
        M = (np.asarray(A, dtype=np.uint8) % 2).copy()
        rows, cols = M.shape
        pivots, top = [], 0
        for c in range(cols):
            if top == rows:
                break
            hits = np.nonzero(M[top:, c])[0]
            if hits.size == 0:
                continue
            p = top + int(hits[0])
            M[[top, p]] = M[[p, top]]
            for i in range(top + 1, rows):  # below only
                if M[i, c]:
                    M[i] ^= M[top]
            pivots.append(c)
            top += 1
        return M[:top].copy(), pivots
    monkeypatch.setattr(O, "rref_gf2", rref_forward_only)
    assert fails(P.test_kernel_basis_properties)


def test_wrong_gray_code_is_caught(monkeypatch):
    monkeypatch.setattr(O, "gray", lambda i: i ^ (i << 1))
    assert fails(P.test_gray_walk_distinct_and_successive_difference)


def test_mix13_constant_typo_is_caught(monkeypatch):
    monkeypatch.setattr(O, "MIX_M2", 0x94D049BB133111EA)
    assert fails(P.test_splitmix64_known_answers)


def test_missing_cz_gate_is_caught(monkeypatch):
    orig = O.statevector_probabilities

    def drop_first_edge(A):
        A = np.asarray(A, dtype=np.uint8).copy()
        n = A.shape[0]
        for i in range(n):
            for j in range(i + 1, n):
                if A[i, j]:
                    A[i, j] = A[j, i] = 0
                    return orig(A)
        return orig(A)
    monkeypatch.setattr(O, "statevector_probabilities", drop_first_edge)
    assert fails(P.test_statevector_support_is_uniform_on_solutions, 3, 1.0, 1)


def test_off_by_one_in_counts_is_caught(monkeypatch):
    orig = O.reduce_range

    def reduce_drop_last(F, begin, count):
        counts, h, xf = orig(F, begin, count)
        counts = counts[:-1] + [0]
        return counts, h, xf
    monkeypatch.setattr(O, "reduce_range", reduce_drop_last)
    assert fails(P.test_counts_closed_form_and_xorfold)


def test_shift_on_pivots_instead_of_free_columns_is_caught(monkeypatch):
    def shift_on_pivots(A):
        A = O.validate(A)
        n = A.shape[0]
        _, piv = O.rref_gf2(A)
        l = 0
        for p, kf in zip(piv, O.kernel_basis(A)):
            q = O.q_form(A, O.bits_to_array(kf, n))
            l |= (q // 2) << p
        return l
    monkeypatch.setattr(O, "canonical_shift", shift_on_pivots)
    assert fails(pins_for_factor)


import test_oracle_stats as ST


def pins_for_stats():
    for A in ST._instances():
        ST.test_pair_quarters_closed_form_equals_counting(A)
    for A in [a for a in ST._instances() if a.shape[0] <= 9]:
        ST.test_is_solution_matches_brute_force(A)
    ST.test_linear_xeb_exact_and_uniform_samples()


def test_unmutated_stats_pins_pass():
    pins_for_stats()


def test_equal_rows_treated_as_independent_is_caught(monkeypatch):
    orig = O.pair_quarters

    def independent_always(A):
        Q = orig(A)
        n = Q.shape[0]
        for i in range(n):
            for j in range(n):
                if i != j and Q[i, j] == 2:
                    Q[i, j] = 1
        return Q
    monkeypatch.setattr(O, "pair_quarters", independent_always)
    assert fails(pins_for_stats)


def test_membership_without_the_quadratic_term_is_caught(monkeypatch):
    def linear_only(A, z, kernel=None):
        A = O.validate(A)
        n = A.shape[0]
        for k in O.kernel_basis(A):
            if bin(k & z).count("1") % 2:
                return False
        return True
    monkeypatch.setattr(O, "is_solution", linear_only)
    assert fails(pins_for_stats)
