"""GPU parity of hlf_solve_dense (A0-A4 + E1 of one instance with n <= 64 in
one launch) against the oracle: the record as hlf_factor writes it and the
solutions as hlf_enumerate writes them, over the N=4 and N=5 grid workloads,
random graphs, ragged ranges and the degenerate cases; range and validation
errors leave the output untouched."""

import numpy as np
import pytest
import torch

from hlf_inputs import CONFIG2_SEEDS, grid_instance, random_symmetric
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import device_matrix, narrow_to_u64, require_gpu

pytestmark = pytest.mark.gpu

_DT = {16: torch.int16, 32: torch.int32, 64: torch.int64}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _check_record(F, ref, name):
    got = F.read()
    assert got["status"] == hlf.HLF_OK, name
    assert got["rank"] == ref["rank"], name
    assert got["pivots"][: ref["rank"]] == ref["pivots"], name
    assert got["basis"] == ref["basis"], name
    assert got["shift"] == ref["shift"], name
    assert got["kernel"] == ref["kernel"], name


def _solve(A, begin, count, word_bits, sentinel=None):
    n = A.shape[0]
    F = hlf.Factors(n)
    out = torch.empty(max(count, 1), dtype=_DT[word_bits], device="cuda")
    if sentinel is not None:
        out.fill_(sentinel)
    hlf.solve_dense(device_matrix(A), F, begin, count, word_bits, out=out[:count] if count else None)
    torch.cuda.synchronize()
    return F, out[:count]


def test_config1_uint16_one_launch():
    A = grid_instance(4, seed=0)
    ref = O.factor(A)
    total = 1 << ref["rank"]
    print(f"[solve] config1 r={ref['rank']}", flush=True)
    F, out = _solve(A, 0, total, 16)
    _check_record(F, ref, "config1")
    assert np.array_equal(narrow_to_u64(out), C.enumerate_range(ref, 0, total)[:, 0])


@pytest.mark.parametrize("seed", CONFIG2_SEEDS)
def test_config2_uint32_many_workgroups(seed):
    # up to 2^25 solutions: hundreds of workgroups, each factoring the instance
    A = grid_instance(5, seed=seed)
    ref = O.factor(A)
    total = 1 << ref["rank"]
    print(f"[solve] config2 seed={seed} r={ref['rank']}", flush=True)
    F, out = _solve(A, 0, total, 32)
    _check_record(F, ref, f"config2 seed {seed}")
    assert np.array_equal(narrow_to_u64(out), C.enumerate_range(ref, 0, total)[:, 0])


@pytest.mark.parametrize("word_bits", [16, 32, 64])
def test_ragged_ranges_random_graph(word_bits):
    n = 16 if word_bits == 16 else 30
    A = random_symmetric(n, 90 + n, 0.4)
    ref = O.factor(A)
    total = 1 << ref["rank"]
    V = 16 // (word_bits // 8)
    for begin, count in [(0, total), (V, total - V - 3), (total - 2 * V, 2 * V), (8 * V, 1), (0, 0)]:
        if count < 0 or begin + count > total:
            continue
        print(f"[solve] ragged wb={word_bits} begin={begin} count={count}", flush=True)
        F, out = _solve(A, begin, count, word_bits)
        _check_record(F, ref, f"ragged {begin} {count}")
        if count:
            assert np.array_equal(narrow_to_u64(out), C.enumerate_range(ref, begin, count)[:, 0])


@pytest.mark.parametrize("name,A", [("zero n=9", np.zeros((9, 9), dtype=np.uint8)),
                                    ("one vertex", np.ones((1, 1), dtype=np.uint8)),
                                    ("full rank n=36", grid_instance(6, b="1" * 36)),
                                    ("ones n=64", np.ones((64, 64), dtype=np.uint8))])
def test_degenerate_cases(name, A):
    ref = O.factor(A)
    r = ref["rank"]
    count = min(1 << r, 1 << 12)
    begin = (1 << r) - count
    print(f"[solve] {name} r={r}", flush=True)
    F, out = _solve(A, begin, count, 64)
    _check_record(F, ref, name)
    assert np.array_equal(narrow_to_u64(out), C.enumerate_range(ref, begin, count)[:, 0])


def test_errors_leave_output_untouched():
    A = grid_instance(4, seed=0)
    r = O.factor(A)["rank"]
    # range past 2^r: HLF_ERANGE, nothing written
    F, out = _solve(A, 0, (1 << r) + 8, 16, sentinel=-3)
    assert int(F.status.item()) == hlf.HLF_ERANGE
    assert bool((out == -3).all())
    # a value other than 0/1, and an asymmetric matrix: HLF_ENOTSYM
    B = A.copy()
    B[0, 5] = 2
    B[5, 0] = 2
    F, out = _solve(B, 0, 64, 16, sentinel=-3)
    assert int(F.status.item()) == hlf.HLF_ENOTSYM
    assert bool((out == -3).all())
    Cm = A.copy()
    Cm[0, 7] ^= 1
    F, out = _solve(Cm, 0, 64, 16, sentinel=-3)
    assert int(F.status.item()) == hlf.HLF_ENOTSYM
    assert bool((out == -3).all())


def test_same_as_three_launches():
    A = random_symmetric(50, 7, 0.5)
    rows, _ = hlf.pack_dense(device_matrix(A))
    F1 = hlf.factor(rows, 50)
    r = int(F1.rank.item())
    count = min(1 << r, 1 << 20)
    z1 = hlf.enumerate_solutions(F1, 0, count, 64)
    F2, z2 = _solve(A, 0, count, 64)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    assert F1.read() == F2.read()
