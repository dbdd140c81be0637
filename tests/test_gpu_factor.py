"""GPU parity of stage 1 (pack + factor) against the oracle, bit for bit.

Both factor variants (one wavefront per instance for n <= 192, one workgroup
for any n) must reproduce the oracle's rank, pivots, basis, canonical shift and
kernel basis exactly.
"""

import numpy as np
import pytest
import torch

from hlf_inputs import CONFIG2_SEEDS, CONFIG3_SEEDS, grid_instance, low_rank_symmetric, paper_diagonal, random_symmetric
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import device_matrix, gpu_factor, oracle_rows, require_gpu, words_to_ints

pytestmark = pytest.mark.gpu


def _embedded(n, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    A = np.zeros((n, n), dtype=np.uint8)
    A[np.ix_(idx, idx)] = random_symmetric(m, seed, density=0.3)
    return A


def small_cases():
    cases = []
    for b in ("0000", "1011", "1111"):
        cases.append((f"2x2 b={b}", grid_instance(2, b=b)))
    for N in (3, 4, 5):
        for m in (0, 1, 2):
            cases.append((f"{N}x{N} paper m={m}", grid_instance(N, b=paper_diagonal(N * N, m))))
    cases.append(("config1 seed0", grid_instance(4, seed=0)))
    for s in CONFIG2_SEEDS:
        cases.append((f"config2 seed{s}", grid_instance(5, seed=s)))
    for s in CONFIG3_SEEDS:
        cases.append((f"config3 seed{s}", grid_instance(6, p=0.5, seed=s)))
    cases.append(("full rank 6x6", grid_instance(6, b="1" * 36)))
    for N, p, s in [(3, 0.3, 1), (7, 0.5, 2), (8, 1.0, 3), (10, 0.3, 4), (12, 0.5, 5), (12, 1.0, 6)]:
        cases.append((f"grid N={N} p={p} s={s}", grid_instance(N, p=p, seed=s)))
    for n in (1, 2, 63, 64, 65, 127, 128, 129, 191, 192):
        cases.append((f"random n={n}", random_symmetric(n, 1000 + n, density=0.5)))
    for n in (1, 64, 65, 192):
        cases.append((f"zero n={n}", np.zeros((n, n), dtype=np.uint8)))
    cases.append(("identity n=100", np.eye(100, dtype=np.uint8)))
    cases.append(("ones n=70", np.ones((70, 70), dtype=np.uint8)))
    cases.append(("embedded n=150", _embedded(150, 40, 9)))
    return cases


def large_cases():
    return [
        ("random n=193", random_symmetric(193, 7, 0.5)),
        ("random n=256", random_symmetric(256, 8, 0.5)),
        ("sparse n=500", random_symmetric(500, 4, 0.02)),
        ("grid N=32 p=0.5", grid_instance(32, p=0.5, seed=11)),
        ("random n=1000", random_symmetric(1000, 9, 0.5)),
        ("random n=1024", random_symmetric(1024, 3, 0.5)),
        ("zero n=1024", np.zeros((1024, 1024), dtype=np.uint8)),
        ("embedded n=700", _embedded(700, 300, 12)),
        # most 8-column blocks find no pivot; the row's current word must
        # still follow every table update
        ("low rank n=1024 k=20", low_rank_symmetric(1024, 20, 5)),
        # partial last word and partial last block
        ("random n=1023", random_symmetric(1023, 21, 0.5)),
        ("sparse n=1017", random_symmetric(1017, 22, 0.01)),
    ]


def assert_record_matches(F, ref, name):
    got = F.read()
    assert got["status"] == hlf.HLF_OK, name
    r = ref["rank"]
    assert got["rank"] == r, name
    assert got["pivots"][:r] == ref["pivots"], name
    assert all(p == -1 for p in got["pivots"][r:]), name
    assert got["basis"] == ref["basis"], name
    assert got["shift"] == ref["shift"], name
    assert got["kernel"] == ref["kernel"], name


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("name,A", small_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_factor_small_both_variants(name, A):
    print(f"[factor] {name} n={A.shape[0]}", flush=True)
    ref = O.factor(A)
    for workgroup in (False, True):
        F, st = gpu_factor(A, workgroup=workgroup)
        assert st == hlf.HLF_OK
        assert_record_matches(F, ref, f"{name} workgroup={workgroup}")


@pytest.mark.parametrize("name,A", large_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_factor_large_workgroup(name, A):
    print(f"[factor] {name} n={A.shape[0]}", flush=True)
    ref = O.factor(A)
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    assert_record_matches(F, ref, name)


@pytest.mark.parametrize("n", [5, 64, 65, 100, 128, 129, 256, 300, 320, 1001, 1008, 1023, 1024])
def test_pack_matches_layout(n):
    print(f"[pack] n={n}", flush=True)
    A = random_symmetric(n, 77 + n, 0.4)
    rows, st = hlf.pack_dense(device_matrix(A))
    torch.cuda.synchronize()
    assert int(st.item()) == hlf.HLF_OK
    assert np.array_equal(hlf.as_uint64(rows), oracle_rows(A))


@pytest.mark.parametrize("n", [4, 65, 100, 128, 129, 200, 256, 1001, 1008, 1024])
def test_pack_rejects_asymmetric_and_non_binary(n):
    print(f"[pack-invalid] n={n}", flush=True)
    A = random_symmetric(n, 5, 0.5)
    A[0, n - 1] ^= 1  # asymmetric
    _, st = hlf.pack_dense(device_matrix(A))
    assert int(st.item()) == hlf.HLF_ENOTSYM
    B = random_symmetric(n, 6, 0.5)
    B[n // 2, n // 2] = 2  # not 0/1
    _, st = hlf.pack_dense(device_matrix(B))
    assert int(st.item()) == hlf.HLF_ENOTSYM


@pytest.mark.parametrize("n", [65, 128, 129, 1001, 1008, 1024])
def test_pack_non_binary_rows_anywhere(n):
    # n > 64 packs rows across workgroups (16-byte loads when n is a multiple
    # of 16, byte loads otherwise): a byte other than 0 and 1 in any row,
    # alone or in adjacent rows, must give ENOTSYM, and a valid matrix right
    # after must give OK again.
    A = random_symmetric(n, 21, 0.5)
    for rows_bad in ([0], [n - 1], [5, 6], [n - 2, n - 1, 0]):
        B = A.copy()
        for i in rows_bad:
            B[i, (3 * i + 1) % n] = 255
        print(f"[pack-invalid] n={n} rows={rows_bad}", flush=True)
        _, st = hlf.pack_dense(device_matrix(B))
        assert int(st.item()) == hlf.HLF_ENOTSYM, rows_bad
        rows, st = hlf.pack_dense(device_matrix(A))
        assert int(st.item()) == hlf.HLF_OK
        assert np.array_equal(hlf.as_uint64(rows), oracle_rows(A))


@pytest.mark.parametrize("workgroup", [False, True])
def test_factor_rejects_asymmetric_rows_and_pad_bits(workgroup):
    print(f"[factor-invalid] workgroup={workgroup}", flush=True)
    A = random_symmetric(40, 3, 0.5)
    rows = oracle_rows(A)
    rows[3, 0] ^= np.uint64(1) << np.uint64(7)  # A[3,7] != A[7,3]
    F = hlf.Factors(40)
    hlf.factor(torch.from_numpy(rows.view(np.int64)).cuda(), 40, F, workgroup=workgroup)
    assert int(F.status.item()) == hlf.HLF_ENOTSYM
    rows = oracle_rows(A)
    rows[0, 0] |= np.uint64(1) << np.uint64(50)  # a pad bit (n = 40)
    F2 = hlf.Factors(40)
    hlf.factor(torch.from_numpy(rows.view(np.int64)).cuda(), 40, F2, workgroup=workgroup)
    assert int(F2.status.item()) == hlf.HLF_ENOTSYM


def test_factor_record_reused_and_kernel_optional():
    print("[factor-reuse]", flush=True)
    F = hlf.Factors(25, kernel=False)
    for s in (0, 3):
        A = grid_instance(5, seed=s)
        rows, _ = hlf.pack_dense(device_matrix(A))
        hlf.factor(rows, 25, F)
        got = F.read()
        ref = O.factor(A)
        assert got["rank"] == ref["rank"] and got["basis"] == ref["basis"]
        assert got["shift"] == ref["shift"] and "kernel" not in got


def test_factor_agrees_with_words_of_basis_layout():
    """basis rows are columns p_k of A (= rows, A symmetric)."""
    A = grid_instance(9, p=0.5, seed=21)
    F, _ = gpu_factor(A)
    got = F.read()
    rows = oracle_rows(A)
    for k, p in enumerate(got["pivots"][:got["rank"]]):
        assert got["basis"][k] == words_to_ints(rows[p:p + 1])[0]


@pytest.mark.parametrize("n", [16, 100, 1024])
def test_factor_keeps_pack_verdict_in_packed_record(n):
    # HLF_FACTOR_PACK_STATUS: pack writes its verdict into the record's
    # status; a failed one stays and the record is not otherwise written.
    F = hlf.Factors.packed(n, kernel=True)
    W = hlf.words_for(n)
    rows = torch.empty((n, W), dtype=torch.int64, device="cuda")
    bad = random_symmetric(n, 60 + n, 0.5)
    bad[1 % n, 2 % n] = bad[2 % n, 1 % n] = 2  # not a 0/1 matrix
    print(f"[factor] pack verdict kept n={n}", flush=True)
    hlf.pack_dense(device_matrix(bad), rows, F.status)
    F.rank.fill_(-7)
    hlf.factor(rows, n, F, pack_status=True)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_ENOTSYM
    assert int(F.rank.item()) == -7
    # a valid matrix through the same record and flag: the plain result
    good = random_symmetric(n, 70 + n, 0.5)
    hlf.pack_dense(device_matrix(good), rows, F.status)
    hlf.factor(rows, n, F, pack_status=True)
    torch.cuda.synchronize()
    ref = O.factor(good)
    assert_record_matches(F, ref, f"packed record n={n}")
    assert F.status_rank.cpu().tolist() == [hlf.HLF_OK, ref["rank"]]
