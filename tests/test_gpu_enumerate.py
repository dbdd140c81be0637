"""GPU parity of the materialise path (hlf_enumerate) against the oracle.

Full arrays are compared element by element at the benchmark's full sizes
(all 2^r solutions of every N=5 seed) and at small sizes that span several
tiles with ragged heads and tails; edge cases cover r = 0, 1, 2, unaligned
begin and output pointers, 64-bit and multiword outputs, and status handling.
"""

import numpy as np
import pytest
import torch

from hlf_inputs import CONFIG2_SEEDS, grid_instance, random_symmetric, sparse_grid_instance
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf

from gpu_util import gpu_factor, narrow_to_u64, require_gpu, words_to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _embedded(n, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    A = np.zeros((n, n), dtype=np.uint8)
    A[np.ix_(idx, idx)] = random_symmetric(m, seed, density=0.3)
    return A


def gpu_enum(F, begin, count, word_bits):
    out = hlf.enumerate_solutions(F, begin, count, word_bits)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_OK
    return out


def ref_enum(Fo, begin, count):
    return C.enumerate_range(Fo, begin, count)


def test_config1_full_all_formats():
    A = grid_instance(4, seed=0)
    Fo = O.factor(A)
    r = Fo["rank"]
    print(f"[enum] config1 r={r}", flush=True)
    F, _ = gpu_factor(A)
    ref = ref_enum(Fo, 0, 1 << r)[:, 0]
    for wb in (16, 32, 64):
        got = narrow_to_u64(gpu_enum(F, 0, 1 << r, wb))
        assert np.array_equal(got, ref), wb


@pytest.mark.parametrize("seed", CONFIG2_SEEDS)
def test_config2_full_u32(seed):
    A = grid_instance(5, seed=seed)
    Fo = O.factor(A)
    r = Fo["rank"]
    print(f"[enum] config2 seed={seed} r={r} count={1 << r}", flush=True)
    F, _ = gpu_factor(A)
    got = narrow_to_u64(gpu_enum(F, 0, 1 << r, 32))
    ref = ref_enum(Fo, 0, 1 << r)[:, 0]
    assert np.array_equal(got, ref)
    # successive solutions differ by B_ctz(i) (Gray step), checked on the GPU output itself
    idx = np.arange(1, 1 << 16, dtype=np.uint64)
    ctz = np.array([(int(i) & -int(i)).bit_length() - 1 for i in idx])
    B = np.array(Fo["basis"], dtype=np.uint64)
    assert np.array_equal(got[1:1 << 16] ^ got[:(1 << 16) - 1], B[ctz])
    if seed == 0:  # all distinct
        assert np.unique(got).size == got.size


RANGES = [(1, 1000), (3, 4095), (5, 1), (1023, 1025), (4, 4096 * 3 + 7), (12345678, (1 << 20) + 7),
          (8, 1 << 21)]


@pytest.mark.parametrize("word_bits", [32, 64])
def test_ragged_and_unaligned_ranges(word_bits):
    A = grid_instance(5, seed=2)  # r = 25
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    for begin, count in RANGES + [((1 << r) - 3, 3), ((1 << r) - 1000, 1000)]:
        print(f"[enum] ragged wb={word_bits} begin={begin} count={count}", flush=True)
        got = narrow_to_u64(gpu_enum(F, begin, count, word_bits))
        assert np.array_equal(got, ref_enum(Fo, begin, count)[:, 0]), (begin, count)



@pytest.mark.parametrize("blocks", [515, 517, 1021])
def test_xcd_dealing_ragged_block_counts(blocks):
    # Launches of more than 512 workgroups whose count is not a multiple of
    # the 8 XCDs: each XCD takes one contiguous run of 128 KiB ranges, the
    # later workgroups seed their lane constants the per-index way, and the
    # last range is short.  The whole output is compared.
    A = grid_instance(5, seed=2)  # r = 25
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    per_block = 8 * 4096  # 8 tiles of 4096 uint32 solutions
    begin = 4
    count = per_block * (blocks - 1) + 4096 * 5 + 7  # 8*blocks - 2 tiles
    assert begin + count <= 1 << Fo["rank"]
    print(f"[enum] xcd dealing blocks={blocks} count={count}", flush=True)
    got = narrow_to_u64(gpu_enum(F, begin, count, 32))
    assert np.array_equal(got, ref_enum(Fo, begin, count)[:, 0])


def test_xcd_dealing_multiword_large_ragged():
    # The W = 2 kernel over more than 512 workgroups with a ragged tail.
    A = _embedded(100, 26, 5)  # r = 24
    Fo = O.factor(A)
    r = Fo["rank"]
    assert r >= 24
    F, _ = gpu_factor(A)
    # tiles of 1024 indices, 16 per workgroup: 8261 tiles, 517 workgroups
    begin, count = 3, 1024 * 8260 + 11
    print(f"[enum] xcd dealing multiword r={r} count={count}", flush=True)
    got = gpu_enum(F, begin, count, 128)
    assert np.array_equal(hlf.as_uint64(got).reshape(count, 2), ref_enum(Fo, begin, count))

def test_misaligned_output_pointer():
    A = grid_instance(5, seed=4)
    Fo = O.factor(A)
    F, _ = gpu_factor(A)
    for wb, dt in ((32, torch.int32), (64, torch.int64)):
        big = torch.zeros(70001, dtype=dt, device="cuda")
        view = big[1:]  # 4- or 8-byte offset from a 256-byte aligned base
        print(f"[enum] misaligned out wb={wb}", flush=True)
        hlf.enumerate_solutions(F, 64, 70000, wb, out=view)
        torch.cuda.synchronize()
        got = narrow_to_u64(view)
        assert np.array_equal(got, ref_enum(Fo, 64, 70000)[:, 0])
        assert int(big[0].item()) == 0


@pytest.mark.parametrize("name,A", [
    ("zero n=5 (r=0)", np.zeros((5, 5), dtype=np.uint8)),
    ("1x1 one (r=1)", np.ones((1, 1), dtype=np.uint8)),
    ("2x2 b=0000 (r=2)", grid_instance(2, b="0000")),
    ("2x2 b=1011 (r=3)", grid_instance(2, b="1011")),
    ("3x3 p=0.3", grid_instance(3, p=0.3, seed=8)),
    ("n=64 embedded", _embedded(64, 30, 4)),
])
def test_small_rank_edge_cases(name, A):
    Fo = O.factor(A)
    r = Fo["rank"]
    n = A.shape[0]
    F, _ = gpu_factor(A)
    ref = ref_enum(Fo, 0, 1 << r)[:, 0]
    for wb in (16, 32, 64):
        if n > wb:
            continue
        print(f"[enum] {name} r={r} wb={wb}", flush=True)
        got = narrow_to_u64(gpu_enum(F, 0, 1 << r, wb))
        assert np.array_equal(got, ref)
        if r >= 1:
            got2 = narrow_to_u64(gpu_enum(F, 1, (1 << r) - 1, wb))
            assert np.array_equal(got2, ref[1:])


@pytest.mark.parametrize("n,m,seed", [(65, 40, 1), (100, 50, 2), (200, 33, 3), (1024, 40, 4)])
def test_multiword(n, m, seed):
    A = _embedded(n, m, seed)
    Fo = O.factor(A)
    r = Fo["rank"]
    W = (n + 63) // 64
    F, _ = gpu_factor(A)
    for begin, count in [(0, min(1 << r, 5000)), (3, min((1 << r) - 3, 777)), ((1 << r) - 300, 300)]:
        print(f"[enum] multiword n={n} r={r} begin={begin} count={count}", flush=True)
        got = gpu_enum(F, begin, count, 64 * W)
        ref = ref_enum(Fo, begin, count)
        assert np.array_equal(hlf.as_uint64(got).reshape(count, W), ref)


def test_out_of_range_sets_erange_and_writes_nothing():
    A = grid_instance(4, seed=0)
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    out = torch.full((100,), -7, dtype=torch.int32, device="cuda")
    print("[enum] erange", flush=True)
    hlf.enumerate_solutions(F, (1 << r) - 50, 100, 32, out=out)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_ERANGE
    assert bool((out == -7).all())
    # the record stays poisoned: later calls write nothing
    hlf.enumerate_solutions(F, 0, 10, 32, out=out)
    torch.cuda.synchronize()
    assert bool((out == -7).all())


def test_rank_above_62_is_erange():
    A = random_symmetric(100, 1, 0.5)
    Fo = O.factor(A)
    assert Fo["rank"] > 62
    F, _ = gpu_factor(A)
    out = torch.full((8, 2), -1, dtype=torch.int64, device="cuda")
    print("[enum] r>62", flush=True)
    hlf.enumerate_solutions(F, 0, 8, 128, out=out)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_ERANGE
    assert bool((out == -1).all())


def test_invalid_matrix_propagates_status():
    A = grid_instance(4, seed=1)
    A[0, 5] = 1  # not symmetric
    F, st = gpu_factor(A)
    assert st == hlf.HLF_ENOTSYM
    assert int(F.status.item()) == hlf.HLF_ENOTSYM
    out = torch.full((16,), -3, dtype=torch.int32, device="cuda")
    hlf.enumerate_solutions(F, 0, 16, 32, out=out)
    torch.cuda.synchronize()
    assert bool((out == -3).all())
    assert int(F.status.item()) == hlf.HLF_ENOTSYM


# -- the paper's circuit in counter order (hlf_enumerate_circuit) ----------------

def gpu_rows(A):
    from gpu_util import device_matrix
    rows, _ = hlf.pack_dense(device_matrix(A))
    return rows


@pytest.mark.parametrize("seed", CONFIG2_SEEDS)
def test_circuit_counter_order_config2(seed):
    A = grid_instance(5, seed=seed)
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    print(f"[circuit] config2 seed={seed} r={r}", flush=True)
    out = hlf.enumerate_circuit(F, gpu_rows(A), 5, 0, 1 << r, 32)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_OK
    got = narrow_to_u64(out)
    assert np.array_equal(got, C.enumerate_counter_range(Fo, 0, 1 << r)[:, 0])
    if seed == 0:  # same set as the Gray-order materialisation
        gray = narrow_to_u64(gpu_enum(F, 0, 1 << r, 32))
        assert np.array_equal(np.sort(got), np.sort(gray))


@pytest.mark.parametrize("name,N,A", [
    ("2x2 b=1011", 2, grid_instance(2, b="1011")),
    ("3x3 p=0.5", 3, grid_instance(3, p=0.5, seed=2)),
    ("4x4 paper 0^15 1", 4, grid_instance(4, b="0" * 15 + "1")),
    ("8x8 p=0.5", 8, grid_instance(8, p=0.5, seed=5)),
])
def test_circuit_matches_literal_python_circuit(name, N, A):
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    n = N * N
    wb = 16 if n <= 16 else 32 if n <= 32 else 64
    count = min(1 << r, 2000)
    print(f"[circuit] {name} r={r}", flush=True)
    out = hlf.enumerate_circuit(F, gpu_rows(A), N, 0, count, wb)
    torch.cuda.synchronize()
    assert [int(v) for v in narrow_to_u64(out)] == O.enumerate_counter_order(A, Fo, 0, count)
    if r > 14:
        b0 = ((1 << r) - 4096) & ~7
        out2 = hlf.enumerate_circuit(F, gpu_rows(A), N, b0, 4096, wb)
        torch.cuda.synchronize()
        assert np.array_equal(narrow_to_u64(out2), C.enumerate_counter_range(Fo, b0, 4096)[:, 0])


def test_circuit_ragged_ranges():
    A = grid_instance(5, seed=1)
    Fo = O.factor(A)
    r = Fo["rank"]
    F, _ = gpu_factor(A)
    rows = gpu_rows(A)
    for begin, count in [(0, 1), (4, 4095), (8, 4096 * 5 + 3), ((1 << r) - 12, 12), (1 << 20, (1 << 20) + 5)]:
        print(f"[circuit] ragged begin={begin} count={count}", flush=True)
        out = hlf.enumerate_circuit(F, rows, 5, begin, count, 32)
        torch.cuda.synchronize()
        assert np.array_equal(narrow_to_u64(out), C.enumerate_counter_range(Fo, begin, count)[:, 0])


def test_circuit_rejects_non_grid_and_bad_arguments():
    A = grid_instance(3, p=1.0, seed=0)
    A[0, 5] = A[5, 0] = 1  # an edge that is not a grid edge
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK and int(F.status.item()) == hlf.HLF_OK
    out = torch.full((16,), -4, dtype=torch.int16, device="cuda")
    hlf.enumerate_circuit(F, gpu_rows(A), 3, 0, 16, 16, out=out)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_EINVAL
    assert bool((out == -4).all())
    G, _ = gpu_factor(grid_instance(3, seed=1))
    with pytest.raises(hlf.HlfError):
        hlf.enumerate_circuit(G, gpu_rows(grid_instance(3, seed=1)), 4, 0, 16, 16)  # N^2 != n
    with pytest.raises(hlf.HlfError):
        hlf.enumerate_circuit(G, gpu_rows(grid_instance(3, seed=1)), 3, 3, 16, 16)  # begin % 8


@pytest.mark.parametrize("N,edges,loops,seed", [(9, 12, 3, 1), (10, 10, 5, 2), (16, 14, 4, 3),
                                                (23, 16, 2, 4), (32, 12, 6, 5)])
def test_circuit_multiword_grids(N, edges, loops, seed):
    """n > 64 (W = 2..16 words): the circuit's layers as multi-word shifts,
    every word against the C oracle's counter order (itself pinned to the
    layer-by-layer circuit), for full tiles and ragged ranges."""
    A = sparse_grid_instance(N, edges, seed, loops)
    Fo = O.factor(A)
    r, W = Fo["rank"], Fo["words"]
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK and 1 <= r <= 40
    rows = gpu_rows(A)
    total = 1 << r
    ranges = [(0, min(total, 5000)), (3, min(total - 3, 1 << 14)), (max(0, total - 1029), min(total, 1029))]
    if total > (1 << 16):
        ranges.append((total // 2 + 7, 70000))
    for begin, count in ranges:
        print(f"[circuit] multiword N={N} W={W} r={r} begin={begin} count={count}", flush=True)
        out = hlf.enumerate_circuit(F, rows, N, begin, count, 64 * W)
        torch.cuda.synchronize()
        assert int(F.status.item()) == hlf.HLF_OK
        assert np.array_equal(hlf.as_uint64(out).reshape(count, W), C.enumerate_counter_range(Fo, begin, count))
    # the literal Python circuit (vertex by vertex, O(n^2) per index) on the first indices
    k = 64 if N * N <= 256 else 4
    out = hlf.enumerate_circuit(F, rows, N, 0, k, 64 * W)
    torch.cuda.synchronize()
    assert words_to_ints(hlf.as_uint64(out).reshape(k, W)) == O.enumerate_counter_order(A, Fo, 0, k)


def test_circuit_multiword_rejects_non_grid():
    A = sparse_grid_instance(12, 10, 9)
    A[0, 40] = A[40, 0] = 1  # not a grid edge
    F, st = gpu_factor(A)
    assert st == hlf.HLF_OK
    out = torch.full((256, 3), -4, dtype=torch.int64, device="cuda")
    hlf.enumerate_circuit(F, gpu_rows(A), 12, 0, 256, 192, out=out)
    torch.cuda.synchronize()
    assert int(F.status.item()) == hlf.HLF_EINVAL
    assert bool((out == -4).all())
    G, _ = gpu_factor(sparse_grid_instance(12, 10, 8))
    with pytest.raises(hlf.HlfError):
        hlf.enumerate_circuit(G, gpu_rows(sparse_grid_instance(12, 10, 8)), 12, 0, 16, 64)  # word_bits != 64*W
