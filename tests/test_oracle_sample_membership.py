"""Pins of the C oracle's sampler and membership check (test infrastructure).

Sampler (uniform single solutions, App. A): z_s = l XOR (XOR over set bits k
of c_s of B_k).  Pinned by
* the published SplitMix64 outputs (Vigna's splitmix64.c, state 0) read back
  through an identity basis, which fixes the generator, the word order of a
  coefficient vector and the clearing of bits >= r without the Python oracle;
* unit and zero coefficient vectors (closed form l XOR B_k, l);
* every sample satisfying every kernel equation (Section 1's definition);
* agreement with the Python oracle's sampler, seed stream and explicit
  coefficients, from one to sixteen words.
Membership (Section 1: q(x) = 2 z.x mod 4 on Ker(A)) is pinned against the
brute-force solution set on tiny n and the Python oracle's definition.
"""

import numpy as np
import pytest

from hlf_inputs import grid_instance, paper_diagonal, random_symmetric
from oracle import c_oracle as C
from oracle import hlf_oracle as O

MASK64 = (1 << 64) - 1
SPLITMIX_STATE0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def ints(a):
    a = np.asarray(a, dtype=np.uint64)
    return [sum(int(a[k, w]) << (64 * w) for w in range(a.shape[1])) for k in range(a.shape[0])]


def identity_record(n, r):
    return {"n": n, "words": (n + 63) // 64, "rank": r, "basis": [1 << k for k in range(r)],
            "shift": 0}


def test_sampler_reads_back_published_splitmix64_outputs():
    # r = 64, basis e_0..e_63: sample s is the coefficient word itself.
    got = ints(C.sample(identity_record(64, 64), 0, 3))
    assert got == SPLITMIX_STATE0
    # r = 128: sample 0 holds outputs 0 (bits 0-63) and 1 (bits 64-127),
    # sample 1 outputs 2 and 3.
    z = ints(C.sample(identity_record(128, 128), 0, 2))
    assert z[0] & MASK64 == SPLITMIX_STATE0[0] and z[0] >> 64 == SPLITMIX_STATE0[1]
    assert z[1] & MASK64 == SPLITMIX_STATE0[2]
    # r = 100: coefficient bits >= 100 are cleared
    z = ints(C.sample(identity_record(128, 100), 0, 1))[0]
    assert z == (SPLITMIX_STATE0[0] | (SPLITMIX_STATE0[1] << 64)) & ((1 << 100) - 1)


@pytest.mark.parametrize("A", [grid_instance(4, seed=0), random_symmetric(100, 5, 0.5),
                               grid_instance(20, p=0.5, seed=3)])
def test_unit_and_zero_coefficients(A):
    F = O.factor(A)
    r, W = F["rank"], F["words"]
    R64 = (r + 63) // 64
    coeffs = np.zeros((r + 1, R64), dtype=np.uint64)
    for k in range(r):
        coeffs[k, k // 64] = np.uint64(1) << np.uint64(k % 64)
    z = ints(C.sample(F, 0, r + 1, coeffs=coeffs))
    assert z[:r] == [F["shift"] ^ B for B in F["basis"]]
    assert z[r] == F["shift"]
    assert all(v < (1 << F["n"]) for v in z)
    del W


CASES = {
    "N=4 seed 0": lambda: grid_instance(4, seed=0),
    "random n=100": lambda: random_symmetric(100, 5, 0.5),
    "grid N=20 p=0.5": lambda: grid_instance(20, p=0.5, seed=3),
    "grid N=32 p=0.5 (r=953)": lambda: grid_instance(32, p=0.5, seed=17),
    "random n=1024 (r=1024)": lambda: random_symmetric(1024, 8, 0.5),
    "zero n=7": lambda: np.zeros((7, 7), dtype=np.uint8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_c_sampler_equals_python_sampler(name):
    A = CASES[name]()
    F = O.factor(A)
    r = F["rank"]
    num = 97
    assert ints(C.sample(F, 0xC0FFEE, num)) == O.sample(F, 0xC0FFEE, num)
    rng = np.random.default_rng(r)
    R64 = max((r + 63) // 64, 1)
    coeffs = rng.integers(0, 2**63, size=(num, R64), dtype=np.int64).view(np.uint64)
    coeffs[:, 0] ^= np.uint64(1) << np.uint64(63)
    if r > 0:
        assert ints(C.sample(F, 0, num, coeffs=coeffs)) == O.sample(F, 0, num, coeffs=ints(coeffs))


def test_c_samples_satisfy_every_kernel_equation_n1024():
    A = grid_instance(32, p=0.5, seed=17)
    F = O.factor(A)
    Z = C.sample(F, 42, 4096)
    free = [c for c in range(1024) if c not in set(F["pivots"])]
    for f, kf in zip(free, F["kernel"]):
        kw = np.array([(kf >> (64 * w)) & MASK64 for w in range(16)], dtype=np.uint64)
        parity = np.bitwise_count(Z & kw).sum(axis=1) & 1
        assert np.all(parity == ((F["shift"] >> f) & 1)), f
    assert len(set(ints(Z))) == 4096  # 2^953 solutions: no repeats expected


def _q(A, F):
    n = A.shape[0]
    return [O.q_form(A, O.bits_to_array(k, n)) for k in F["kernel"]]


@pytest.mark.parametrize("A", [random_symmetric(n, seed=80 + n, density=0.4) for n in (1, 5, 9, 12)]
                         + [grid_instance(3, p=1.0, seed=0), grid_instance(3, b=paper_diagonal(9, 2)),
                            np.zeros((6, 6), dtype=np.uint8)])
def test_c_membership_equals_brute_force(A):
    n = A.shape[0]
    F = O.factor(A)
    allz = np.arange(1 << n, dtype=np.uint64).reshape(-1, 1)
    m = C.membership(F["kernel"], _q(A, F), 1, allz)
    assert [z for z in range(1 << n) if m[z]] == sorted(O.brute_force_solutions(A))


@pytest.mark.parametrize("A", [random_symmetric(100, 3, 0.3), grid_instance(12, p=0.5, seed=4),
                               grid_instance(20, p=0.5, seed=5)])
def test_c_membership_equals_python_definition(A):
    n = A.shape[0]
    F = O.factor(A)
    W = F["words"]
    rng = np.random.default_rng(n)
    members = O.sample(F, 9, 60)
    flips = [z ^ (1 << int(rng.integers(n))) for z in members[:30]]
    flips += [z ^ (1 << int(rng.integers(n))) ^ (1 << int(rng.integers(n))) for z in members[30:]]
    uniform = [int.from_bytes(rng.bytes((n + 7) // 8), "little") & ((1 << n) - 1) for _ in range(30)]
    zs = members + flips + uniform
    words = np.array([[(z >> (64 * w)) & MASK64 for w in range(W)] for z in zs], dtype=np.uint64)
    m = C.membership(F["kernel"], _q(A, F), W, words)
    assert [bool(v) for v in m] == [O.is_solution(A, z, kernel=F["kernel"]) for z in zs]
    assert all(m[:60])
