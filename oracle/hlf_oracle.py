"""Plain CPU oracle of the FS2D HLF method -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It is slow on purpose: every function is the textbook definition of
what it computes, written so that it can be checked against the paper by eye.

Notation (Section 1 and 2 of the paper): A is an n x n symmetric binary
matrix, b_i = A_ii, Ker(A) = {x : Ax = 0 mod 2}, q(x) = x^T A x mod 4 computed
over the integers, r = rank of A over GF(2), P = (p_1 < ... < p_r) the pivot
positions, L_ind the columns of A at P, z^a one solution.

Bit vectors are Python ints: bit j (LSB first) holds z_{j+1}, i.e. vertex j
in 0-based numbering.  A word-packed form splits an int into W = ceil(n/64)
64-bit words, word w holding bits 64w .. 64w+63.

Conventions where the paper leaves a free choice (each is a reading, listed
with its justification in the design notes):

* shift ``l``: the unique solution with l_p = 0 for every pivot p.  It
  satisfies l_f = q(k_f)/2 for every free column f, where k_f is the Ker(A)
  basis vector that is 1 at f and 0 at the other free columns.
* basis ``B_k`` = column p_k of A (k = 0..r-1, ascending p_k).
* enumeration order: index i in [0, 2^r) maps to the coefficient vector
  g(i) = i XOR (i >> 1) (binary reflected Gray code); bit k of g(i) is the
  paper's R_{p_{k+1}}.  ``counter order`` uses i itself, as the FPGA's binary
  counter does (Section 4).
* hash of one solution: h_0 = 0, h_{w+1} = mix13(h_w XOR z_w XOR GAMMA) over
  the W words of z, h(z) = h_W; the hash of a set is the sum of h(z) mod 2^64.
  mix13 is the output function of Vigna's public-domain SplitMix64
  (Stafford's "Mix13" variant of the MurmurHash3 64-bit finaliser); GAMMA is
  SplitMix64's increment 0x9E3779B97F4A7C15.
* sampling coefficients: word w of the coefficient vector of sample s is the
  SplitMix64 output number s*ceil(r/64) + w of the generator whose state
  starts at ``seed``, i.e. mix13(seed + (s*ceil(r/64) + w + 1) * GAMMA); the
  bits at positions >= r of the last word are cleared.

Parity pins: every function here is pinned by a test in
``tests/test_oracle_pins.py`` against values the paper prints (Fig. 3, App. C,
Section 4), closed forms (App. B rank interval, counts, XOR-fold), brute force
over the problem definition, and the state-vector simulation of App. A.
"""

from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MIX_M1 = 0xBF58476D1CE4E5B9
MIX_M2 = 0x94D049BB133111EB


# ----------------------------------------------------------------------------
# Problem statement (Section 1)
# ----------------------------------------------------------------------------

def validate(A) -> np.ndarray:
    """A must be a square, symmetric 0/1 matrix (Section 1)."""
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if A.shape[0] < 1:
        raise ValueError("A must have at least one row")
    if not np.all((A == 0) | (A == 1)):
        raise ValueError("A must be binary")
    if not np.array_equal(A, A.T):
        raise ValueError("A must be symmetric")
    return A.astype(np.uint8)


def q_form(A, x) -> int:
    """q(x) = x^T A x mod 4 over the integers (Section 1)."""
    A = np.asarray(A, dtype=np.int64)
    xv = np.asarray(x, dtype=np.int64)
    return int(xv @ A @ xv) % 4


def kernel_vectors_all(A) -> list[np.ndarray]:
    """Every x in {0,1}^n with A x = 0 mod 2, by exhaustive search (tiny n)."""
    A = validate(A)
    n = A.shape[0]
    out = []
    for v in range(1 << n):
        x = np.array([(v >> j) & 1 for j in range(n)], dtype=np.int64)
        if not np.any((A.astype(np.int64) @ x) % 2):
            out.append(x)
    return out


def brute_force_solutions(A) -> set[int]:
    """All z in {0,1}^n with q(x) = 2 z.x mod 4 for every x in Ker(A).

    The problem definition of Section 1, checked over every kernel vector and
    every candidate z.  Exponential in n: use for n <= 12 only.
    """
    A = validate(A)
    n = A.shape[0]
    ker = kernel_vectors_all(A)
    qs = [q_form(A, x) for x in ker]
    sols = set()
    for zv in range(1 << n):
        z = np.array([(zv >> j) & 1 for j in range(n)], dtype=np.int64)
        if all((2 * int(z @ x)) % 4 == qx for x, qx in zip(ker, qs)):
            sols.add(zv)
    return sols


# ----------------------------------------------------------------------------
# Stage 1: the CLA module (Section 2, tasks (1)-(4))
# ----------------------------------------------------------------------------

def rref_gf2(A):
    """Reduced row echelon form of A over GF(2), textbook Gauss-Jordan.

    Returns (R, pivots): R holds the r nonzero rows of the RREF, pivots the
    ascending pivot columns.  The pivot columns are the positions P of the
    maximal independent column set L_ind of task (1) in Section 2 (row
    operations keep the linear relations among columns).
    """
    M = (np.asarray(A, dtype=np.uint8) % 2).copy()
    rows, cols = M.shape
    pivots = []
    top = 0
    for c in range(cols):
        if top == rows:
            break
        hits = np.nonzero(M[top:, c])[0]
        if hits.size == 0:
            continue
        p = top + int(hits[0])
        if p != top:
            M[[top, p]] = M[[p, top]]
        for i in range(rows):
            if i != top and M[i, c]:
                M[i] ^= M[top]
        pivots.append(c)
        top += 1
    return M[:top].copy(), pivots


def independent_columns_greedy(A) -> list[int]:
    """Lexicographically first maximal independent column set, greedily.

    Column c is taken iff it is not in the span of the columns taken before
    it.  A second, independent route to the pivot set P of task (1).
    """
    A = validate(A)
    n = A.shape[0]
    taken = []
    span_basis = {}  # leading bit -> vector (an echelon basis of the span)
    for c in range(n):
        v = 0
        for i in range(n):
            if A[i, c]:
                v |= 1 << i
        w = v
        while w:
            lead = w.bit_length() - 1
            if lead in span_basis:
                w ^= span_basis[lead]
            else:
                break
        if w:
            span_basis[w.bit_length() - 1] = w
            taken.append(c)
    return taken


def kernel_basis(A):
    """Basis of L_q = Ker(A), task (2) of Section 2.

    For every free (non-pivot) column f in ascending order, k_f is 1 at f, 0 at
    the other free columns, and at pivot p_k equals RREF[k][f].  Returns a list
    of int bit vectors.
    """
    A = validate(A)
    n = A.shape[0]
    R, piv = rref_gf2(A)
    free = [c for c in range(n) if c not in set(piv)]
    basis = []
    for f in free:
        v = 1 << f
        for k, p in enumerate(piv):
            if R[k, f]:
                v |= 1 << p
        basis.append(v)
    return basis


def bits_to_array(v: int, n: int) -> np.ndarray:
    return np.array([(v >> j) & 1 for j in range(n)], dtype=np.int64)


def array_to_bits(x) -> int:
    v = 0
    for j, bit in enumerate(np.asarray(x).tolist()):
        if int(bit) & 1:
            v |= 1 << j
    return v


def canonical_shift(A) -> int:
    """One solution z^a, tasks (3) and (4) of Section 2.

    Task (3) evaluates q on the kernel basis; task (4) solves
    2 z^T x = q(x) mod 4 for z.  q is linear on Ker(A) with values in {0, 2}
    (proof in the cited supplementary material, Section 2), so the equations
    on the basis vectors suffice: z . k_f = q(k_f)/2 (mod 2).  With z = 0 on
    the pivot positions the system is diagonal, z_f = q(k_f)/2, because k_f is
    1 at its own free column f and 0 at every other free column.
    """
    A = validate(A)
    n = A.shape[0]
    _, piv = rref_gf2(A)
    free = [c for c in range(n) if c not in set(piv)]
    l = 0
    for f, kf in zip(free, kernel_basis(A)):
        q = q_form(A, bits_to_array(kf, n))
        if q % 2:
            raise AssertionError("q(x) is odd on a kernel vector")
        l |= (q // 2) << f
    return l


def column_basis(A) -> list[int]:
    """L_ind: the columns of A at the pivot positions, ascending (task (1))."""
    A = validate(A)
    n = A.shape[0]
    _, piv = rref_gf2(A)
    out = []
    for p in piv:
        v = 0
        for i in range(n):
            if A[i, p]:
                v |= 1 << i
        out.append(v)
    return out


def factor(A) -> dict:
    """All stage-1 quantities: rank, pivots, basis, shift, kernel basis."""
    A = validate(A)
    n = A.shape[0]
    _, piv = rref_gf2(A)
    return {
        "n": n,
        "words": (n + 63) // 64,
        "rank": len(piv),
        "pivots": list(piv),
        "basis": column_basis(A),
        "shift": canonical_shift(A),
        "kernel": kernel_basis(A),
    }


# ----------------------------------------------------------------------------
# Stage 2: the classical parallel circuit (Section 2, Eqs. (1)-(3))
# ----------------------------------------------------------------------------

def gray(i: int) -> int:
    """Binary reflected Gray code g(i) = i XOR (i >> 1)."""
    return i ^ (i >> 1)


def solution_at(F: dict, i: int) -> int:
    """Solution number i: z = z^a XOR sum_k R_{p_k} l_{p_k}, R^(r) = g(i).

    The final CNOT layer of Section 2 adds z^a to y = sum_k R_{p_k} l_{p_k}
    (Eq. (3) restricted to the pivot inputs).
    """
    coeff = gray(i)
    z = F["shift"]
    for k, Bk in enumerate(F["basis"]):
        if (coeff >> k) & 1:
            z ^= Bk
    return z


def cpc_output(A, pivots, R_bits: int, shift: int) -> int:
    """The literal stage-2 circuit of Fig. 1(c) for one input pattern.

    R^(r) = R_bits is scattered onto the pivot positions (other inputs 0);
    layers 1-4 give y_i = XOR of R_j over the neighbours j of i (Eq. (1));
    the Toffoli layer adds b_i R_i (Eq. (2)); the last CNOT layer adds z^a.
    """
    A = validate(A)
    n = A.shape[0]
    R = [0] * n
    for k, p in enumerate(pivots):
        R[p] = (R_bits >> k) & 1
    y = 0
    for i in range(n):
        yi = 0
        for j in range(n):
            if j != i and A[i, j]:
                yi ^= R[j]
        yi ^= int(A[i, i]) & R[i]
        y |= yi << i
    return y ^ shift


def enumerate_range(F: dict, begin: int, count: int) -> list[int]:
    """Solutions begin .. begin+count-1 in Gray order, by direct definition."""
    r = F["rank"]
    if begin < 0 or count < 0 or begin + count > (1 << r):
        raise ValueError("range outside [0, 2^r)")
    return [solution_at(F, i) for i in range(begin, begin + count)]


def enumerate_counter_order(A, F: dict, begin: int, count: int) -> list[int]:
    """Solutions in the FPGA's binary-counter order via the literal circuit."""
    r = F["rank"]
    if begin < 0 or count < 0 or begin + count > (1 << r):
        raise ValueError("range outside [0, 2^r)")
    return [cpc_output(A, F["pivots"], i, F["shift"]) for i in range(begin, begin + count)]


# ----------------------------------------------------------------------------
# Hash, counts, XOR-fold (reduce mode) and sampling
# ----------------------------------------------------------------------------

def mix13(x: int) -> int:
    """SplitMix64 output function (Stafford Mix13), 64-bit arithmetic."""
    x &= MASK64
    x ^= x >> 30
    x = (x * MIX_M1) & MASK64
    x ^= x >> 27
    x = (x * MIX_M2) & MASK64
    x ^= x >> 31
    return x


def splitmix64_output(seed: int, k: int) -> int:
    """Output number k (0-based) of SplitMix64 whose state starts at seed."""
    return mix13((seed + (k + 1) * GAMMA) & MASK64)


def to_words(z: int, W: int) -> list[int]:
    return [(z >> (64 * w)) & MASK64 for w in range(W)]


def hash_solution(z: int, W: int) -> int:
    """h(z): chain mix13 over the W words of z (see the module header)."""
    h = 0
    for zw in to_words(z, W):
        h = mix13(h ^ zw ^ GAMMA)
    return h


def reduce_range(F: dict, begin: int, count: int):
    """(counts, hash, xorfold) over solutions begin .. begin+count-1.

    counts[j] = number of solutions with z_{j+1} = 1; hash = sum of h(z)
    mod 2^64; xorfold = XOR of all solutions.  Plain loops over the direct
    definition.
    """
    n, W = F["n"], F["words"]
    counts = [0] * n
    h = 0
    xf = 0
    for z in enumerate_range(F, begin, count):
        for j in range(n):
            counts[j] += (z >> j) & 1
        h = (h + hash_solution(z, W)) & MASK64
        xf ^= z
    return counts, h, xf


def sample_coefficients(seed: int, r: int, s: int) -> int:
    """Coefficient vector c_s (an int of r bits) of sample s."""
    R64 = (r + 63) // 64
    c = 0
    for w in range(R64):
        c |= splitmix64_output(seed, s * R64 + w) << (64 * w)
    return c & ((1 << r) - 1)


def sample(F: dict, seed: int, num: int, coeffs=None) -> list[int]:
    """Samples z_s = l XOR sum_k c_{s,k} B_k, s = 0..num-1.

    Each c_s is uniform on {0,1}^r and c -> z is a bijection onto the solution
    set, so z_s is a uniform solution -- the output distribution of the
    quantum circuit (App. A).  ``coeffs`` (a list of ints) replaces the
    generator when given.
    """
    r = F["rank"]
    out = []
    for s in range(num):
        c = sample_coefficients(seed, r, s) if coeffs is None else (coeffs[s] & ((1 << r) - 1))
        z = F["shift"]
        for k, Bk in enumerate(F["basis"]):
            if (c >> k) & 1:
                z ^= Bk
        out.append(z)
    return out


# ----------------------------------------------------------------------------
# Distribution statistics and membership (verification, Section 5: the ideal
# output distribution as the input of a cross-entropy benchmark)
# ----------------------------------------------------------------------------

def pair_counts(F: dict):
    """C[i][j] = number of solutions with z_{i+1} = z_{j+1} = 1, by plain
    counting over every solution (direct definition, Gray order).  C[i][i] is
    the per-qubit count of reduce mode.  Python ints (exact)."""
    n, r = F["n"], F["rank"]
    C = [[0] * n for _ in range(n)]
    for z in enumerate_range(F, 0, 1 << r):
        ones = [j for j in range(n) if (z >> j) & 1]
        for i in ones:
            for j in ones:
                C[i][j] += 1
    return C


def pair_quarters(A) -> np.ndarray:
    """4 * P(z_i = z_j = 1) for a uniform solution z, in closed form.

    Writing z = l XOR sum_k c_k B_k with c uniform, coordinate i is l_i plus
    the functional c -> <c, beta_i>, beta_i = (B_k[i])_k = row i of A at the
    pivot columns.  Because the pivot columns are an information set of the
    row space, beta_i = beta_j exactly when A_i = A_j and beta_i = 0 exactly
    when A_i = 0.  Hence: a zero row gives z_i = 0 always (e_i is in Ker(A)
    with q = 0); two equal nonzero rows give z_i = z_j always (e_i + e_j is
    in Ker(A) with q = 4 A_ij = 0 mod 4), so the pair is 1 with probability
    1/2; distinct nonzero rows give independent uniform bits, probability
    1/4.  Pinned against pair_counts by brute force in the tests.
    """
    A = validate(A)
    n = A.shape[0]
    Q = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for j in range(n):
            if not A[i].any() or not A[j].any():
                Q[i, j] = 0
            elif np.array_equal(A[i], A[j]):
                Q[i, j] = 2
            else:
                Q[i, j] = 1
    return Q


def is_solution(A, z: int, kernel=None) -> bool:
    """The problem's definition (Section 1): q(x) = 2 z.x mod 4 for every x in
    Ker(A).  q is linear on Ker(A) (values in {0, 2}), so checking a basis of
    Ker(A) suffices; ``kernel`` may pass that basis (ints), else it is
    computed.  The tests pin this against all of span(Ker) for tiny n."""
    A = validate(A)
    n = A.shape[0]
    ks = kernel_basis(A) if kernel is None else kernel
    for k in ks:
        x = bits_to_array(k, n) if isinstance(k, int) else np.asarray(k)
        zx = sum(((z >> j) & 1) * int(x[j]) for j in range(n))
        if (q_form(A, x) - 2 * zx) % 4 != 0:
            return False
    return True


def linear_xeb(n: int, r: int, members) -> float:
    """Linear cross-entropy benchmark estimate 2^n * mean(p(z_s)) - 1 with
    the ideal probabilities p(z) = 2^-r on the solution set and 0 elsewhere
    (App. A): 2^(n-r) * (fraction of samples that are solutions) - 1."""
    members = list(members)
    if not members:
        raise ValueError("no samples")
    return (2.0 ** (n - r)) * (sum(1 for m in members if m) / len(members)) - 1.0


# ----------------------------------------------------------------------------
# The quantum circuit of Appendix A, as a dense state vector
# ----------------------------------------------------------------------------

def statevector_probabilities(A) -> np.ndarray:
    """Output distribution of Q_N (App. A, Eqs. (A1)-(A2)), dense, n <= 16.

    |0>^n -> H^n -> CZ on every edge (i, j), A_ij = 1 -> S on every vertex with
    A_ii = 1 -> H^n -> computational-basis probabilities.  Index v of the
    result is the bit string with z_{j+1} = bit j of v.
    """
    A = validate(A)
    n = A.shape[0]
    if n > 16:
        raise ValueError("state vector limited to n <= 16")
    dim = 1 << n
    idx = np.arange(dim, dtype=np.int64)
    psi = np.zeros(dim, dtype=np.complex128)
    psi[0] = 1.0

    def hadamard_all(v):
        v = v.copy()
        for q in range(n):
            v = v.reshape(-1, 2, 1 << q)
            a = v[:, 0, :].copy()
            b = v[:, 1, :].copy()
            v[:, 0, :] = (a + b) / np.sqrt(2.0)
            v[:, 1, :] = (a - b) / np.sqrt(2.0)
            v = v.reshape(dim)
        return v

    psi = hadamard_all(psi)
    for i in range(n):
        for j in range(i + 1, n):
            if A[i, j]:
                both = ((idx >> i) & 1) & ((idx >> j) & 1)
                psi = np.where(both == 1, -psi, psi)
    for i in range(n):
        if A[i, i]:
            psi = np.where(((idx >> i) & 1) == 1, 1j * psi, psi)
    psi = hadamard_all(psi)
    return np.abs(psi) ** 2
