"""Seeded synthetic instances of the 2D hidden-linear-function (HLF) problem.

This module is shared by the CPU oracle, the tests and the benchmark.  It only
draws inputs: it holds none of the method's arithmetic (no rank, no kernel, no
enumeration).

Conventions (the paper gives the instance class, Section 1 and Fig. 1(a), and
the diagonal strings of its experiments, Section 4 and Appendix C):

* An N x N grid has n = N*N vertices.  Vertex j (0-based) sits at grid row
  j // N and column j % N (row-major).  Vertex j corresponds to the paper's
  vertex v_{j+1} and to bit z_{j+1} of a solution.  Appendix B puts v_{t+N}
  directly below v_t, which is what row-major order gives.
* The off-diagonal part of A holds the grid edges; the diagonal holds the
  vertex colours b_i = A_ii (Section 1).
* Random instances use ``numpy.random.default_rng(seed)``: first
  ``b = rng.integers(0, 2, size=n)``; then, only when the edge probability p is
  below one, ``keep = rng.random(2*N*(N-1)) < p`` over the edge list, which
  is built per vertex in row-major order as (right edge, down edge).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "grid_edges",
    "grid_instance",
    "paper_diagonal",
    "random_symmetric",
    "sparse_grid_instance",
    "batch_instances",
    "serve_requests",
    "CONFIG2_SEEDS",
    "CONFIG3_SEEDS",
]

# Seeds of the benchmark workloads.
CONFIG2_SEEDS = tuple(range(8))  # N=5, all edges
CONFIG3_SEEDS = tuple(range(4))  # N=6, p=0.5


def grid_edges(N: int) -> list[tuple[int, int]]:
    """All nearest-neighbour edges of an N x N grid, per vertex (right, down)."""
    edges = []
    for j in range(N * N):
        row, col = divmod(j, N)
        if col < N - 1:
            edges.append((j, j + 1))
        if row < N - 1:
            edges.append((j, j + N))
    return edges


def paper_diagonal(n: int, ones_at_end: int) -> np.ndarray:
    """The diagonal strings of the experiments: 0^(n-m) 1^(m) (Section 4, App. C).

    ``0^(15)1`` on a 4x4 grid is ``paper_diagonal(16, 1)``: b_16 = 1, the
    bottom-right vertex.
    """
    b = np.zeros(n, dtype=np.uint8)
    if ones_at_end:
        b[n - ones_at_end:] = 1
    return b


def grid_instance(N: int, p: float = 1.0, seed: int | None = None,
                  b=None) -> np.ndarray:
    """Adjacency matrix A (uint8, n x n, symmetric) of an N x N grid instance.

    Either ``b`` is given (a 0/1 sequence of length n, or a string such as
    "1011" read as b_1 b_2 ... b_n), or it is drawn from ``seed``.  With p < 1
    each edge is kept independently with probability p (drawn after b).
    """
    n = N * N
    rng = np.random.default_rng(seed) if seed is not None else None
    if b is None:
        if rng is None:
            raise ValueError("either b or seed is required")
        bvec = rng.integers(0, 2, size=n).astype(np.uint8)
    else:
        if isinstance(b, str):
            bvec = np.array([int(ch) for ch in b], dtype=np.uint8)
        else:
            bvec = np.asarray(b, dtype=np.uint8).copy()
        if bvec.shape != (n,):
            raise ValueError(f"b must have {n} entries")
    edges = grid_edges(N)
    if p < 1.0:
        if rng is None:
            rng = np.random.default_rng(0 if seed is None else seed)
        keep = rng.random(len(edges)) < p
    else:
        keep = np.ones(len(edges), dtype=bool)
    A = np.zeros((n, n), dtype=np.uint8)
    for (u, v), k in zip(edges, keep):
        if k:
            A[u, v] = 1
            A[v, u] = 1
    A[np.arange(n), np.arange(n)] = bvec
    return A


def sparse_grid_instance(N: int, edges: int, seed: int, loops: int = 0) -> np.ndarray:
    """An N x N grid subgraph with `edges` distinct grid edges and `loops`
    coloured vertices drawn uniformly (a small rank at large n, so that all
    solutions of a large grid can be traversed)."""
    rng = np.random.default_rng(seed)
    E = grid_edges(N)
    A = np.zeros((N * N, N * N), dtype=np.uint8)
    for k in rng.choice(len(E), size=edges, replace=False):
        u, v = E[k]
        A[u, v] = A[v, u] = 1
    for v in rng.choice(N * N, size=loops, replace=False):
        A[v, v] = 1
    return A


def random_symmetric(n: int, seed: int, density: float = 0.5) -> np.ndarray:
    """A dense random symmetric 0/1 matrix (any graph with self-loops)."""
    rng = np.random.default_rng(seed)
    upper = (rng.random((n, n)) < density).astype(np.uint8)
    A = np.triu(upper)
    A = A | A.T
    return A.astype(np.uint8)


def low_rank_symmetric(n: int, k: int, seed: int) -> np.ndarray:
    """A symmetric 0/1 matrix of rank at most k: A = M^T M mod 2 with M a
    uniform random k x n 0/1 matrix (a graph whose adjacency has a small
    GF(2) rank, so all of its solutions can be enumerated at large n)."""
    rng = np.random.default_rng(seed)
    M = rng.integers(0, 2, size=(k, n)).astype(np.int64)
    return ((M.T @ M) % 2).astype(np.uint8)


def batch_instances(count: int = 4096, master_seed: int = 0):
    """The batched workload: grid side N ~ U{3..12}, p ~ U{0.3, 0.5, 1.0}.

    Returns a list of (N, p, seed, A).
    """
    rng = np.random.default_rng(master_seed)
    Ns = rng.integers(3, 13, size=count)
    ps = rng.choice(np.array([0.3, 0.5, 1.0]), size=count)
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for N, p, s in zip(Ns, ps, seeds):
        out.append((int(N), float(p), int(s), grid_instance(int(N), float(p), int(s))))
    return out


def serve_requests(count: int, rate_per_s: float, master_seed: int = 0,
                   n_min: int = 4, n_max: int = 32, p: float = 0.5):
    """Poisson-arrival request stream: N ~ U{n_min..n_max}, edge probability p.

    Returns a list of dicts with keys ``t`` (arrival time in seconds from the
    start), ``N``, ``seed`` and ``A``.
    """
    rng = np.random.default_rng(master_seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    Ns = rng.integers(n_min, n_max + 1, size=count)
    seeds = rng.integers(0, 2**62, size=count)
    reqs = []
    for k in range(count):
        reqs.append({"t": float(t[k]), "N": int(Ns[k]), "seed": int(seeds[k]),
                     "A": grid_instance(int(Ns[k]), p, int(seeds[k]))})
    return reqs
