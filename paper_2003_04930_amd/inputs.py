"""Seeded synthetic inputs for the quantum-PageRank solver.

This module only *draws* inputs: directed graphs as (src, dst) edge lists and
random density matrices.  It holds none of the method's arithmetic (no Google
matrix, no Hamiltonian, no Lindblad right-hand side), so both the HIP path and
the CPU oracle may consume what it produces.

Edge convention: an edge ``src -> dst`` is a connection from node ``src`` to
node ``dst`` (Supplementary Note 1: A_ij = 1 when node j links to node i, so
the edge sets A[dst, src]).

Workloads (the paper measures on the USA airline network, N = 922, which is not
available; the scale-free generator below stands in for it at the same N):

* ``er_digraph(16, 0.2, seed=0)``      directed Erdos-Renyi, N = 16.
* ``ba_digraph(922, 3, seed=0)``       Barabasi-Albert m = 3, every undirected
  edge given a random direction, 10 % made reciprocal.
* ``ba_digraph(2048|4096, 4, seed=0)`` the same recipe with m = 4.
* ``batch_graph(k)``                   the mixed ER/BA family of the batched
  solve: N uniform in [50, 922].
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Graph", "er_digraph", "ba_digraph", "family_graph", "batch_graph", "batch_set",
    "random_density", "random_hermitian", "BATCH_OMEGAS",
]

BATCH_OMEGAS = (0.1, 0.3, 0.5, 0.7, 0.9)


class Graph:
    """A directed graph on ``n`` nodes given as int32 edge arrays."""

    __slots__ = ("n", "src", "dst", "name")

    def __init__(self, n: int, src, dst, name: str = ""):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.name = name

    @property
    def n_edges(self) -> int:
        return int(self.src.size)

    def relabel(self, perm) -> "Graph":
        """Graph with node v renamed perm[v]."""
        perm = np.asarray(perm, dtype=np.int32)
        return Graph(self.n, perm[self.src], perm[self.dst], self.name + "-perm")

    def __repr__(self) -> str:
        return f"Graph({self.name or 'anon'}, n={self.n}, E={self.n_edges})"


def er_digraph(n: int, p: float, seed: int = 0) -> Graph:
    """Directed Erdos-Renyi graph.

    Ordered pairs (i, j), i != j, are scanned row-major; with probability p the
    edge j -> i is added.  One uniform draw per ordered pair, in scan order.
    """
    rng = np.random.default_rng(seed)
    u = rng.random(n * (n - 1))
    ii, jj = np.nonzero(~np.eye(n, dtype=bool))   # row-major, diagonal skipped
    keep = u < p
    return Graph(n, jj[keep], ii[keep], f"er{n}-p{p:g}-s{seed}")


def ba_digraph(n: int, m: int, seed: int = 0, reciprocal: float = 0.1) -> Graph:
    """Scale-free directed graph.

    An undirected Barabasi-Albert graph (networkx, m edges per new node) is
    drawn; for every edge in ``g.edges()`` order a fair coin picks the
    direction and, with probability ``reciprocal``, the reverse edge is added
    too.
    """
    import networkx as nx

    g = nx.barabasi_albert_graph(n, m, seed=seed)
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for (u, v) in g.edges():
        s, d = (u, v) if rng.random() < 0.5 else (v, u)
        src.append(s)
        dst.append(d)
        if rng.random() < reciprocal:
            src.append(d)
            dst.append(s)
    return Graph(n, src, dst, f"ba{n}-m{m}-s{seed}")


def family_graph(seed: int) -> Graph:
    """One graph of the mixed family with an explicit seed, N ~ U{50..922}.

    Even seed: ER with edge probability 4/(N-1) (mean out-degree 4).
    Odd seed: BA with m ~ U{2..5}, directed as in :func:`ba_digraph`.
    """
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50, 923))
    if seed % 2 == 0:
        return er_digraph(n, 4.0 / (n - 1), seed=seed)
    m = int(rng.integers(2, 6))
    return ba_digraph(n, m, seed=seed)


def batch_graph(k: int) -> Graph:
    """Graph k of the batched workload: the family graph with seed 1000 + k."""
    return family_graph(1000 + k)


def batch_set(count: int, first: int = 0):
    """[(graph, omega)] for graphs first..first+count-1, each at the five batch omegas."""
    out = []
    for k in range(first, first + count):
        g = batch_graph(k)
        for w in BATCH_OMEGAS:
            out.append((g, w))
    return out


def random_hermitian(n: int, seed: int = 0) -> np.ndarray:
    """Random complex Hermitian matrix with standard-normal entries (complex128)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (x + x.conj().T)


def random_density(n: int, seed: int = 0, rank: int | None = None) -> np.ndarray:
    """Random density matrix X X^dagger / tr (complex128, trace 1); X is n x n
    (full rank) or n x rank."""
    rng = np.random.default_rng(seed)
    k = n if rank is None else rank
    x = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    r = x @ x.conj().T
    r = 0.5 * (r + r.conj().T)
    return r / np.trace(r).real
