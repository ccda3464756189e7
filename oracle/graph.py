"""Graph and operator (Sec. 2.1).

The paper works with an undirected graph, its adjacency A (a_ij > 0 on edges),
the degree matrix D_ii = sum_j a_ij, and -- in every experiment -- the
normalized adjacency  Abar = D^{-1/2} A D^{-1/2}, whose spectrum lies in [-1, 1].

Readings fixed here (the paper is silent on input cleaning):
* the edge list is symmetrised and treated as a *set*: duplicates collapse to
  weight 1, self-loops are dropped (unweighted pattern);
* isolated nodes (degree 0, where D^{-1/2} is undefined) are dropped and the
  survivors relabelled 0..N-1 in ascending order of their original id;
* CSR rows list their columns in ascending order;
* the per-node scale shipped to the GPU is fp32(1/sqrt(d)) with the inverse
  square root taken in fp64 (correctly rounded) and then rounded to fp32.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Graph:
    n: int                 # nodes after dropping isolated ones
    row_ptr: np.ndarray    # int64 [n+1]
    col: np.ndarray        # int32 [nnz], ascending within a row
    deg: np.ndarray        # int64 [n]
    old_id: np.ndarray     # int32 [n], original id of each kept node (ascending)
    dinv_sqrt: np.ndarray  # float32 [n] = fp32(1/sqrt(fp64 d))

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def neighbors(self, i: int) -> np.ndarray:
        return self.col[self.row_ptr[i]:self.row_ptr[i + 1]]


def build_csr(n_nodes: int, src, dst) -> Graph:
    """Symmetric simple graph from an undirected edge list (set semantics)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n_nodes or dst.max() >= n_nodes):
        raise ValueError("node id out of range")
    keep = src != dst
    u = np.concatenate([src[keep], dst[keep]])
    v = np.concatenate([dst[keep], src[keep]])
    key = np.unique(u * np.int64(n_nodes) + v)  # sorted set of directed pairs
    u = key // n_nodes
    v = key % n_nodes
    present = np.zeros(n_nodes, dtype=bool)
    present[u] = True
    old_id = np.flatnonzero(present)
    new_of_old = np.full(n_nodes, -1, dtype=np.int64)
    new_of_old[old_id] = np.arange(old_id.size)
    row = new_of_old[u]
    col = new_of_old[v]
    n = int(old_id.size)
    deg = np.bincount(row, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    dinv = (1.0 / np.sqrt(deg.astype(np.float64))).astype(np.float32)
    return Graph(n, row_ptr, col.astype(np.int32), deg, old_id.astype(np.int32), dinv)


def normalized_adjacency(g: Graph) -> sp.csr_matrix:
    """H = D^{-1/2} A D^{-1/2} in fp64 (Sec. 2.1), A the 0/1 pattern."""
    d = 1.0 / np.sqrt(g.deg.astype(np.float64))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    vals = d[rows] * d[g.col.astype(np.int64)]
    return sp.csr_matrix((vals, g.col.astype(np.int64), g.row_ptr), shape=(g.n, g.n))


def neighbor_sets_from_edges(src, dst, nodes) -> dict:
    """N(v) (sorted array of input ids) for each input id v in `nodes`, read
    straight from an edge list (symmetrised, deduplicated, self-loops
    dropped).  Used for sampled checks on graphs too large to build here."""
    src = np.asarray(src)
    dst = np.asarray(dst)
    nodes = np.unique(np.asarray(nodes, dtype=np.int64))
    m1 = np.isin(src, nodes, kind="table")
    m2 = np.isin(dst, nodes, kind="table")
    a = np.concatenate([src[m1], dst[m2]]).astype(np.int64)
    b = np.concatenate([dst[m1], src[m2]]).astype(np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    base = np.int64(max(int(src.max(initial=0)), int(dst.max(initial=0))) + 1)
    key = np.unique(a * base + b)
    a, b = key // base, key % base
    starts = np.searchsorted(a, nodes, side="left")
    ends = np.searchsorted(a, nodes, side="right")
    return {int(v): b[s0:s1] for v, s0, s1 in zip(nodes, starts, ends)}


def compact_ids_from_edges(n_nodes: int, src, dst) -> np.ndarray:
    """Compact id of every input id (-1 for isolated ones): the rank among the
    ids that have at least one non-loop edge (ascending), as in build_csr."""
    src = np.asarray(src)
    dst = np.asarray(dst)
    keep = src != dst
    present = np.zeros(n_nodes, dtype=bool)
    present[src[keep]] = True
    present[dst[keep]] = True
    cid = np.cumsum(present, dtype=np.int64) - 1
    cid[~present] = -1
    return cid
