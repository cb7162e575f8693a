"""Symmetric joint probabilities p_ij in CSR form (oracle side).

Eq. (2): p_ij = (p_{j|i} + p_{i|j}) / (2n). The support is the union of every
selected pair (i, j), j in N_k(i), and its transpose; entries that are zero
(levels past the first in a HIGH row) stay in the support.

Reading for rows with no neighbours: an isolated vertex has no p_{.|i}, so the
plain 2n denominator would leave sum(P) < 1. The denominator used is twice the
number of non-empty rows of the graph, which equals 2n when every vertex has
an edge and keeps sum(P) = 1 otherwise. In a batch of graphs each graph is
normalised on its own.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .neighbours import k_from_perplexity, select_all
from .perplexity import STATUS_EMPTY, row_probabilities
from .tiebreak import TIE_HASH


@dataclass
class OracleP:
    rowptr: np.ndarray        # int64 [n+1]
    col: np.ndarray           # int32 [nnz], ascending within a row
    val: np.ndarray           # float64 [nnz]
    beta: np.ndarray          # float64 [n] (inf for HIGH rows)
    status: np.ndarray        # int8 [n]
    cond_ptr: np.ndarray      # int64 [n+1]   conditional rows (selection order)
    cond_nbr: np.ndarray      # int32
    cond_dist: np.ndarray     # int32
    cond_p: np.ndarray        # float64
    graph_offsets: np.ndarray  # int64 [G+1]

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def conditional_rows(indptr, indices, perplexity: float, k: int = 0, seed: int = 0,
                     tie_mode: str = TIE_HASH, rows=None):
    """Selection plus Eq. (3) calibration for every vertex (or ``rows``)."""
    if k <= 0:
        k = k_from_perplexity(perplexity)
    ptr, nbr, dist = select_all(indptr, indices, k, seed, tie_mode, rows)
    r = ptr.shape[0] - 1
    p = np.zeros(nbr.shape[0])
    beta = np.zeros(r)
    status = np.zeros(r, dtype=np.int8)
    for i in range(r):
        a, b = int(ptr[i]), int(ptr[i + 1])
        p[a:b], beta[i], status[i] = row_probabilities(dist[a:b], perplexity)
    return ptr, nbr, dist, p, beta, status


def symmetrize(n: int, cond_ptr, cond_nbr, cond_p, status, graph_offsets):
    """Eq. (2) over the union support, in CSR with sorted columns."""
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(cond_ptr))
    cols = cond_nbr.astype(np.int64)
    r_all = np.concatenate([rows, cols])
    c_all = np.concatenate([cols, rows])
    v_all = np.concatenate([cond_p, cond_p])
    order = np.lexsort((c_all, r_all))
    r_all, c_all, v_all = r_all[order], c_all[order], v_all[order]
    key = r_all * n + c_all
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    starts = np.nonzero(first)[0]
    val = np.add.reduceat(v_all, starts) if starts.shape[0] else np.zeros(0)
    row_u = r_all[starts]
    col_u = c_all[starts]
    # per-graph denominator: twice the number of non-empty rows
    denom = np.zeros(n)
    for g in range(graph_offsets.shape[0] - 1):
        a, b = int(graph_offsets[g]), int(graph_offsets[g + 1])
        nonempty = int(np.sum(status[a:b] != STATUS_EMPTY))
        denom[a:b] = 2.0 * max(nonempty, 1)
    val = val / denom[row_u]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row_u, minlength=n), out=rowptr[1:])
    return rowptr, col_u.astype(np.int32), val


def build_P(indptr, indices, perplexity: float, k: int = 0, seed: int = 0,
            tie_mode: str = TIE_HASH, graph_offsets=None) -> OracleP:
    """C0 of Algorithm 3: partial BFS, Eq. (3) per row, Eq. (2) symmetrisation."""
    indptr = np.asarray(indptr, dtype=np.int64)
    n = indptr.shape[0] - 1
    if graph_offsets is None:
        graph_offsets = np.array([0, n], dtype=np.int64)
    graph_offsets = np.asarray(graph_offsets, dtype=np.int64)
    ptr, nbr, dist, p, beta, status = conditional_rows(indptr, indices, perplexity, k, seed,
                                                       tie_mode)
    rowptr, col, val = symmetrize(n, ptr, nbr, p, status, graph_offsets)
    return OracleP(rowptr, col, val, beta, status, ptr, nbr, dist, p, graph_offsets)
