"""Pivot MDS starting layout (oracle side).

Algorithms 1-3 (Sec. 3) start the iteration from a layout computed by Pivot
MDS, as tsNET* does (Sec. 2.1) and as the experiments use (Sec. 4.1); the
method is the eigensolver of Brandes and Pich (Graph Drawing 2006). The paper
gives no settings; the readings below are this project's, shared with the GPU
path. Per graph g of a
batch (vertices a..b-1, n_g = b - a), in FP64:

1. k_g = min(pivots, n_g) pivots. The first is vertex a + (mix64(seed XOR g)
   mod n_g) (the SplitMix64 finaliser of ``tiebreak``). Each further pivot is
   the vertex whose hop distance to the nearest pivot chosen so far is largest
   (an unreachable vertex counts as infinitely far); ties go to the smallest
   id (max-min selection).
2. Full BFS hop distances d_j(v) from every pivot j. A pair with no path gets
   1 + the largest finite distance among all of the graph's searches.
3. S = d^2 (n_g x k_g), double-centred: C_vj = -1/2 (S_vj - r_v - c_j + m),
   with r, c and m the row, column and grand means of S.
4. e1, e2: unit eigenvectors of C^T C for its two largest eigenvalues
   lambda1 >= lambda2, each signed so that sum_j (j + 1) e_j > 0 over the
   pivot order (a symmetric graph can give an eigenvector two entries of
   equal largest magnitude, so that entry alone cannot fix the sign); if that
   sum is exactly 0, so that its entry of largest magnitude is positive.
5. Y = C [e1 e2], scaled so that the first axis has population standard
   deviation ``scale`` (the spread of the random start, 1e-2); the second
   axis takes the same factor. Y is centred because C is. A graph with fewer
   than two pivots (C is then zero) or with lambda1 = 0 gets zeros.

Library primitives used as steps: scipy's unweighted shortest paths (BFS) and
numpy's symmetric eigensolver.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from .tiebreak import mix64


@dataclass
class PmdsResult:
    X: np.ndarray          # [n, 2] float64 layout
    pivots: list           # per graph: array of pivot ids (global)
    eig: np.ndarray        # [G, 2] lambda1, lambda2 of C^T C (0 where absent)
    dist: list             # per graph: [n_g, k_g] int64 hop distances (unreachable replaced)


def first_pivot(g: int, a: int, n_g: int, seed: int) -> int:
    return a + int(mix64(seed ^ g) % n_g)


def _csr(indptr, indices):
    n = len(indptr) - 1
    data = np.ones(len(indices), dtype=np.float64)
    return sp.csr_matrix((data, np.asarray(indices, np.int64), np.asarray(indptr, np.int64)),
                         shape=(n, n))


def hop_distances(A, src: int, a: int, b: int) -> np.ndarray:
    """BFS hop distances from src to vertices a..b-1, -1 where unreachable."""
    d = shortest_path(A, method="D", unweighted=True, directed=False, indices=[src])[0, a:b]
    out = np.full(b - a, -1, dtype=np.int64)
    fin = np.isfinite(d)
    out[fin] = d[fin].astype(np.int64)
    return out


def select_pivots(A, a: int, b: int, k: int, p0: int):
    """Max-min pivots of graph [a, b): returns pivots and the raw distances [n_g, k]."""
    n_g = b - a
    big = np.iinfo(np.int64).max
    mind = np.full(n_g, big, dtype=np.int64)
    piv, cols = [p0], []
    for j in range(k):
        d = hop_distances(A, piv[j], a, b)
        cols.append(d)
        mind = np.minimum(mind, np.where(d >= 0, d, big))
        if j + 1 < k:
            piv.append(a + int(np.argmax(mind)))   # argmax takes the first (smallest id)
    return np.array(piv, dtype=np.int64), np.stack(cols, axis=1)


def signed(e: np.ndarray) -> np.ndarray:
    t = float(np.dot(np.arange(1, e.shape[0] + 1, dtype=np.float64), e))
    if t == 0.0:
        t = e[int(np.argmax(np.abs(e)))]
    return e if t >= 0 else -e


def double_centre(S: np.ndarray) -> np.ndarray:
    r = S.mean(axis=1, keepdims=True)
    c = S.mean(axis=0, keepdims=True)
    return -0.5 * (S - r - c + S.mean())


def pmds(indptr, indices, pivots: int = 50, seed: int = 0, scale: float = 1e-2,
         graph_offsets=None) -> PmdsResult:
    indptr = np.asarray(indptr, np.int64)
    n = len(indptr) - 1
    off = np.array([0, n], np.int64) if graph_offsets is None else np.asarray(graph_offsets, np.int64)
    A = _csr(indptr, indices)
    X = np.zeros((n, 2))
    eig = np.zeros((len(off) - 1, 2))
    piv_all, dist_all = [], []
    for g in range(len(off) - 1):
        a, b = int(off[g]), int(off[g + 1])
        n_g = b - a
        k = min(pivots, n_g)
        piv, D = select_pivots(A, a, b, k, first_pivot(g, a, n_g, seed))
        if (D < 0).any():
            D = np.where(D < 0, D.max() + 1, D)
        piv_all.append(piv)
        dist_all.append(D)
        C = double_centre(D.astype(np.float64) ** 2)
        w, V = np.linalg.eigh(C.T @ C)            # ascending
        Y = np.zeros((n_g, 2))
        for ax in range(min(2, k) if k >= 2 else 0):
            e = signed(V[:, k - 1 - ax])
            eig[g, ax] = w[k - 1 - ax]
            Y[:, ax] = C @ e
        sd = Y[:, 0].std()
        X[a:b] = Y * (scale / sd) if (k >= 2 and eig[g, 0] > 0 and sd > 0) else 0.0
    return PmdsResult(X, piv_all, eig, dist_all)


def classical_mds(D: np.ndarray, dims: int = 2) -> np.ndarray:
    """Textbook classical MDS of a full distance matrix (for the pins)."""
    B = double_centre(np.asarray(D, np.float64) ** 2)
    w, V = np.linalg.eigh(B)
    return V[:, ::-1][:, :dims] * np.sqrt(np.maximum(w[::-1][:dims], 0.0))
