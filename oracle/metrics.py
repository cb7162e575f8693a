"""Layout quality metrics: neighbourhood preservation and stress (oracle side).

Sec. 4.3 judges drawings by neighbourhood preservation (Sec. 4.3.1, r = 2) and
by stress (Sec. 4.3.2). The paper states the two formulas; the readings below
are this project's, shared with the GPU path.

Neighbourhood preservation of vertex v (r = 2):
* N_G(v) = the vertices at hop distance 1 or 2 from v (v itself excluded);
  k_v = |N_G(v)|.
* N_D(v) = the k_v vertices of v's own graph closest to v in the layout,
  v excluded. Closeness is the squared distance computed in FP32 from the
  FP32 coordinates as dx*dx + dy*dy with dx = x_w - x_v, dy = y_w - y_v, each
  operation rounded on its own (no fused multiply-add); equal distances are
  taken in increasing vertex id.
* hits_v = |N_G(v) & N_D(v)|; since both sets have k_v members, the Jaccard
  ratio of the two sets is hits_v / (2 k_v - hits_v).
* NP of a graph is the mean of that ratio over the evaluated vertices of the
  graph (all of them, or a sample the caller names); a vertex with k_v = 0
  has two empty sets and is left out of the mean. A graph with no vertex
  left has NP = NaN.

Stress over the ordered pairs (s, j), s a source vertex, j != s reachable
from s in the same graph, d = hop distance, e = Euclidean layout distance in
FP64 from the FP32 coordinates:
* pairs = the number of such pairs; S1 = sum (1 - e/d)^2 (the paper's term
  ((d - e)/d)^2); B = sum e/d; C = sum (e/d)^2.
* raw stress = S1 / pairs. With every vertex a source and a connected graph,
  pairs = n(n-1) and this is the paper's normalised sum exactly. Pairs with
  no path are left out (the formula needs a finite d).
* The sums also give the stress of the layout scaled by the factor that
  minimises it, alpha = B / C: (pairs - B^2 / C) / pairs.

Library primitives used as steps: numpy's stable lexicographic sort and
scipy's unweighted shortest paths (BFS).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path


def _offsets(n: int, graph_offsets):
    if graph_offsets is None:
        return np.array([0, n], dtype=np.int64)
    return np.asarray(graph_offsets, dtype=np.int64)


def _graph_of(off: np.ndarray, v: int) -> int:
    return int(np.searchsorted(off, v, side="right") - 1)


def ball2(indptr, indices, v: int) -> np.ndarray:
    """N_G(v, 2): sorted ids at hop distance 1 or 2 from v, v excluded."""
    nb = indices[indptr[v]:indptr[v + 1]]
    parts = [nb] + [indices[indptr[a]:indptr[a + 1]] for a in nb]
    allv = np.unique(np.concatenate(parts)) if len(nb) else np.zeros(0, np.int64)
    return allv[allv != v].astype(np.int64)


def layout_d2(X32: np.ndarray, v: int, ids: np.ndarray) -> np.ndarray:
    """FP32 squared layout distances from v to ids, one rounding per operation."""
    dx = X32[ids, 0] - X32[v, 0]
    dy = X32[ids, 1] - X32[v, 1]
    return dx * dx + dy * dy


def nearest(X32: np.ndarray, v: int, k: int, a: int, b: int) -> np.ndarray:
    """The k vertices of [a, b) other than v closest to v, by (distance, id)."""
    ids = np.arange(a, b, dtype=np.int64)
    ids = ids[ids != v]
    d2 = layout_d2(X32, v, ids)
    order = np.lexsort((ids, d2))      # primary key d2, then id
    return ids[order[:k]]


def np_vertex(indptr, indices, X32: np.ndarray, v: int, a: int, b: int):
    """(k_v, hits_v) of vertex v of the graph [a, b)."""
    B = ball2(indptr, indices, v)
    k = len(B)
    if k == 0:
        return 0, 0
    D = nearest(X32, v, k, a, b)
    return k, int(np.intersect1d(B, D, assume_unique=True).size)


def neighbourhood_preservation(indptr, indices, X, vertices=None, graph_offsets=None):
    """Per evaluated vertex k_v and hits_v, and NP per graph (Sec. 4.3.1)."""
    indptr = np.asarray(indptr, np.int64)
    indices = np.asarray(indices, np.int64)
    n = len(indptr) - 1
    off = _offsets(n, graph_offsets)
    X32 = np.asarray(X, dtype=np.float32).reshape(n, 2)
    verts = np.arange(n, dtype=np.int64) if vertices is None else np.asarray(vertices, np.int64)
    ball = np.zeros(len(verts), np.int64)
    hits = np.zeros(len(verts), np.int64)
    G = len(off) - 1
    total = np.zeros(G)
    count = np.zeros(G, np.int64)
    for i, v in enumerate(verts):
        g = _graph_of(off, int(v))
        k, h = np_vertex(indptr, indices, X32, int(v), int(off[g]), int(off[g + 1]))
        ball[i], hits[i] = k, h
        if k > 0:
            total[g] += h / (2 * k - h)
            count[g] += 1
    with np.errstate(invalid="ignore", divide="ignore"):
        per_graph = np.where(count > 0, total / np.maximum(count, 1), np.nan)
    return ball, hits, per_graph


def stress_sums(indptr, indices, X, sources, graph_offsets=None) -> np.ndarray:
    """[G, 4] sums (pairs, S1, B, C) over the pairs (s, j) of each source s."""
    indptr = np.asarray(indptr, np.int64)
    n = len(indptr) - 1
    off = _offsets(n, graph_offsets)
    X64 = np.asarray(X, dtype=np.float32).reshape(n, 2).astype(np.float64)
    A = sp.csr_matrix((np.ones(len(indices)), np.asarray(indices, np.int64), indptr), shape=(n, n))
    out = np.zeros((len(off) - 1, 4))
    for s in np.asarray(sources, np.int64):
        g = _graph_of(off, int(s))
        a, b = int(off[g]), int(off[g + 1])
        d = shortest_path(A, method="D", unweighted=True, directed=False, indices=[int(s)])[0, a:b]
        j = np.nonzero(np.isfinite(d) & (d > 0))[0]
        dist = d[j]
        dx = X64[a + j, 0] - X64[s, 0]
        dy = X64[a + j, 1] - X64[s, 1]
        ratio = np.sqrt(dx * dx + dy * dy) / dist
        out[g] += [len(j), np.sum((1.0 - ratio) ** 2), np.sum(ratio), np.sum(ratio * ratio)]
    return out


def stress_values(sums: np.ndarray):
    """(raw stress, stress at the best uniform scale) per graph from the sums."""
    sums = np.atleast_2d(sums)
    pairs, S1, B, C = sums[:, 0], sums[:, 1], sums[:, 2], sums[:, 3]
    with np.errstate(invalid="ignore", divide="ignore"):
        raw = np.where(pairs > 0, S1 / pairs, np.nan)
        best = np.where((pairs > 0) & (C > 0), (pairs - B * B / np.where(C > 0, C, 1)) / pairs, raw)
    return raw, best
