"""Partial-BFS k-nearest neighbours of every vertex (oracle side).

Sec. 3.1 and the C0 block of Algorithm 3: from each vertex v a BFS runs until
k other vertices have been visited, where k = 3u for perplexity u; vertices
at equal hop distance are taken in random order. The visited set is the
k-nearest-neighbour set N_k(v) in hop distance.

Written out: BFS levels are expanded one at a time; once the levels seen so
far hold at least k vertices besides v, the last level is cut by the tie key
(``tiebreak``). If the component of v holds fewer than k other vertices, all
of them are taken. The result is sorted by (hop distance, tie key, id).
"""
from __future__ import annotations

import numpy as np

from .tiebreak import TIE_HASH, tie_keys


def k_from_perplexity(perplexity: float) -> int:
    """k = 3u (Sec. 3.1); a fractional 3u is rounded down."""
    if not perplexity > 0:
        raise ValueError("perplexity must be positive")
    return int(np.floor(3.0 * perplexity + 1e-9))


def bfs_hops(indptr: np.ndarray, indices: np.ndarray, src: int) -> np.ndarray:
    """Full single-source BFS: hop distance to every vertex, -1 if unreachable."""
    n = indptr.shape[0] - 1
    dist = np.full(n, -1, dtype=np.int64)
    dist[src] = 0
    frontier = [src]
    level = 0
    while frontier:
        level += 1
        nxt = []
        for f in frontier:
            for j in indices[indptr[f]:indptr[f + 1]]:
                if dist[j] < 0:
                    dist[j] = level
                    nxt.append(int(j))
        frontier = nxt
    return dist


def _expand(indptr, indices, frontier: np.ndarray) -> np.ndarray:
    """All neighbours (with repeats) of the vertices in ``frontier``."""
    starts = indptr[frontier]
    lens = indptr[frontier + 1] - starts
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    base = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return indices[base + np.arange(total)].astype(np.int64)


class NeighbourSelector:
    """Runs the partial BFS from many sources over one graph.

    A distance array of length n is reused between sources and reset through
    the list of touched vertices, so one source costs only what it visits.
    """

    def __init__(self, indptr, indices, k: int, seed: int = 0, tie_mode: str = TIE_HASH):
        self.indptr = np.asarray(indptr, dtype=np.int64)
        self.indices = np.asarray(indices, dtype=np.int64)
        self.k = int(k)
        self.seed = int(seed)
        self.tie_mode = tie_mode
        self._dist = np.full(self.indptr.shape[0] - 1, -1, dtype=np.int64)

    def select(self, src: int):
        """Return (neighbour ids int64, hop distances int64) sorted by (d, key, id)."""
        dist = self._dist
        touched = [np.array([src], dtype=np.int64)]
        dist[src] = 0
        frontier = np.array([src], dtype=np.int64)
        chosen_ids, chosen_d = [], []
        have = 0
        level = 0
        while frontier.shape[0] and have < self.k:
            level += 1
            cand = np.unique(_expand(self.indptr, self.indices, frontier))
            cand = cand[dist[cand] < 0]
            dist[cand] = level
            touched.append(cand)
            if cand.shape[0] == 0:
                break
            keys = tie_keys(src, cand, self.seed, self.tie_mode)
            order = np.lexsort((cand, keys))       # by key, then id
            take = cand[order][: self.k - have]
            chosen_ids.append(take)
            chosen_d.append(np.full(take.shape[0], level, dtype=np.int64))
            have += take.shape[0]
            frontier = cand
        for t in touched:
            dist[t] = -1
        if not chosen_ids:
            return np.zeros(0, np.int64), np.zeros(0, np.int64)
        return np.concatenate(chosen_ids), np.concatenate(chosen_d)


def select_all(indptr, indices, k: int, seed: int = 0, tie_mode: str = TIE_HASH, rows=None):
    """Partial-BFS selection for every vertex (or for ``rows``).

    Returns (row_ptr int64 [r+1], nbr int32, dist int32) as a ragged list.
    """
    sel = NeighbourSelector(indptr, indices, k, seed, tie_mode)
    n = indptr.shape[0] - 1
    rows = np.arange(n) if rows is None else np.asarray(rows)
    ids, ds = [], []
    ptr = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    for r, i in enumerate(rows):
        a, d = sel.select(int(i))
        ids.append(a)
        ds.append(d)
        ptr[r + 1] = ptr[r] + a.shape[0]
    nbr = np.concatenate(ids).astype(np.int32) if ids else np.zeros(0, np.int32)
    dist = np.concatenate(ds).astype(np.int32) if ds else np.zeros(0, np.int32)
    return ptr, nbr, dist
