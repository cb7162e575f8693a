"""Seeded synthetic graphs and initial layouts.

This module only produces inputs. It holds none of the layout method's
arithmetic, so both the FP64 oracle and the GPU path may use it.

Every generator returns an undirected simple graph in CSR form:
``indptr`` int64 [n+1] and ``indices`` int32 [2m], each row sorted ascending,
no duplicates and no self loops.

The graph families stand in for the shapes of the paper's benchmark suites
(Sec. 4.1 and the data-set table in the appendix): grids and random
geometric graphs for meshes, stochastic block models for clustered networks,
Barabasi-Albert graphs for heavy-tailed scale-free networks and random
recursive trees for very sparse graphs. None of those data sets is reproduced.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSRGraph:
    indptr: np.ndarray   # int64 [n+1]
    indices: np.ndarray  # int32 [2m]

    @property
    def n(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.indices.shape[0] // 2)

    def degrees(self) -> np.ndarray:
        return np.diff(self.indptr)


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray) -> CSRGraph:
    """Undirected simple CSR from an edge list (self loops and repeats dropped)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * np.int64(n) + dst)
    src = key // n
    dst = key % n
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=indptr[1:])
    return CSRGraph(indptr, dst.astype(np.int32))


def _bernoulli_positions(rng: np.random.Generator, total: int, p: float) -> np.ndarray:
    """Sorted positions in [0, total), each present independently with prob. p.

    Geometric skip sampling: the gaps between successive hits are geometric.
    """
    if total <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(total, dtype=np.int64)
    out = []
    pos = -1
    while True:
        batch = max(1024, int(total * p * 1.1) + 64)
        gaps = rng.geometric(p, size=batch).astype(np.int64)
        cand = pos + np.cumsum(gaps)
        hit = cand[cand < total]
        out.append(hit)
        if hit.shape[0] < cand.shape[0]:
            break
        pos = int(cand[-1])
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def grid(rows: int, cols: int) -> CSRGraph:
    """rows x cols 4-neighbour grid; vertex id = r*cols + c."""
    n = rows * cols
    ids = np.arange(n, dtype=np.int64).reshape(rows, cols)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return csr_from_edges(n, u, v)


def grid_prefix(n: int) -> CSRGraph:
    """First n vertices (row-major) of an r x ceil(n/r) grid with r = floor(sqrt(n))."""
    r = max(1, int(np.floor(np.sqrt(n))))
    c = -(-n // r)
    ids = np.arange(r * c, dtype=np.int64).reshape(r, c)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    keep = (u < n) & (v < n)
    return csr_from_edges(n, u[keep], v[keep])


def sbm(block_sizes, p_in: float, p_out: float, seed: int) -> CSRGraph:
    """Stochastic block model over consecutive id blocks (geometric-skip sampling)."""
    rng = np.random.default_rng(seed)
    sizes = [int(s) for s in block_sizes]
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(starts[-1])
    us, vs = [], []
    for a in range(len(sizes)):
        for b in range(a, len(sizes)):
            sa, sb = sizes[a], sizes[b]
            p = p_in if a == b else p_out
            pos = _bernoulli_positions(rng, sa * sb, p)
            i = pos // sb
            j = pos % sb
            if a == b:
                keep = i < j          # each unordered pair considered once
                i, j = i[keep], j[keep]
            us.append(starts[a] + i)
            vs.append(starts[b] + j)
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return csr_from_edges(n, u, v)


def rgg(n: int, radius: float, seed: int) -> CSRGraph:
    """Random geometric graph: n uniform points in [0,1)^2, edge iff distance <= radius."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    return csr_from_edges(n, pairs[:, 0], pairs[:, 1])


def rgg_radius_for_degree(n: int, mean_degree: float) -> float:
    """Radius giving the requested mean degree without boundary correction."""
    return float(np.sqrt(mean_degree / (np.pi * (n - 1))))


def barabasi_albert(n: int, m0: int, seed: int) -> CSRGraph:
    """Preferential attachment: a K_{m0+1} seed, then each new vertex joins m0
    distinct earlier vertices drawn from the endpoint list (probability
    proportional to degree); repeated targets of one vertex are redrawn.

    The draws are resolved in vectorised form: a uniform position in the
    endpoint list either names a new vertex directly (even slot of a later
    edge) or points at the target of an earlier edge (odd slot), which is
    followed until it reaches a known vertex.
    """
    rng = np.random.default_rng(seed)
    s = m0 + 1
    if n <= s:
        iu, ju = np.triu_indices(n, 1)
        return csr_from_edges(n, iu, ju)
    iu, ju = np.triu_indices(s, 1)
    e0 = iu.shape[0]
    seed_ends = np.empty(2 * e0, dtype=np.int64)
    seed_ends[0::2] = iu
    seed_ends[1::2] = ju
    nv = n - s
    ne = nv * m0
    new_vertex = s + np.arange(ne, dtype=np.int64) // m0        # source of edge e0+t
    list_len = 2 * (e0 + (new_vertex - s) * m0)                  # list length seen by that vertex
    pos = (rng.random(ne) * list_len).astype(np.int64)

    def resolve(pos):
        tgt = np.full(ne, -1, dtype=np.int64)
        is_seed = pos < 2 * e0
        tgt[is_seed] = seed_ends[pos[is_seed]]
        later = ~is_seed
        edge = (pos - 2 * e0) // 2
        even = later & ((pos % 2) == 0)
        tgt[even] = new_vertex[edge[even]]
        ref = np.where(later & ~even, edge, -1)
        pending = np.nonzero(ref >= 0)[0]
        while pending.shape[0]:
            r = ref[pending]
            done = tgt[r] >= 0
            tgt[pending[done]] = tgt[r[done]]
            pending = pending[~done]
        return tgt

    while True:
        tgt = resolve(pos)
        t2 = tgt.reshape(nv, m0)
        srt = np.sort(t2, axis=1)
        dup_rows = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
        if dup_rows.shape[0] == 0:
            break
        # within each offending vertex redraw every repeat after the first
        redo = []
        for r in dup_rows:
            seen = set()
            for c in range(m0):
                t = int(t2[r, c])
                if t in seen:
                    redo.append(r * m0 + c)
                seen.add(t)
        redo = np.asarray(redo, dtype=np.int64)
        pos[redo] = (rng.random(redo.shape[0]) * list_len[redo]).astype(np.int64)
    u = np.concatenate([iu.astype(np.int64), new_vertex])
    v = np.concatenate([ju.astype(np.int64), tgt])
    return csr_from_edges(n, u, v)


def random_recursive_tree(n: int, seed: int) -> CSRGraph:
    """Vertex v >= 1 attaches to a uniform earlier vertex."""
    rng = np.random.default_rng(seed)
    if n <= 1:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    v = np.arange(1, n, dtype=np.int64)
    parent = (rng.random(n - 1) * v).astype(np.int64)
    return csr_from_edges(n, v, parent)


@dataclass
class GraphBatch:
    graphs: list            # list[CSRGraph], each with local ids
    kinds: list             # list[str]
    indptr: np.ndarray      # int64 [N+1], concatenated with global ids
    indices: np.ndarray     # int32
    graph_offsets: np.ndarray  # int32 [G+1] vertex offsets

    @property
    def num_graphs(self) -> int:
        return len(self.graphs)


def concat_graphs(graphs, kinds=None) -> GraphBatch:
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([g.n for g in graphs])
    eoffs = np.zeros(len(graphs) + 1, dtype=np.int64)
    eoffs[1:] = np.cumsum([g.indices.shape[0] for g in graphs])
    indptr = np.zeros(int(offs[-1]) + 1, dtype=np.int64)
    indices = np.zeros(int(eoffs[-1]), dtype=np.int32)
    for gi, g in enumerate(graphs):
        a, b = int(offs[gi]), int(offs[gi + 1])
        indptr[a + 1:b + 1] = g.indptr[1:] + eoffs[gi]
        indices[eoffs[gi]:eoffs[gi + 1]] = g.indices + np.int32(a)
    if int(offs[-1]) >= 2**31:
        raise ValueError("batch too large for int32 vertex ids")
    return GraphBatch(list(graphs), list(kinds or ["?"] * len(graphs)), indptr, indices,
                      offs.astype(np.int32))


def mixed_batch(num_graphs: int, seed: int, n_min: int = 500, n_max: int = 50000) -> GraphBatch:
    """Independent SBM / grid / random-recursive-tree graphs with n ~ U{n_min..n_max}."""
    rng = np.random.default_rng(seed)
    graphs, kinds = [], []
    for gi in range(num_graphs):
        kind = ("sbm", "grid", "tree")[int(rng.integers(0, 3))]
        n = int(rng.integers(n_min, n_max + 1))
        sub = int(rng.integers(0, 2**31 - 1))
        if kind == "sbm":
            sizes = [1000] * (n // 1000) + ([n % 1000] if n % 1000 else [])
            g = sbm(sizes, 0.01, 1.0 / n, sub)
        elif kind == "grid":
            g = grid_prefix(n)
        else:
            g = random_recursive_tree(n, sub)
        graphs.append(g)
        kinds.append(kind)
    return concat_graphs(graphs, kinds)


def initial_layout(n: int, seed: int, std: float = 0.01) -> np.ndarray:
    """N(0, std^2 I) positions, returned as float32 [n, 2] (variance 1e-4 by default)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=(n, 2)).astype(np.float32)


def uniform_square(n: int, side: float, seed: int) -> np.ndarray:
    """n positions uniform in the square [-side/2, side/2]^2 (a spread-out
    layout with no far points: its interpolation grid covers the whole box).
    float32 [n, 2]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5 * side, 0.5 * side, size=(n, 2)).astype(np.float32)


def bulk_with_far_points(n: int, seed: int, n_far: int = 100, std: float = 0.18,
                         r_min: float = 1.0, r_max: float = 60.0) -> np.ndarray:
    """A dense bulk N(0, std^2 I) with ``n_far`` of its points moved far out: at
    radii log-uniform in [r_min, r_max] and uniform directions. The shape of
    the layouts a descent from a small random start passes through at
    n = 1e6 (a bulk about a unit wide, a few dozen to a hundred points out to
    tens of units setting the bounding box). float32 [n, 2]."""
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, std, size=(n, 2))
    idx = rng.choice(n, size=min(n_far, n), replace=False)
    r = np.exp(rng.uniform(np.log(r_min), np.log(r_max), size=idx.shape[0]))
    a = rng.uniform(0.0, 2.0 * np.pi, size=idx.shape[0])
    X[idx, 0] = r * np.cos(a)
    X[idx, 1] = r * np.sin(a)
    return X.astype(np.float32)


def random_affinity(n: int, mean_len: float, seed: int, hub_rows: int = 0, hub_len: int = 0,
                    empty_frac: float = 0.0):
    """A seeded sparse nonnegative n x n matrix in CSR form for layout-independent
    tests of the sparse sums: row lengths Poisson(mean_len) (the first
    ``hub_rows`` rows get ``hub_len`` entries, a fraction ``empty_frac`` of the
    rest none), columns uniform without the diagonal, sorted and distinct,
    values uniform in (0.1, 1] scaled to sum 1. Returns (rowptr int64,
    col int32, val float64)."""
    rng = np.random.default_rng(seed)
    lens = rng.poisson(mean_len, size=n).astype(np.int64)
    lens[:hub_rows] = hub_len
    if empty_frac > 0:
        lens[hub_rows:][rng.random(n - hub_rows) < empty_frac] = 0
    lens = np.minimum(lens, n - 1)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    col = rng.integers(0, n - 1, size=rows.shape[0], dtype=np.int64)
    col += col >= rows                                  # skip the diagonal
    key = np.unique(rows * n + col)                     # sorted, distinct per row
    rows, col = key // n, key % n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    val = rng.uniform(0.1, 1.0, size=col.shape[0])
    val /= val.sum() if val.size else 1.0
    return rowptr, col.astype(np.int32), val


# Named workloads (shapes of the paper's graph families, sizes from the
# benchmark configurations).

def workload_grid32():
    """2-D grid 32x32: n=1024, m=1984, unweighted."""
    return grid(32, 32)


def workload_sbm20k():
    """SBM, 20 blocks of 1000, p_in=0.01, p_out=5e-5, seed 1."""
    return sbm([1000] * 20, 0.01, 5e-5, 1)


def workload_rgg100k():
    """Random geometric graph n=1e5 in the unit square, mean degree 8, seed 2."""
    n = 100_000
    return rgg(n, rgg_radius_for_degree(n, 8.0), 2)


def workload_ba1m(n: int = 1_000_000):
    """Barabasi-Albert n=1e6, m0=4, seed 3."""
    return barabasi_albert(n, 4, 3)


def workload_mixed256():
    """256 independent SBM/grid/tree graphs, n ~ U{500..50000}, seed 4."""
    return mixed_batch(256, 4)
