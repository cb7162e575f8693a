"""Pins for the oracle's tie keys, BFS and partial-BFS selection (CPU only)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from oracle import neighbours, tiebreak
from synth import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    for _, state, out in rows:
        assert tiebreak.mix64(int(state, 16)) == int(out, 16)


def test_mix64_array_matches_scalar():
    rng = np.random.default_rng(7)
    z = rng.integers(0, 2**63, size=200, dtype=np.int64).astype(np.uint64) * np.uint64(3)
    got = tiebreak.mix64_array(z)
    for a, b in zip(z, got):
        assert tiebreak.mix64(int(a)) == int(b)


def test_tie_keys_definition():
    seed = 12345
    for i, j in [(0, 1), (7, 3), (123456, 654321), (2**31 - 1, 5)]:
        want = tiebreak.mix64(seed ^ tiebreak.mix64((i << 32) | j))
        assert int(tiebreak.tie_keys(i, np.array([j]), seed)[0]) == want
    assert list(tiebreak.tie_keys(3, np.array([9, 4]), 0, tiebreak.TIE_ID)) == [9, 4]


def test_bfs_grid_is_manhattan():
    g = graphs.grid(9, 13)
    for src in [0, 5, 58, 116]:
        d = neighbours.bfs_hops(g.indptr, g.indices, src)
        r, c = divmod(np.arange(g.n), 13)
        sr, sc = divmod(src, 13)
        assert np.array_equal(d, np.abs(r - sr) + np.abs(c - sc))


def test_bfs_tree_is_lca_distance():
    n = 300
    g = graphs.random_recursive_tree(n, 11)
    # parent pointers: every v >= 1 has exactly one neighbour with a smaller id
    parent = np.full(n, -1)
    for v in range(1, n):
        nb = g.indices[g.indptr[v]:g.indptr[v + 1]]
        parent[v] = nb[nb < v].max()
    depth = np.zeros(n, dtype=np.int64)
    for v in range(1, n):
        depth[v] = depth[parent[v]] + 1

    def ancestors(v):
        out = [v]
        while v:
            v = parent[v]
            out.append(v)
        return out

    for src in [0, 17, 299]:
        d = neighbours.bfs_hops(g.indptr, g.indices, src)
        anc_s = set(ancestors(src))
        for v in range(0, n, 7):
            lca = next(a for a in ancestors(v) if a in anc_s)
            assert d[v] == depth[src] + depth[v] - 2 * depth[lca]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bfs_matches_scipy(seed):
    g = graphs.sbm([40, 30, 50], 0.08, 0.01, seed)
    A = sp.csr_matrix((np.ones(g.indices.shape[0]), g.indices, g.indptr), shape=(g.n, g.n))
    D = shortest_path(A, unweighted=True, directed=False)
    for src in range(0, g.n, 9):
        d = neighbours.bfs_hops(g.indptr, g.indices, src).astype(float)
        ref = D[src].copy()
        ref[np.isinf(ref)] = -1
        assert np.array_equal(d, ref)


def _brute_select(g, src, k, seed, mode):
    d = neighbours.bfs_hops(g.indptr, g.indices, src)
    cand = np.nonzero(d > 0)[0]
    keys = tiebreak.tie_keys(src, cand, seed, mode)
    trip = sorted(zip(d[cand].tolist(), [int(x) for x in keys], cand.tolist()))
    trip = trip[:k]
    return np.array([t[2] for t in trip], dtype=np.int64), np.array([t[0] for t in trip])


@pytest.mark.parametrize("mode", [tiebreak.TIE_HASH, tiebreak.TIE_ID])
@pytest.mark.parametrize("k", [1, 5, 17, 60])
def test_selection_matches_brute_force(mode, k):
    g = graphs.barabasi_albert(400, 3, 5)
    sel = neighbours.NeighbourSelector(g.indptr, g.indices, k, seed=99, tie_mode=mode)
    for src in range(0, g.n, 13):
        ids, ds = sel.select(src)
        bi, bd = _brute_select(g, src, k, 99, mode)
        assert np.array_equal(ids, bi)
        assert np.array_equal(ds, bd)


def test_selection_small_components_take_everything():
    # two components: a path of 4 and a triangle; k larger than both
    g = graphs.csr_from_edges(7, np.array([0, 1, 2, 4, 5, 6]), np.array([1, 2, 3, 5, 6, 4]))
    sel = neighbours.NeighbourSelector(g.indptr, g.indices, 10)
    ids, ds = sel.select(0)
    assert sorted(ids.tolist()) == [1, 2, 3] and ds.tolist() == [1, 2, 3]
    ids, ds = sel.select(5)
    assert sorted(ids.tolist()) == [4, 6]
    lone = graphs.csr_from_edges(3, np.array([0]), np.array([1]))
    ids, _ = neighbours.NeighbourSelector(lone.indptr, lone.indices, 5).select(2)
    assert ids.shape[0] == 0


def test_grid_hand_cases():
    g = graphs.grid(32, 32)
    sel = neighbours.NeighbourSelector(g.indptr, g.indices, 120, tie_mode=tiebreak.TIE_ID)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "grid32_k120_selection.txt"))
            if l.strip() and not l.startswith("#")]
    for src, counts, last in rows:
        ids, ds = sel.select(int(src))
        want_counts = [int(c) for c in counts.split(",")]
        got_counts = np.bincount(ds)[1:].tolist()
        assert got_counts == want_counts
        if last != "-":
            assert sorted(ids[ds == ds.max()].tolist()) == [int(x) for x in last.split(",")]


def test_k_from_perplexity():
    assert neighbours.k_from_perplexity(40) == 120
    assert neighbours.k_from_perplexity(33.4) == 100
    with pytest.raises(ValueError):
        neighbours.k_from_perplexity(0)
