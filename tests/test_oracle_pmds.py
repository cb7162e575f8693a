"""Pins of the oracle's Pivot MDS starting layout (no GPU).

Each check ties oracle.pmds to something other than itself:
* max-min pivots against a brute-force search over all-pairs BFS distances
  (the oracle's own pure-Python BFS, not scipy);
* the first pivot against a published SplitMix64 output;
* a path graph, whose squared distances double-centre to a rank-one matrix:
  the layout is exactly linear in the position along the path, the second
  axis is zero and lambda2 = 0;
* with every vertex a pivot, Pivot MDS spans the same two axes as textbook
  classical MDS (each axis equal up to its scale);
* a rectangular grid: the first axis follows the long side;
* a batch gives every graph the layout it gets alone; disconnected pieces and
  tiny graphs follow the stated conventions.
"""
import numpy as np
import pytest

from oracle import neighbours, pmds
from oracle.tiebreak import mix64
from synth import graphs

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _all_pairs(g):
    return np.stack([neighbours.bfs_hops(g.indptr, g.indices, s) for s in range(g.n)])


def _brute_maxmin(D, p0, k):
    piv = [p0]
    for _ in range(k - 1):
        mind = np.where(D[piv] >= 0, D[piv], np.iinfo(np.int64).max).min(axis=0)
        best = mind.max()
        piv.append(int(np.nonzero(mind == best)[0][0]))
    return piv


@pytest.mark.parametrize("maker", [lambda: graphs.grid(7, 5), lambda: graphs.random_recursive_tree(60, 3),
                                   lambda: graphs.sbm([30, 30], 0.2, 0.02, 5)])
def test_maxmin_pivots_brute_force(maker):
    g = maker()
    D = _all_pairs(g)
    r = pmds.pmds(g.indptr, g.indices, pivots=8, seed=11)
    p0 = pmds.first_pivot(0, 0, g.n, 11)
    assert list(r.pivots[0]) == _brute_maxmin(D, p0, 8)
    # distances of every pivot are the BFS distances (no unreachable pairs here)
    assert np.array_equal(r.dist[0], D[r.pivots[0]].T)


def test_first_pivot_golden():
    # the first output of SplitMix64 seeded with 0 is the finaliser of its increment,
    # 0xE220A8397B1DCDAF (published reference value)
    assert mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert pmds.first_pivot(0, 100, 1000, 0x9E3779B97F4A7C15) == 100 + 0xE220A8397B1DCDAF % 1000


def test_path_is_linear():
    n = 41
    g = graphs.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    r = pmds.pmds(g.indptr, g.indices, pivots=6, seed=2, scale=0.5)
    pos = np.arange(n) - (n - 1) / 2
    x = r.X[:, 0]
    assert abs(abs(np.corrcoef(x, pos)[0, 1]) - 1.0) < 1e-12
    assert np.abs(r.X[:, 1]).max() < 1e-9 * np.abs(x).max()
    assert r.eig[0, 1] <= 1e-9 * r.eig[0, 0]
    assert abs(x.std() - 0.5) < 1e-12 and abs(x.mean()) < 1e-12
    # the end pivots: the first pivot's farthest vertex is an end of the path
    p0 = int(r.pivots[0][0])
    assert int(r.pivots[0][1]) == (0 if p0 >= n - 1 - p0 else n - 1)


def test_all_pivots_is_classical_mds():
    g = graphs.grid(9, 5)
    D = _all_pairs(g)
    r = pmds.pmds(g.indptr, g.indices, pivots=g.n, seed=4)
    # with every vertex a pivot, columns are a permutation of the vertices
    perm = np.asarray(r.pivots[0])
    assert sorted(perm.tolist()) == list(range(g.n))
    ref = pmds.classical_mds(D)
    for ax in range(2):
        c = np.corrcoef(r.X[:, ax], ref[:, ax])[0, 1]
        assert abs(abs(c) - 1.0) < 1e-9, (ax, c)


def test_rectangular_grid_long_axis():
    g = graphs.grid(10, 30)        # 10 rows, 30 columns: the long side is the column index
    r = pmds.pmds(g.indptr, g.indices, pivots=20, seed=1)
    col = np.arange(g.n) % 30
    row = np.arange(g.n) // 30
    assert abs(np.corrcoef(r.X[:, 0], col)[0, 1]) > 0.99
    assert abs(np.corrcoef(r.X[:, 1], row)[0, 1]) > 0.95
    assert r.eig[0, 0] > r.eig[0, 1] > 0


def test_batch_equals_single_and_conventions():
    parts = [graphs.grid(6, 4), graphs.random_recursive_tree(30, 7),
             graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)),
             graphs.csr_from_edges(5, np.array([0, 1, 3]), np.array([1, 2, 4]))]  # 2 pieces
    b = graphs.concat_graphs(parts)
    r = pmds.pmds(b.indptr, b.indices, pivots=5, seed=9, graph_offsets=b.graph_offsets)
    off = b.graph_offsets
    for gi, g in enumerate(parts):
        # alone, graph gi is graph 0: seed 9 ^ gi gives it the same first pivot
        alone = pmds.pmds(g.indptr, g.indices, pivots=5, seed=9 ^ gi)
        assert np.array_equal(r.pivots[gi] - off[gi], alone.pivots[0])
        assert np.allclose(r.X[off[gi]:off[gi + 1]], alone.X, rtol=0, atol=1e-15)
    # one-vertex graph: zeros
    assert np.all(r.X[off[2]:off[3]] == 0)
    # two pieces: the unreachable pairs take 1 + the largest finite distance (2 here)
    D = r.dist[3]
    assert D.max() == 3 and (D == 3).any()
    # the first pivot follows the hash of (seed XOR graph index)
    for gi in range(len(parts)):
        n_g = int(off[gi + 1] - off[gi])
        assert int(r.pivots[gi][0]) == int(off[gi]) + int(mix64(9 ^ gi) % n_g)
