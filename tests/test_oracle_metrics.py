"""Pins of the oracle's layout quality metrics (no GPU).

Neighbourhood preservation (r = 2) is tied to:
* graphs whose 2-hop balls are everything (complete graph, star): NP = 1 for
  any layout, since N_D then has to be every other vertex;
* a path drawn on a line with unit spacing and the interior of a grid drawn
  on the integer lattice: the nearest points are exactly the 2-hop ball;
* coincident points (all distances equal): N_D is the k smallest other ids;
* a random layout (no ties): the ball from all-pairs BFS of the oracle's own
  search (not scipy) and the nearest points from scipy's k-d tree;
* a batch: every graph's vertices are ranked only among their own graph.

Stress is tied to:
* a path on a line: zero at unit spacing, (1 - alpha)^2 per pair at spacing
  alpha, zero again after the best rescaling;
* the unit square drawing of the 4-cycle (closed form);
* a disconnected graph: only the n_c (n_c - 1) pairs inside components count;
* additivity over source sets.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import metrics, neighbours
from synth import graphs


def _path(n):
    return graphs.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))


def _complete(n):
    u, v = np.triu_indices(n, 1)
    return graphs.csr_from_edges(n, u, v)


def test_np_complete_and_star_are_one():
    rng = np.random.default_rng(0)
    for g in (_complete(12), graphs.csr_from_edges(30, np.zeros(29, np.int64), np.arange(1, 30))):
        X = rng.normal(size=(g.n, 2)).astype(np.float32)
        ball, hits, npg = metrics.neighbourhood_preservation(g.indptr, g.indices, X)
        assert np.all(ball == g.n - 1) and np.all(hits == ball)
        assert npg[0] == 1.0


def test_np_path_on_a_line():
    n = 50
    g = _path(n)
    X = np.stack([np.arange(n, dtype=np.float32), np.zeros(n, np.float32)], axis=1)
    ball, hits, npg = metrics.neighbourhood_preservation(g.indptr, g.indices, X)
    expect = np.minimum(np.arange(n), 2) + np.minimum(n - 1 - np.arange(n), 2)
    assert np.array_equal(ball, expect)
    # ties at the ends: vertex 1 has ball {0, 2, 3}; its 3 nearest are 0, 2 (distance 1) and 3
    assert np.array_equal(hits, ball) and npg[0] == 1.0


def test_np_grid_interior_on_lattice():
    rows, cols = 11, 13
    g = graphs.grid(rows, cols)
    r, c = np.divmod(np.arange(g.n), cols)
    X = np.stack([c, r], axis=1).astype(np.float32)
    inner = [v for v in range(g.n) if 2 <= r[v] < rows - 2 and 2 <= c[v] < cols - 2]
    ball, hits, _ = metrics.neighbourhood_preservation(g.indptr, g.indices, X, vertices=inner)
    # 4 at distance 1, 4 diagonal at sqrt(2), 4 straight at 2: the 12 closest points exactly
    assert np.all(ball == 12) and np.all(hits == 12)


def test_np_coincident_points_take_smallest_ids():
    g = graphs.random_recursive_tree(40, 5)
    X = np.zeros((g.n, 2), np.float32)
    ball, hits, _ = metrics.neighbourhood_preservation(g.indptr, g.indices, X)
    for v in range(g.n):
        B = set(np.nonzero((neighbours.bfs_hops(g.indptr, g.indices, v) >= 1)
                           & (neighbours.bfs_hops(g.indptr, g.indices, v) <= 2))[0].tolist())
        D = [w for w in range(g.n) if w != v][:len(B)]
        assert ball[v] == len(B) and hits[v] == len(B & set(D))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_np_random_layout_against_kdtree(seed):
    g = graphs.sbm([40, 40, 40], 0.15, 0.01, seed)
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(g.n, 2)).astype(np.float32)
    ball, hits, npg = metrics.neighbourhood_preservation(g.indptr, g.indices, X)
    tree = cKDTree(X.astype(np.float64))
    ratios, checked = [], 0
    for v in range(g.n):
        d = neighbours.bfs_hops(g.indptr, g.indices, v)
        B = set(np.nonzero((d == 1) | (d == 2))[0].tolist())
        k = len(B)
        assert ball[v] == k
        if k == 0:
            continue
        ratios.append(hits[v] / (2 * k - hits[v]))
        dist, idx = tree.query(X[v].astype(np.float64), k=k + 2)
        # only where no near tie sits at the k-th place (there float32 and float64 agree)
        if dist[k + 1] - dist[k] <= 1e-6 * dist[k + 1]:
            continue
        D = set(int(i) for i in idx[:k + 1] if i != v)
        assert len(D) == k and hits[v] == len(B & D)
        checked += 1
    assert checked >= 0.9 * g.n
    assert npg[0] == pytest.approx(np.mean(ratios), rel=1e-15)


def test_np_batch_ranks_within_graph():
    parts = [graphs.grid(5, 6), graphs.random_recursive_tree(25, 2), graphs.sbm([15, 15], 0.3, 0.05, 7)]
    b = graphs.concat_graphs(parts)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(int(b.graph_offsets[-1]), 2)).astype(np.float32)
    ball, hits, npg = metrics.neighbourhood_preservation(b.indptr, b.indices, X,
                                                         graph_offsets=b.graph_offsets)
    off = b.graph_offsets
    for gi, g in enumerate(parts):
        bl, hl, ng = metrics.neighbourhood_preservation(g.indptr, g.indices, X[off[gi]:off[gi + 1]])
        assert np.array_equal(ball[off[gi]:off[gi + 1]], bl)
        assert np.array_equal(hits[off[gi]:off[gi + 1]], hl)
        assert npg[gi] == ng[0]


def test_np_isolated_vertices_left_out():
    g = graphs.csr_from_edges(4, np.array([0]), np.array([1]))   # 2 and 3 isolated
    X = np.arange(8, dtype=np.float32).reshape(4, 2)
    ball, hits, npg = metrics.neighbourhood_preservation(g.indptr, g.indices, X)
    assert list(ball) == [1, 1, 0, 0] and list(hits) == [1, 1, 0, 0] and npg[0] == 1.0
    _, _, none = metrics.neighbourhood_preservation(g.indptr, g.indices, X, vertices=[2, 3])
    assert np.isnan(none[0])


def test_stress_path_line_and_scale():
    n = 30
    g = _path(n)
    for alpha in (1.0, 0.5, 2.0):
        X = np.stack([alpha * np.arange(n), np.zeros(n)], axis=1).astype(np.float32)
        s = metrics.stress_sums(g.indptr, g.indices, X, np.arange(n))
        assert s[0, 0] == n * (n - 1)
        assert s[0, 1] == pytest.approx(n * (n - 1) * (1 - alpha) ** 2, abs=1e-12)
        raw, best = metrics.stress_values(s)
        assert raw[0] == pytest.approx((1 - alpha) ** 2, abs=1e-14)
        assert abs(best[0]) < 1e-12


def test_stress_square_cycle_closed_form():
    g = graphs.csr_from_edges(4, np.array([0, 1, 2, 3]), np.array([1, 2, 3, 0]))
    X = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    s = metrics.stress_sums(g.indptr, g.indices, X, np.arange(4))
    raw, _ = metrics.stress_values(s)
    # 8 ordered pairs of neighbours (d = 1 = e) and 4 diagonal pairs (d = 2, e = sqrt 2)
    assert s[0, 0] == 12
    assert raw[0] == pytest.approx(4 * (1 - np.sqrt(2) / 2) ** 2 / 12, rel=1e-15)


def test_stress_disconnected_and_additive():
    g = graphs.csr_from_edges(9, np.array([0, 1, 2, 4, 5, 7]), np.array([1, 2, 3, 5, 6, 8]))
    rng = np.random.default_rng(3)
    X = rng.normal(size=(9, 2)).astype(np.float32)
    s = metrics.stress_sums(g.indptr, g.indices, X, np.arange(9))
    assert s[0, 0] == 4 * 3 + 3 * 2 + 2 * 1
    a = metrics.stress_sums(g.indptr, g.indices, X, [0, 4, 8])
    b = metrics.stress_sums(g.indptr, g.indices, X, [1, 2, 3, 5, 6, 7])
    assert np.allclose(a + b, s, rtol=1e-14, atol=0)
    # the single pair (7, 8): d = 1
    e = float(np.hypot(*(X[7].astype(np.float64) - X[8].astype(np.float64))))
    one = metrics.stress_sums(g.indptr, g.indices, X, [8])
    assert one[0, 0] == 1 and one[0, 1] == pytest.approx((1 - e) ** 2, rel=1e-15)


def test_stress_batch_per_graph():
    parts = [_path(6), graphs.grid(3, 4)]
    b = graphs.concat_graphs(parts)
    rng = np.random.default_rng(8)
    X = rng.normal(size=(int(b.graph_offsets[-1]), 2)).astype(np.float32)
    s = metrics.stress_sums(b.indptr, b.indices, X, np.arange(int(b.graph_offsets[-1])), graph_offsets=b.graph_offsets)
    off = b.graph_offsets
    for gi, g in enumerate(parts):
        alone = metrics.stress_sums(g.indptr, g.indices, X[off[gi]:off[gi + 1]], np.arange(g.n))
        assert np.allclose(s[gi], alone[0], rtol=1e-15, atol=0)
