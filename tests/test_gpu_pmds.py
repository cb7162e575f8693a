"""GPU parity of the Pivot MDS starting layout (tsnet_pmds) against the oracle.

Integer work is compared bit for bit: the pivots (max-min selection over the
BFS distances). The FP64 eigenvalues of C^T C agree to 1e-9 relative. The
float32 layout is compared element by element, to 2e-6 of the graph's largest
coordinate, where the two leading eigenvalues are apart (relative gap 1e-6 or
more: otherwise the eigenvectors are not unique and only the spread of the
first axis is compared). Graphs: a path (the exact linear case), rectangular
grids, a tree, an SBM, a batch with a disconnected graph and a one-vertex
graph, and the Barabasi-Albert graph of the benchmark (n = 1e6).
"""
import numpy as np
import pytest

from helpers import say
from oracle import pmds as opmds
from synth import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_2509_19785_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


def _compare(api, ctx, indptr, indices, pivots, seed, scale=1e-2, graph_offsets=None, label=""):
    got = api.pmds(ctx, indptr, indices, pivots=pivots, seed=seed, scale=scale,
                   graph_offsets=graph_offsets)
    torch.cuda.synchronize()
    ref = opmds.pmds(indptr, indices, pivots=pivots, seed=seed, scale=scale,
                     graph_offsets=graph_offsets)
    X = got["X"].cpu().numpy().astype(np.float64)
    piv = got["pivots"].cpu().numpy()
    n = len(indptr) - 1
    off = np.array([0, n]) if graph_offsets is None else np.asarray(graph_offsets)
    worst = 0.0
    for g in range(len(off) - 1):
        a, b = int(off[g]), int(off[g + 1])
        k = len(ref.pivots[g])
        assert np.array_equal(piv[g, :k], ref.pivots[g]), (label, g)
        assert np.all(piv[g, k:] == -1), (label, g)
        for ax in range(2):
            e_ref = ref.eig[g, ax]
            assert abs(got["eig"][g, ax] - e_ref) <= 1e-9 * max(abs(ref.eig[g, 0]), 1e-300), (label, g)
        span = np.abs(ref.X[a:b]).max()
        gap = (ref.eig[g, 0] - ref.eig[g, 1]) / ref.eig[g, 0] if ref.eig[g, 0] > 0 else 0.0
        if span == 0:
            assert np.all(X[a:b] == 0), (label, g)
        elif gap >= 1e-6:
            err = np.abs(X[a:b] - ref.X[a:b]).max() / span
            worst = max(worst, err)
            assert err <= 2e-6, (label, g, err)
        else:
            assert abs(X[a:b, 0].std() - scale) <= 1e-6 * scale, (label, g)
    say(f"[pmds] {label}: n={n} graphs={len(off) - 1} levels={got['levels']} "
        f"max rel err {worst:.2e} lambda {got['eig'][0]}")
    return got, ref


def test_path_linear(api, ctx):
    n = 300
    g = graphs.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    got, _ = _compare(api, ctx, g.indptr, g.indices, pivots=10, seed=5, label="path")
    x = got["X"].cpu().numpy().astype(np.float64)
    assert abs(abs(np.corrcoef(x[:, 0], np.arange(n))[0, 1]) - 1) < 1e-6
    assert np.abs(x[:, 1]).max() <= 1e-4 * np.abs(x[:, 0]).max()


@pytest.mark.parametrize("rows,cols,pivots", [(40, 20, 50), (9, 37, 128), (3, 5, 50)])
def test_grids(api, ctx, rows, cols, pivots):
    g = graphs.grid(rows, cols)
    _compare(api, ctx, g.indptr, g.indices, pivots=pivots, seed=rows, label=f"grid {rows}x{cols}")


def test_tree_and_sbm(api, ctx):
    t = graphs.random_recursive_tree(5000, 3)
    _compare(api, ctx, t.indptr, t.indices, pivots=50, seed=1, label="tree 5000")
    s = graphs.sbm([500] * 4, 0.02, 0.001, 2)
    _compare(api, ctx, s.indptr, s.indices, pivots=64, seed=2, label="sbm 2000")


def test_batch_with_pieces_and_single_vertex(api, ctx):
    parts = [graphs.grid(12, 7), graphs.random_recursive_tree(700, 9),
             graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)),
             graphs.csr_from_edges(9, np.array([0, 1, 2, 4, 5, 7]), np.array([1, 2, 3, 5, 6, 8])),
             graphs.sbm([200, 300], 0.05, 0.002, 4)]
    b = graphs.concat_graphs(parts)
    got, ref = _compare(api, ctx, b.indptr, b.indices, pivots=20, seed=11,
                        graph_offsets=b.graph_offsets, label="batch")
    off = b.graph_offsets
    assert np.all(got["X"].cpu().numpy()[off[2]:off[3]] == 0)
    # reproducible bit for bit
    again = api.pmds(ctx, b.indptr, b.indices, pivots=20, seed=11, graph_offsets=b.graph_offsets)
    assert torch.equal(again["X"], got["X"]) and torch.equal(again["pivots"], got["pivots"])


def test_ba1m(api, ctx):
    g = graphs.workload_ba1m()
    say(f"[pmds] BA n={g.n}: oracle (50 BFS on the host)")
    _compare(api, ctx, g.indptr, g.indices, pivots=50, seed=3, label="BA 1e6")


def test_rejects_bad_graph(api, ctx):
    from paper_2509_19785_amd._lib import TsnetError
    g = graphs.grid(4, 4)
    bad = g.indices.copy()
    bad[0] = 15  # breaks symmetry and order
    with pytest.raises(TsnetError):
        api.pmds(ctx, g.indptr, bad, pivots=4)
