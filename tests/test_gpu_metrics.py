"""GPU parity of the layout quality metrics (tsnet_np, tsnet_stress) against the oracle.

Neighbourhood preservation is integer work and is compared bit for bit: the
2-hop ball size and the hits of every evaluated vertex. NP per graph (FP64
mean of the ratios, summed in another order) agrees to 1e-12 relative.
Stress: the pair counts exactly, the FP64 sums to 1e-12 relative (1e-10 at
n = 1e6, where a million terms are summed in different orders).

Layouts: uniform, clustered (90% of the points in a cloud 1e4 times smaller),
two far clumps, coincident points, points on a quarter lattice (many equal
distances), a grid drawn on its own lattice, on a line and on a diagonal, a
far outlier, coordinates near the float range and at scale 1e-30; graphs: SBM, grid, tree, star (its leaves take the heavy
path: more than 4096 two-hop walks), a batch with a single vertex, isolated
vertices and a disconnected graph, and the Barabasi-Albert graph of the
benchmark (n = 1e6) on sampled vertices and sources.
"""
import numpy as np
import pytest

from helpers import say
from oracle import metrics as om
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


def _layouts(n, seed):
    rng = np.random.default_rng(seed)
    clump = np.where(rng.random((n, 1)) < 0.9, 1e-4, 1.0)
    return {
        "uniform": rng.uniform(-1, 1, (n, 2)),
        "clustered": rng.normal(size=(n, 2)) * clump,
        "coincident": np.zeros((n, 2)),
        "quarter lattice": np.round(rng.uniform(-1, 1, (n, 2)) * 4) / 4,
    }


def _np_compare(api, ctx, g, X, vertices=None, graph_offsets=None, label=""):
    X32 = np.ascontiguousarray(X, dtype=np.float32)
    Xd = torch.from_numpy(X32).cuda()
    got = api.neighbourhood_preservation(ctx, g.indptr, g.indices, Xd, vertices=vertices,
                                         graph_offsets=graph_offsets)
    torch.cuda.synchronize()
    ball, hits, npg = om.neighbourhood_preservation(g.indptr, g.indices, X32, vertices=vertices,
                                                    graph_offsets=graph_offsets)
    gb = got["ball"].cpu().numpy()
    gh = got["hits"].cpu().numpy()
    assert np.array_equal(gb, ball), label
    bad = np.nonzero(gh != hits)[0]
    assert bad.size == 0, (label, bad[:5], gh[bad[:5]], hits[bad[:5]])
    assert np.array_equal(np.isnan(got["np"]), np.isnan(npg)), label
    ok = ~np.isnan(npg)
    assert np.allclose(got["np"][ok], npg[ok], rtol=1e-12, atol=0), label
    say(f"[np] {label}: {len(gb)} vertices, sum k {int(gb.sum())}, NP {got['np'][:3]}")
    return got


def _stress_compare(api, ctx, g, X, sources, graph_offsets=None, rtol=1e-12, label=""):
    X32 = np.ascontiguousarray(X, dtype=np.float32)
    got = api.stress(ctx, g.indptr, g.indices, torch.from_numpy(X32).cuda(), sources,
                     graph_offsets=graph_offsets)
    ref = om.stress_sums(g.indptr, g.indices, X32, sources, graph_offsets=graph_offsets)
    raw, best = om.stress_values(ref)
    assert np.array_equal(got["sums"][:, 0], ref[:, 0]), label
    assert np.allclose(got["sums"][:, 1:], ref[:, 1:], rtol=rtol, atol=0), label
    ok = ~np.isnan(raw)
    assert np.array_equal(np.isnan(got["stress"]), ~ok), label
    assert np.allclose(got["stress"][ok], raw[ok], rtol=rtol, atol=0), label
    assert np.allclose(got["stress_best_scale"][ok], best[ok], rtol=1e-9, atol=1e-15), label
    say(f"[stress] {label}: {len(sources)} sources, pairs {int(ref[:, 0].sum())}, "
        f"stress {got['stress'][:3]}, levels {got['levels']}")
    return got


@pytest.mark.parametrize("layout", ["uniform", "clustered", "coincident", "quarter lattice"])
def test_np_sbm_layouts(api, ctx, layout):
    g = graphs.sbm([300, 300, 300], 0.02, 0.002, 1)
    _np_compare(api, ctx, g, _layouts(g.n, 3)[layout], label=f"sbm 900 {layout}")


def test_np_member_outside_candidates(api, ctx):
    # vertex 1 of this drawing has a 2-hop neighbour outside the cells searched
    # whose key shares the top bits of the k-th key: it must not count as a hit
    g = graphs.sbm([100, 100, 100], 0.05, 0.003, 1)
    X = np.random.default_rng(0).uniform(-1, 1, (g.n, 2))
    got = _np_compare(api, ctx, g, X, label="sbm 300 uniform")
    assert int(got["hits"][1]) == 1 and int(got["ball"][1]) == 35
    rng = np.random.default_rng(1)
    two = rng.normal(size=(g.n, 2)) * 1e-3 + np.where(rng.random((g.n, 1)) < 0.5, 0, 50)
    _np_compare(api, ctx, g, two, label="sbm 300 two far clumps")


def test_np_grid_drawings(api, ctx):
    rows, cols = 31, 45
    g = graphs.grid(rows, cols)
    r, c = np.divmod(np.arange(g.n), cols)
    got = _np_compare(api, ctx, g, np.stack([c, r], 1), label="grid on its lattice")
    inner = (r >= 2) & (r < rows - 2) & (c >= 2) & (c < cols - 2)
    assert np.all(got["hits"].cpu().numpy()[inner] == 12)
    _np_compare(api, ctx, g, np.stack([np.arange(g.n), np.zeros(g.n)], 1), label="grid on a line")
    X = np.random.default_rng(5).normal(size=(g.n, 2))
    X[17] = [1e6, -1e6]
    _np_compare(api, ctx, g, X, label="grid with an outlier")
    big = np.random.default_rng(6).uniform(-3e38, 3e38, (g.n, 2))
    _np_compare(api, ctx, g, big, label="grid near the float range")
    _np_compare(api, ctx, g, np.random.default_rng(7).normal(size=(g.n, 2)) * 1e-30,
                label="grid at scale 1e-30 (squared distances underflow)")
    diag = np.stack([np.arange(g.n), np.arange(g.n)], 1) * 1e-3
    _np_compare(api, ctx, g, diag, label="grid on a diagonal")


def test_np_heavy_star_and_tree(api, ctx):
    n = 6000   # every leaf has 5999 two-hop walks: the block-per-vertex path
    star = graphs.csr_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    X = np.random.default_rng(7).normal(size=(n, 2))
    got = _np_compare(api, ctx, star, X, label="star 6000")
    assert np.all(got["ball"].cpu().numpy() == n - 1) and np.all(got["hits"].cpu().numpy() == n - 1)
    t = graphs.random_recursive_tree(5000, 4)
    _np_compare(api, ctx, t, _layouts(t.n, 8)["clustered"], label="tree 5000 clustered")


def test_np_batch_and_samples(api, ctx):
    parts = [graphs.grid(12, 9), graphs.random_recursive_tree(700, 9),
             graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)),
             graphs.csr_from_edges(9, np.array([0, 1, 2, 4, 5, 7]), np.array([1, 2, 3, 5, 6, 8])),
             graphs.csr_from_edges(5, np.array([0]), np.array([1])),
             graphs.sbm([200, 300], 0.05, 0.002, 4)]
    b = graphs.concat_graphs(parts)
    n = int(b.graph_offsets[-1])
    X = np.random.default_rng(9).normal(size=(n, 2))
    full = _np_compare(api, ctx, b, X, graph_offsets=b.graph_offsets, label="batch")
    # the one-vertex graph has no evaluated vertex with k > 0
    assert np.isnan(full["np"][2])
    sample = np.sort(np.random.default_rng(10).choice(n, 300, replace=False))
    part = _np_compare(api, ctx, b, X, vertices=sample, graph_offsets=b.graph_offsets,
                       label="batch sample")
    assert torch.equal(part["hits"], full["hits"][torch.from_numpy(sample).cuda()])
    again = api.neighbourhood_preservation(ctx, b.indptr, b.indices,
                                           torch.from_numpy(X.astype(np.float32)).cuda(),
                                           graph_offsets=b.graph_offsets)
    assert torch.equal(again["hits"], full["hits"]) and np.array_equal(again["np"], full["np"], equal_nan=True)


def test_np_rejects_bad_input(api, ctx):
    from paper_2509_19785_amd._lib import TsnetError
    g = graphs.grid(5, 5)
    X = torch.zeros((g.n, 2), device="cuda")
    with pytest.raises(TsnetError):
        api.neighbourhood_preservation(ctx, g.indptr, g.indices, X, vertices=[3, 2])
    with pytest.raises(TsnetError):
        api.neighbourhood_preservation(ctx, g.indptr, g.indices, X, vertices=[0, 25])
    X[4, 1] = float("nan")
    with pytest.raises(TsnetError):
        api.neighbourhood_preservation(ctx, g.indptr, g.indices, X)


def test_stress_small_graphs(api, ctx):
    n = 40
    path = graphs.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    line = np.stack([np.arange(n) * 0.5, np.zeros(n)], 1)
    got = _stress_compare(api, ctx, path, line, np.arange(n), label="path at spacing 1/2")
    assert got["stress"][0] == pytest.approx(0.25, abs=1e-15)
    assert abs(got["stress_best_scale"][0]) < 1e-12
    g = graphs.sbm([300, 300, 300], 0.02, 0.002, 1)
    for name, X in _layouts(g.n, 3).items():
        _stress_compare(api, ctx, g, X, np.arange(g.n), label=f"sbm 900 {name}")
    grid = graphs.grid(17, 23)
    r, c = np.divmod(np.arange(grid.n), 23)
    _stress_compare(api, ctx, grid, np.stack([c, r], 1), np.arange(grid.n), label="grid lattice")


def test_stress_batch_and_repeats(api, ctx):
    parts = [graphs.grid(6, 7), graphs.random_recursive_tree(300, 2),
             graphs.csr_from_edges(9, np.array([0, 1, 2, 4, 5, 7]), np.array([1, 2, 3, 5, 6, 8])),
             graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64))]
    b = graphs.concat_graphs(parts)
    n = int(b.graph_offsets[-1])
    X = np.random.default_rng(11).normal(size=(n, 2))
    got = _stress_compare(api, ctx, b, X, np.arange(n), graph_offsets=b.graph_offsets,
                          label="batch, all sources")
    assert got["sums"][2, 0] == 4 * 3 + 3 * 2 + 2 * 1 and np.isnan(got["stress"][3])
    # sources in any order, repeated, across graphs, more than one bit-parallel batch
    src = np.random.default_rng(12).integers(0, n, 150)
    first = _stress_compare(api, ctx, b, X, src, graph_offsets=b.graph_offsets, label="batch, sampled")
    again = api.stress(ctx, b.indptr, b.indices, torch.from_numpy(X.astype(np.float32)).cuda(), src,
                       graph_offsets=b.graph_offsets)
    assert np.array_equal(again["sums"], first["sums"])


def test_stress_rejects_bad_source(api, ctx):
    from paper_2509_19785_amd._lib import TsnetError
    g = graphs.grid(4, 4)
    with pytest.raises(TsnetError):
        api.stress(ctx, g.indptr, g.indices, torch.zeros((g.n, 2), device="cuda"), [0, 16])


def test_metrics_ba1m_sampled(api, ctx):
    g = graphs.workload_ba1m()
    rng = np.random.default_rng(13)
    X = rng.normal(size=(g.n, 2)) * np.where(rng.random((g.n, 1)) < 0.5, 0.05, 1.0)
    deg = np.diff(g.indptr)
    hubs = np.argsort(deg)[-4:]
    sample = np.unique(np.concatenate([hubs, rng.choice(g.n, 60, replace=False)]))
    say(f"[np] BA n={g.n}: oracle on {len(sample)} sampled vertices (hub degrees {deg[hubs]})")
    X32 = X.astype(np.float32)
    Xd = torch.from_numpy(X32).cuda()
    _np_compare(api, ctx, g, X32, vertices=sample, label="BA 1e6 sample")
    allv = api.neighbourhood_preservation(ctx, g.indptr, g.indices, Xd)
    part = api.neighbourhood_preservation(ctx, g.indptr, g.indices, Xd, vertices=sample)
    idx = torch.from_numpy(sample.astype(np.int64)).cuda()
    assert torch.equal(allv["hits"][idx], part["hits"]) and torch.equal(allv["ball"][idx], part["ball"])
    kb = allv["ball"].cpu().numpy().astype(np.int64)
    # ball sizes at full size: k_v <= the 2-hop walk count, and the sum of k_v over all
    # vertices is even (the 2-hop relation is symmetric)
    walks = deg + np.add.reduceat(deg[g.indices], g.indptr[:-1]) * (deg > 0)
    assert np.all(kb <= walks) and kb.sum() % 2 == 0
    say(f"[np] BA 1e6 all vertices: NP {allv['np'][0]:.6f}, sum k {kb.sum()}")
    src = rng.choice(g.n, 64, replace=False)
    _stress_compare(api, ctx, g, X32, src, rtol=1e-10, label="BA 1e6, 64 sources")
