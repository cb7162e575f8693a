"""GPU parity of the tiled attraction layout (row tiles x column windows of X in LDS).

The tiled layout computes the same attractive sums as the row layout in
another order. Expected values come from the FP64 oracle (attraction of
Eq. 6 and the full gradient of the interpolation scheme) on seeded inputs:
P from the oracle's build for small graphs, and seeded random sparse
matrices (hub rows, empty rows, several column windows, pieces that need
several passes) where only the sparse sum is under test.
Tolerances: F_attr 1e-6 relative L2 against FP64 (FP32 products and sums);
the total gradient 1e-3 as for the row layout.
"""
import numpy as np
import pytest

from helpers import P32, rel_l2, say
from oracle import affinities, gradient
from oracle.gradient import CostParams
from synth import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROWS, TILED = 1, 2


@pytest.fixture(scope="module")
def api():
    from paper_2509_19785_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


class _CSR:
    def __init__(self, rowptr, col, val):
        self.rowptr, self.col, self.val = rowptr, col, val


def _terms(api, prob, X, layout, **kw):
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    out = prob.grad_terms(Xt, api.Params(attract_layout=layout, **kw))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _compare_layouts(api, ctx, rowptr, col, val, X, label, goff=None, **kw):
    say(f"[tiled attraction] {label} n={rowptr.shape[0] - 1} nnz={col.shape[0]}")
    prob = api.Problem.from_host(ctx, rowptr, col, val.astype(np.float32), goff)
    t = _terms(api, prob, X, TILED, **kw)
    r = _terms(api, prob, X, ROWS, **kw)
    P = _CSR(rowptr, col, val)
    fa = gradient.attraction_all(X.astype(np.float64), rowptr, col, P32(P).val)
    e_t = rel_l2(t["F_attr"], fa)
    e_r = rel_l2(r["F_attr"], fa)
    e_g = rel_l2(t["G"], r["G"])
    say(f"   F_attr tiled {e_t:.2e} rows {e_r:.2e}; G tiled vs rows {e_g:.2e}")
    assert e_t <= 1e-6
    assert e_g <= 1e-6
    # the repulsive and entropy terms do not depend on the layout of P
    for k in ("F_rep", "F_ent", "Z_i", "Z"):
        assert np.array_equal(t[k], r[k]), k
    return prob, t


def test_grid32_full_gradient(api, ctx):
    g = graphs.workload_grid32()
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=0)
    X = graphs.initial_layout(g.n, 2, std=2.0)
    prob, t = _compare_layouts(api, ctx, P.rowptr, P.col, P.val, X, "grid32")
    ex = gradient.grad_terms(X.astype(np.float64), P, CostParams())
    assert rel_l2(t["G"], ex.G) <= 1e-3


def test_sbm_ragged_full_gradient(api, ctx):
    g = graphs.sbm([700, 900, 1433], 0.012, 4e-4, 11)
    P = affinities.build_P(g.indptr, g.indices, 15.0, seed=3)
    X = graphs.initial_layout(g.n, 5, std=0.7)
    prob, t = _compare_layouts(api, ctx, P.rowptr, P.col, P.val, X, "sbm 3033", min_intervals=8)
    ex = gradient.grad_terms(X.astype(np.float64), P, CostParams())
    assert rel_l2(t["G"], ex.G) <= 1e-3


def test_batch_and_tiny_graphs(api, ctx):
    parts = [graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)),
             graphs.grid(16, 20), graphs.random_recursive_tree(777, 9),
             graphs.csr_from_edges(2, np.array([0]), np.array([1]))]
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 10.0, seed=1, graph_offsets=b.graph_offsets)
    n = b.indptr.shape[0] - 1
    X = graphs.initial_layout(n, 3, std=1.5)
    prob, t = _compare_layouts(api, ctx, P.rowptr, P.col, P.val, X, "batch G=4", goff=b.graph_offsets)
    ex = gradient.grad_terms(X.astype(np.float64), P, CostParams(), b.graph_offsets)
    assert np.allclose(t["G"][0], 1.2 * X[0], rtol=1e-6)
    assert rel_l2(t["G"][1:], ex.G[1:]) <= 1e-3


@pytest.mark.parametrize("n,mean_len,hubs,hub_len,empty,seed", [
    (9000, 30.0, 3, 4000, 0.0, 1),      # two column windows, hub rows across many pieces
    (20000, 400.0, 4, 15000, 0.0, 2),   # pieces longer than one pass (> 512 entries)
    (70000, 12.0, 2, 30000, 0.2, 3),    # nine windows, empty rows, unused slots
    (8192, 5.0, 0, 0, 0.0, 4),          # exactly one full window
    (8193, 5.0, 1, 8192, 0.0, 5),       # one vertex in the second window
])
def test_random_sparse(api, ctx, n, mean_len, hubs, hub_len, empty, seed):
    rowptr, col, val = graphs.random_affinity(n, mean_len, seed, hubs, hub_len, empty)
    X = graphs.initial_layout(n, seed, std=3.0)
    _compare_layouts(api, ctx, rowptr, col, val, X, f"random n={n} len={mean_len}", min_intervals=8,
                     max_intervals=64)


def test_batch_tiles_per_graph(api, ctx):
    """A batch whose graphs start and end inside column windows: graphs of 1,
    300 and 5000 vertices sharing windows, one of 20000 spanning four, hub
    rows and empty rows. Each graph's rows get tiles of their own that walk
    only the windows of that graph."""
    sizes = [5000, 1, 12000, 300, 20000, 9000, 1, 7000]
    parts, off = [], [0]
    for k, m in enumerate(sizes):
        if m == 1:
            parts.append((np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0)))
        else:
            parts.append(graphs.random_affinity(m, 25.0, 40 + k, 2 if m > 1000 else 0,
                                                min(m - 1, 3000), 0.1))
        off.append(off[-1] + m)
    rowptr = np.concatenate([[0]] + [p[0][1:] + sum(q[1].shape[0] for q in parts[:k])
                                     for k, p in enumerate(parts)]).astype(np.int64)
    col = np.concatenate([p[1] + off[k] for k, p in enumerate(parts)]).astype(np.int32)
    val = np.concatenate([p[2] for p in parts])
    goff = np.asarray(off, np.int64)
    X = graphs.initial_layout(off[-1], 8, std=3.0)
    _compare_layouts(api, ctx, rowptr, col, val, X, "batch of 8, windows shared and spanned",
                     goff=goff, min_intervals=8, max_intervals=64)


def test_empty_P(api, ctx):
    n = 5000
    rowptr = np.zeros(n + 1, np.int64)
    X = graphs.initial_layout(n, 1, std=1.0)
    prob, t = _compare_layouts(api, ctx, rowptr, np.zeros(0, np.int32), np.zeros(0), X, "empty P",
                               max_intervals=64)
    assert not t["F_attr"].any()


def test_tiled_bitwise_deterministic(api, ctx):
    rowptr, col, val = graphs.random_affinity(30000, 60.0, 7, 3, 20000)
    prob = api.Problem.from_host(ctx, rowptr, col, val.astype(np.float32))
    X = torch.tensor(graphs.initial_layout(30000, 4, std=2.0), device="cuda")
    prm = api.Params(attract_layout=TILED, max_intervals=64)
    a = prob.grad_terms(X, prm)
    b = prob.grad_terms(X, prm)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_invalid_layout_rejected(api, ctx):
    from paper_2509_19785_amd import _lib
    rowptr, col, val = graphs.random_affinity(100, 3.0, 1)
    prob = api.Problem.from_host(ctx, rowptr, col, val.astype(np.float32))
    X = torch.zeros(100, 2, device="cuda")
    with pytest.raises(RuntimeError):
        prob.grad(X, api.Params(attract_layout=3))
    assert b"attract_layout" in _lib.lib.tsnet_last_error()
