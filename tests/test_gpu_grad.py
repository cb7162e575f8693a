"""GPU parity of the interpolation gradient, step, cost and FP64 direct path.

Every expected value comes from the FP64 oracle on the same seeded inputs;
P is built by the oracle and handed to the library with tsnet_P_from_host.
Tolerances: kernel arithmetic against the FP64 interpolation oracle (same
scheme) 2e-5; the total gradient against the exact O(n^2) oracle 1e-3
relative L2. Only at a converged layout, where the gradient itself is ~0 and
its relative error says nothing, the error is measured against the size of
its terms instead (both numbers are printed for every case).
"""
import numpy as np
import pytest

from helpers import P32, rel_l2, say
from oracle import affinities, gradient, interp, step as ostep
from oracle.gradient import CostParams
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


@pytest.fixture(scope="module")
def grid_problem():
    g = graphs.workload_grid32()
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=0)
    return g, P


def _upload(api, ctx, P, goff=None):
    return api.Problem.from_host(ctx, P.rowptr, P.col, P.val.astype(np.float32), goff)


def _terms(api, prob, X, prm=None):
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    out = prob.grad_terms(Xt, prm or api.Params())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _interp_tol(X32):
    """FP32 tolerance against the FP64 interpolation oracle.

    F_rep and F_ent are formed as (x - c) phi[K,1] - half * phi[K,x]; both
    products are of size half-span times the local sum, so FP32 rounding of
    the transforms (about 1e-7 log2 M relative) is amplified by the ratio of
    the half-span to the local interaction range (~1).
    """
    half = 0.5 * float((X32.max(0) - X32.min(0)).max())
    return 2e-5 * max(1.0, half / 4.0)


def _check_against_oracles(api, prob, P, X32, prm, tol_interp=None, tol_total=1e-3, label="",
                           tol_terms=None, tol_Z=1e-4, converged=False):
    say(f"[grad parity] {label} n={X32.shape[0]}")
    tol_interp = tol_interp or _interp_tol(X32)
    tol_terms = tol_terms or tol_total
    got = _terms(api, prob, X32, prm)
    X = X32.astype(np.float64)
    cp = CostParams(prm.lambda_kl, prm.lambda_c, prm.lambda_r, prm.eps_r)
    ex = gradient.grad_terms(X, P, cp)
    it = interp.interp_terms(X, prm.eps_r, prm.interval_width, prm.min_intervals, prm.max_intervals,
                             far_trim=prm.far_trim)
    fa = gradient.attraction_all(X, P.rowptr, P.col, P32(P).val)
    e_attr = rel_l2(got["F_attr"], fa)
    e_rep_i = rel_l2(got["F_rep"], it.F_rep)
    e_ent_i = rel_l2(got["F_ent"], it.F_ent)
    e_z_i = rel_l2(got["Z_i"], it.Z_i)
    e_rep = rel_l2(got["F_rep"], ex.F_rep)
    e_ent = rel_l2(got["F_ent"], ex.F_ent)
    e_Z = abs(got["Z"][0] - ex.Z[0]) / ex.Z[0]
    n = X.shape[0]
    scale = (np.linalg.norm(4 * cp.lambda_kl * ex.F_attr) + np.linalg.norm(4 * cp.lambda_kl * ex.F_rep / ex.Z[0])
             + np.linalg.norm(cp.lambda_c / n * X) + np.linalg.norm(cp.lambda_r / n ** 2 * ex.F_ent))
    e_G = rel_l2(got["G"], ex.G)
    e_G_terms = np.linalg.norm(got["G"] - ex.G) / scale
    say(f"   attr {e_attr:.2e} rep(interp) {e_rep_i:.2e} ent(interp) {e_ent_i:.2e} Zi(interp) {e_z_i:.2e}"
        f" rep {e_rep:.2e} ent {e_ent:.2e} Z {e_Z:.2e} G {e_G:.2e} G/terms {e_G_terms:.2e}"
        f" n_int {it.grid.n_int} far {int(it.far.sum())}")
    assert e_attr <= 1e-6
    assert e_rep_i <= tol_interp and e_ent_i <= tol_interp and e_z_i <= tol_interp
    assert e_rep <= tol_terms and e_ent <= tol_terms and e_Z <= tol_Z
    if converged:
        assert e_G_terms <= 1e-5
    else:
        assert e_G <= tol_total
    # the grid the GPU used is the oracle's grid, with the same far points
    gi = prob.grid_info()
    assert int(gi["n_intervals"][0]) == it.grid.n_int
    assert abs(float(gi["box_side"][0]) - it.grid.h) <= 1e-6 * it.grid.h
    assert int(gi["far_points"][0]) == int(it.far.sum())
    return got, ex


def test_grid32_initial_layout(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = graphs.initial_layout(g.n, 0)
    _check_against_oracles(api, prob, P, X, api.Params(), label="grid32 init")


@pytest.mark.parametrize("std,max_int", [(1.0, 512), (4.0, 256), (8.0, 256), (12.0, 512), (1.0, 64)])
def test_grid32_spread_layouts(api, ctx, grid_problem, std, max_int):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = graphs.initial_layout(g.n, 7, std=std)
    ctx.status()
    _check_against_oracles(api, prob, P, X, api.Params(max_intervals=max_int),
                           label=f"grid32 std={std} cap={max_int}")
    assert ctx.status() == 0


def test_capped_grid_flags_status(api, ctx, grid_problem):
    # span ~150 needs ~600 boxes of 0.25; with a cap of 256 the box side is
    # ~0.6, so the per-term interpolation error grows as h^3 (about 1e-2) and
    # the status word says so; the total gradient still meets 1e-3.
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = graphs.initial_layout(g.n, 7, std=25.0)
    ctx.status()
    _check_against_oracles(api, prob, P, X, api.Params(max_intervals=256), tol_terms=3e-2,
                           tol_Z=1e-2, label="grid32 capped")
    from paper_2509_19785_amd import _lib
    assert ctx.status() & _lib.TSNET_STATUS_GRID_CAPPED


@pytest.mark.parametrize("max_int", [1024, 512])
def test_span_200_grid(api, ctx, max_int):
    """A uniform square of side 200 (no far points) needs 800 boxes of 0.25
    per axis. With max_intervals = 1024 the grid has 1024 intervals (FFT
    length 6144, the large transform class), is not capped, and every term
    matches exact pair sums on sampled rows within the interpolation error
    at h = 0.195 (the FP64 interpolation oracle gives 2.6e-4 for F_rep,
    1.8e-4 for F_ent and 1.1e-5 for Z_i on a square of the same density and
    box side) plus FP32 rounding amplified by the half-span. With the cap of
    512 the same layout is capped (h = 0.39, about 8x those errors) and
    flagged."""
    from paper_2509_19785_amd import _lib
    n = 60000
    X = graphs.uniform_square(n, 200.0, 21)
    rowptr, col, val = graphs.random_affinity(n, 8.0, 3)
    prob = api.Problem.from_host(ctx, rowptr, col, val.astype(np.float32))
    prm = api.Params(max_intervals=max_int)
    say(f"[grad parity] uniform square side 200, n={n}, max_intervals {max_int}")
    ctx.status()
    t = _terms(api, prob, X, prm)
    st = ctx.status()
    ni = int(prob.grid_info()["n_intervals"][0])
    rows = np.arange(0, n, 117)
    zi, frep, fent = gradient.pair_sums(X.astype(np.float64), prm.eps_r, rows)
    e_rep = rel_l2(t["F_rep"][rows], frep)
    e_ent = rel_l2(t["F_ent"][rows], fent)
    e_z = rel_l2(t["Z_i"][rows], zi)
    say(f"   n_int {ni}, status {st:#x}: F_rep {e_rep:.2e} F_ent {e_ent:.2e} Z_i {e_z:.2e}")
    if max_int == 1024:
        assert ni == 1024
        assert not st & _lib.TSNET_STATUS_GRID_CAPPED
        assert e_rep <= 1e-3 and e_ent <= 1e-3 and e_z <= 3e-4
    else:
        assert ni == 512
        assert st & _lib.TSNET_STATUS_GRID_CAPPED
        assert e_rep <= 1e-2 and e_ent <= 1e-2
    prob.free()


def test_converged_layout(api, ctx, grid_problem):
    g, P = grid_problem
    X = graphs.initial_layout(g.n, 0).astype(np.float64)
    upd, gains = np.zeros_like(X), np.ones_like(X)
    for t in range(120):
        G = gradient.grad_terms(X, P).G
        X, upd, gains = ostep.step(X, upd, gains, G, t)
    prob = _upload(api, ctx, P)
    # the gradient has converged (|G| << |4 F_attr|): measured against its terms
    _check_against_oracles(api, prob, P, X.astype(np.float32), api.Params(), label="grid32 t=120",
                           converged=True)


def test_sbm_ragged(api, ctx):
    g = graphs.sbm([700, 900, 1433], 0.012, 4e-4, 11)
    P = affinities.build_P(g.indptr, g.indices, 15.0, seed=3)
    prob = _upload(api, ctx, P)
    X = graphs.initial_layout(g.n, 5, std=0.7)
    _check_against_oracles(api, prob, P, X, api.Params(min_intervals=8), label="sbm 3033")


@pytest.mark.parametrize("n_far,std,seed", [(40, 0.15, 1), (100, 0.3, 2), (8, 0.05, 3)])
def test_far_points_sbm(api, ctx, n_far, std, seed):
    # a dense bulk with far points setting the bounding box: the grid covers
    # the bulk, the far points meet it through the nodes
    g = graphs.sbm([700, 900, 1433], 0.012, 4e-4, 11)
    P = affinities.build_P(g.indptr, g.indices, 15.0, seed=3)
    prob = _upload(api, ctx, P)
    X = graphs.bulk_with_far_points(g.n, seed, n_far=n_far, std=std)
    _, ex = _check_against_oracles(api, prob, P, X, api.Params(), label=f"sbm 3033 far={n_far}")
    assert prob.grid_info()["far_points"][0] >= n_far
    # with the rule off the grid covers the bounding box (and the oracle agrees)
    _check_against_oracles(api, prob, P, X, api.Params(far_trim=0), tol_terms=5e-2, tol_Z=1e-3,
                           tol_total=5e-2, label=f"sbm 3033 far={n_far} rule off")
    assert prob.grid_info()["far_points"][0] == 0


def test_far_points_cost(api, ctx, grid_problem):
    # the ln(eps + r^2) channel of the cost with far points (their own ln
    # sums and their ln kernel at the nodes)
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = graphs.bulk_with_far_points(g.n, 4, n_far=12, std=0.2)
    got = prob.cost(torch.tensor(X, device="cuda")).cpu().numpy()[0]
    assert prob.grid_info()["far_points"][0] >= 12
    ex = gradient.cost_terms(X.astype(np.float64), P, CostParams())
    say(f"[cost parity] far points: gpu {got} oracle {ex.kl[0]} {ex.cmp[0]} {ex.ent[0]}")
    assert abs(got[0] - ex.kl[0]) <= 1e-5 * abs(ex.kl[0])
    assert abs(got[2] - ex.ent[0]) <= 1e-4 * abs(ex.ent[0])
    assert abs(got[3] - ex.total[0]) <= 1e-5 * abs(ex.total[0])


def test_nonfinite_layout_raises_status(api, ctx, grid_problem):
    # NaN or Inf in X: the grid set-up raises TSNET_STATUS_NONFINITE through
    # the C ABI (the call itself is asynchronous and returns TSNET_OK)
    from paper_2509_19785_amd import _lib
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    for bad in (np.nan, np.inf):
        X = graphs.initial_layout(g.n, 1, std=1.0)
        X[17, 1] = bad
        ctx.status()
        prob.grad(torch.tensor(X, device="cuda"))
        st = ctx.status()
        say(f"[status] X[17] = {bad}: status {st:#x}")
        assert st & _lib.TSNET_STATUS_NONFINITE
    X = graphs.initial_layout(g.n, 1, std=1.0)
    prob.grad(torch.tensor(X, device="cuda"))
    assert not ctx.status() & _lib.TSNET_STATUS_NONFINITE


def test_batch_of_graphs(api, ctx):
    parts = [graphs.grid(16, 20), graphs.sbm([250, 260], 0.05, 0.004, 2), graphs.random_recursive_tree(777, 9)]
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 10.0, seed=1, graph_offsets=b.graph_offsets)
    prob = _upload(api, ctx, P, b.graph_offsets)
    n = b.indptr.shape[0] - 1
    X = graphs.initial_layout(n, 3, std=1.5)
    # the second graph: a dense bulk with far points (the others have none)
    a1, a2 = int(b.graph_offsets[1]), int(b.graph_offsets[2])
    X[a1:a2] = graphs.bulk_with_far_points(a2 - a1, 6, n_far=9, std=0.2)
    say(f"[grad parity] batch G=3 n={n}")
    got = _terms(api, prob, X)
    X64 = X.astype(np.float64)
    ex = gradient.grad_terms(X64, P, CostParams(), b.graph_offsets)
    gi = prob.grid_info()
    for gidx in range(3):
        a0, a1 = int(b.graph_offsets[gidx]), int(b.graph_offsets[gidx + 1])
        it = interp.interp_terms(X64[a0:a1], 0.05)
        assert int(gi["n_intervals"][gidx]) == it.grid.n_int
        assert int(gi["far_points"][gidx]) == int(it.far.sum())
        assert (it.far.sum() > 0) == (gidx == 1)
        assert rel_l2(got["F_rep"][a0:a1], it.F_rep) <= 2e-5
        assert rel_l2(got["F_ent"][a0:a1], it.F_ent) <= 2e-5
        assert rel_l2(got["Z_i"][a0:a1], it.Z_i) <= 2e-5
        assert abs(got["Z"][gidx] - ex.Z[gidx]) <= 1e-4 * ex.Z[gidx]
        assert rel_l2(got["G"][a0:a1], ex.G[a0:a1]) <= 1e-3


def test_batch_of_72_column_layouts(api, ctx):
    """72 small graphs with grids of 8, 16 and 32 intervals in one batch
    (FFT lengths 48, 96 and 192 side by side; with 64 graphs or more every
    graph gets four blocks per transform stage, each packing several
    sequences). Every graph against the FP64 interpolation oracle on its own."""
    parts, stds = [], []
    for k in range(72):
        parts.append(graphs.grid(6, 7) if k % 2 else graphs.random_recursive_tree(50 + k % 9, 100 + k))
        stds.append((0.25, 0.5, 1.0)[k % 3])
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 5.0, seed=2, graph_offsets=b.graph_offsets)
    prob = _upload(api, ctx, P, b.graph_offsets)
    n = b.indptr.shape[0] - 1
    X = np.zeros((n, 2), np.float32)
    for k in range(72):
        a0, a1 = int(b.graph_offsets[k]), int(b.graph_offsets[k + 1])
        X[a0:a1] = graphs.initial_layout(a1 - a0, 500 + k, std=stds[k])
    prm = api.Params(min_intervals=8, max_intervals=32)
    say(f"[grad parity] batch G=72 n={n}, 8-32 intervals")
    got = _terms(api, prob, X, prm)
    gi = prob.grid_info()
    X64 = X.astype(np.float64)
    seen = set()
    for k in range(72):
        a0, a1 = int(b.graph_offsets[k]), int(b.graph_offsets[k + 1])
        it = interp.interp_terms(X64[a0:a1], prm.eps_r, prm.interval_width, prm.min_intervals,
                                 prm.max_intervals, far_trim=prm.far_trim)
        assert int(gi["n_intervals"][k]) == it.grid.n_int
        seen.add(it.grid.n_int)
        assert rel_l2(got["F_rep"][a0:a1], it.F_rep) <= 2e-5, k
        assert rel_l2(got["F_ent"][a0:a1], it.F_ent) <= 2e-5, k
        assert rel_l2(got["Z_i"][a0:a1], it.Z_i) <= 2e-5, k
    assert {8, 16, 32} <= seen


def test_batch_workspace_grows(api, ctx):
    """A batch's grid buffers are pools sized from its first plan (four times
    its needs). A layout whose grids need more is planned down once, with
    TSNET_STATUS_WORKSPACE and GRID_CAPPED raised; the pools then grow before
    the next evaluation, which matches the oracle again."""
    from paper_2509_19785_amd import _lib
    parts = [graphs.grid(16, 20), graphs.sbm([250, 260], 0.05, 0.004, 2),
             graphs.random_recursive_tree(777, 9)]
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 10.0, seed=1, graph_offsets=b.graph_offsets)
    prob = _upload(api, ctx, P, b.graph_offsets)
    n = b.indptr.shape[0] - 1
    X1 = graphs.initial_layout(n, 3, std=0.5)
    ctx.status()
    _terms(api, prob, X1)                      # 64 intervals per graph: sizes the pools
    assert not ctx.status() & _lib.TSNET_STATUS_WORKSPACE
    X2 = X1.copy()
    a1, a2 = int(b.graph_offsets[1]), int(b.graph_offsets[2])
    X2[a1:a2] = graphs.initial_layout(a2 - a1, 4, std=12.0)   # needs 512 intervals
    _terms(api, prob, X2)
    st = ctx.status()
    say(f"[workspace] after the larger layout: status {st:#x}, intervals {prob.grid_info()['n_intervals']}")
    assert st & _lib.TSNET_STATUS_WORKSPACE and st & _lib.TSNET_STATUS_GRID_CAPPED
    got = _terms(api, prob, X2)                # the pools have grown
    assert not ctx.status() & (_lib.TSNET_STATUS_WORKSPACE | _lib.TSNET_STATUS_GRID_CAPPED)
    gi = prob.grid_info()
    X64 = X2.astype(np.float64)
    for gidx in range(3):
        a0, a1_ = int(b.graph_offsets[gidx]), int(b.graph_offsets[gidx + 1])
        it = interp.interp_terms(X64[a0:a1_], 0.05)
        assert int(gi["n_intervals"][gidx]) == it.grid.n_int
        assert rel_l2(got["F_rep"][a0:a1_], it.F_rep) <= _interp_tol(X2[a0:a1_])
        assert rel_l2(got["F_ent"][a0:a1_], it.F_ent) <= _interp_tol(X2[a0:a1_])
    assert int(gi["n_intervals"][1]) == 512


def test_batch_of_twelve_graphs(api, ctx):
    # 8 or more graphs: each graph's FFT stages get 32 blocks, so the column
    # stage packs several columns per block (6 at M = 384), fewer than the
    # buffer holds; every graph against the oracle's interpolated sums
    parts = []
    for i in range(12):
        if i % 3 == 0:
            parts.append(graphs.grid(6 + i, 9))
        elif i % 3 == 1:
            parts.append(graphs.random_recursive_tree(150 + 37 * i, 20 + i))
        else:
            parts.append(graphs.sbm([60 + 5 * i, 90], 0.08, 0.01, 30 + i))
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 10.0, seed=2, graph_offsets=b.graph_offsets)
    prob = _upload(api, ctx, P, b.graph_offsets)
    n = b.indptr.shape[0] - 1
    X = graphs.initial_layout(n, 8, std=1.5)
    say(f"[grad parity] batch G=12 n={n}")
    got = _terms(api, prob, X)
    X64 = X.astype(np.float64)
    ex = gradient.grad_terms(X64, P, CostParams(), b.graph_offsets)
    gi = prob.grid_info()
    for gidx in range(12):
        a0, a1 = int(b.graph_offsets[gidx]), int(b.graph_offsets[gidx + 1])
        it = interp.interp_terms(X64[a0:a1], 0.05)
        assert int(gi["n_intervals"][gidx]) == it.grid.n_int
        assert rel_l2(got["F_rep"][a0:a1], it.F_rep) <= 2e-5, gidx
        assert rel_l2(got["F_ent"][a0:a1], it.F_ent) <= 2e-5, gidx
        assert abs(got["Z"][gidx] - ex.Z[gidx]) <= 1e-4 * ex.Z[gidx]
        assert rel_l2(got["G"][a0:a1], ex.G[a0:a1]) <= 1e-3


@pytest.mark.parametrize("n", [100000, 300000, 600000, 1200000])
def test_mid_size_interpolated_terms(api, ctx, n):
    # sizes whose spread ranges are 64, 128, 256 and 512 sorted points (the
    # range halves from 1024 while the problem has fewer than 2048 ranges; from
    # 2,096,129 vertices on it stays 1024); 30% of the points in a tight
    # cluster, so dense boxes span many ranges: every vertex's interpolated
    # sums against the oracle's
    rowptr, col, val = graphs.random_affinity(n, 4.0, 50)
    prob = api.Problem.from_host(ctx, rowptr, col, val.astype(np.float32))
    rng = np.random.default_rng(n)
    X = (rng.normal(size=(n, 2)) * np.where(rng.random((n, 1)) < 0.3, 0.2, 3.0)).astype(np.float32)
    prm = api.Params(max_intervals=128)
    got = _terms(api, prob, X, prm)
    it = interp.interp_terms(X.astype(np.float64), prm.eps_r, prm.interval_width, prm.min_intervals,
                             prm.max_intervals)
    errs = {k: rel_l2(got[k], getattr(it, k)) for k in ("F_rep", "F_ent", "Z_i")}
    say(f"[grad parity] n={n}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()) +
        f" n_int {it.grid.n_int}")
    assert max(errs.values()) <= _interp_tol(X)
    assert int(prob.grid_info()["n_intervals"][0]) == it.grid.n_int


def test_tiny_graphs(api, ctx):
    # n = 1: no pairs, G = (lambda_c / n) X; n = 2 and 3 in one batch with it
    parts = [graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)),
             graphs.csr_from_edges(2, np.array([0]), np.array([1])),
             graphs.csr_from_edges(3, np.array([0, 1]), np.array([1, 2]))]
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 2.0, graph_offsets=b.graph_offsets)
    prob = _upload(api, ctx, P, b.graph_offsets)
    X = np.array([[0.3, -0.4], [0.0, 0.0], [1.0, 0.5], [2.0, 1.0], [2.5, 1.2], [1.7, 0.1]], np.float32)
    got = _terms(api, prob, X)
    ex = gradient.grad_terms(X.astype(np.float64), P, CostParams(), b.graph_offsets)
    assert np.allclose(got["G"][0], 1.2 * X[0], rtol=1e-6)
    assert got["Z"][0] == 0.0
    assert rel_l2(got["G"][1:], ex.G[1:]) <= 1e-3


def test_bitwise_deterministic(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = torch.tensor(graphs.initial_layout(g.n, 4, std=2.0), device="cuda")
    a = prob.grad_terms(X)
    b = prob.grad_terms(X)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_step_matches_oracle(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (g.n, 2)).astype(np.float32)
    U = rng.normal(0, 0.01, (g.n, 2)).astype(np.float32)
    K = rng.uniform(0.005, 3, (g.n, 2)).astype(np.float32)
    G = rng.normal(0, 1e-3, (g.n, 2)).astype(np.float32)
    for it, sp in [(3, api.StepParams()), (400, api.StepParams(eta=50.0))]:
        tX, tU, tK, tG = (torch.tensor(a, device="cuda") for a in (X, U, K, G))
        prob.step(tX, tU, tK, tG, it, sp)
        torch.cuda.synchronize()
        osp = ostep.StepParams(eta=sp.eta)
        eX, eU, eK = ostep.step(X, U, K, G, it, osp)
        # FP32 bound: a few units of rounding of the operands of each sum
        # (X + update cancels where X ~ -update, so relative error is unbounded)
        e32 = 2.0 ** -24
        mu = 0.5 if it < 250 else 0.8
        eta = sp.eta if sp.eta > 0 else 200.0
        bU = 4 * e32 * (np.abs(mu * U) + np.abs(eta * eK * G))
        bX = 4 * e32 * (np.abs(X) + np.abs(eU)) + 2 * bU
        assert np.allclose(tK.cpu().numpy(), eK, rtol=2e-7, atol=0)
        assert np.all(np.abs(tU.cpu().numpy() - eU) <= bU)
        assert np.all(np.abs(tX.cpu().numpy() - eX) <= bX)


def test_step_odd_n_and_unaligned_arrays(api, ctx):
    """The step at an odd n (the last vertex outside the pairs of the 16-byte
    path) and on arrays offset by 8 bytes (the one-vertex path): both against
    the step oracle, and bit for bit against each other (same arithmetic)."""
    g = graphs.grid(31, 33)  # n = 1023
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=0)
    prob = _upload(api, ctx, P)
    n = g.n
    assert n % 2 == 1
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (n, 2)).astype(np.float32)
    U = rng.normal(0, 0.01, (n, 2)).astype(np.float32)
    K = rng.uniform(0.005, 3, (n, 2)).astype(np.float32)
    G = rng.normal(0, 1e-3, (n, 2)).astype(np.float32)
    it, sp = 3, api.StepParams()
    eX, eU, eK = ostep.step(X, U, K, G, it, ostep.StepParams(eta=sp.eta))
    out = {}
    for offset in (0, 1):  # rows of 8 bytes: offset 1 leaves every array 8 mod 16
        bufs = []
        for a in (X, U, K, G):
            t = torch.zeros((n + offset, 2), dtype=torch.float32, device="cuda")
            t[offset:] = torch.tensor(a, device="cuda")
            bufs.append(t[offset:])
        assert all((b.data_ptr() % 16 == 0) == (offset == 0) for b in bufs)
        tX, tU, tK, tG = bufs
        prob.step(tX, tU, tK, tG, it, sp)
        torch.cuda.synchronize()
        out[offset] = [t.cpu().numpy() for t in (tX, tU, tK)]
        e32 = 2.0 ** -24
        bU = 4 * e32 * (np.abs(0.5 * U) + np.abs(200.0 * eK * G))
        bX = 4 * e32 * (np.abs(X) + np.abs(eU)) + 2 * bU
        gX, gU, gK = out[offset]
        assert np.allclose(gK, eK, rtol=2e-7, atol=0)
        assert np.all(np.abs(gU - eU) <= bU)
        assert np.all(np.abs(gX - eX) <= bX)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_cost_matches_oracle(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    for std in (0.01, 1.0):
        X = graphs.initial_layout(g.n, 2, std=std)
        say(f"[cost parity] std={std}")
        got = prob.cost(torch.tensor(X, device="cuda")).cpu().numpy()[0]
        ex = gradient.cost_terms(X.astype(np.float64), P, CostParams())
        say(f"   gpu {got} oracle {ex.kl[0]} {ex.cmp[0]} {ex.ent[0]}")
        assert abs(got[0] - ex.kl[0]) <= 1e-5 * abs(ex.kl[0])
        assert abs(got[1] - ex.cmp[0]) <= 1e-6 * abs(ex.cmp[0])
        assert abs(got[2] - ex.ent[0]) <= 1e-4 * abs(ex.ent[0])
        assert abs(got[3] - ex.total[0]) <= 1e-5 * abs(ex.total[0])


@pytest.mark.parametrize("std", [0.01, 3.0])
def test_direct_f64_matches_oracle(api, ctx, grid_problem, std):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = graphs.initial_layout(g.n, 8, std=std).astype(np.float64)
    say(f"[direct parity] std={std}")
    Gd, Zd, T = prob.grad_direct_f64(torch.tensor(X, device="cuda"), with_terms=True)
    torch.cuda.synchronize()
    ex = gradient.grad_terms(X, P32(P), CostParams())
    T = T.cpu().numpy()
    assert abs(Zd.item() - ex.Z[0]) <= 1e-12 * ex.Z[0]
    assert rel_l2(T[:, 0:2], ex.F_attr) <= 1e-12
    assert rel_l2(T[:, 2:4], ex.F_rep) <= 1e-12
    assert rel_l2(T[:, 4:6], ex.F_ent) <= 1e-12
    assert rel_l2(T[:, 6], ex.Z_i) <= 1e-12
    assert rel_l2(Gd.cpu().numpy(), ex.G) <= 1e-12
    rows = np.array([0, 5, 511, 1023, 77], dtype=np.int32)
    Gr, Zr = prob.grad_direct_f64(torch.tensor(X, device="cuda"), rows=rows)
    assert abs(Zr.item() - ex.Z[0]) <= 1e-12 * ex.Z[0]
    assert rel_l2(Gr.cpu().numpy(), ex.G[rows]) <= 1e-12


def test_context_outlives_its_problems(api):
    from paper_2509_19785_amd import _lib
    c = api.Context(0)
    rowptr, col, val = graphs.random_affinity(50, 3.0, 1)
    prob = api.Problem.from_host(c, rowptr, col, val.astype(np.float32))
    assert _lib.lib.tsnet_ctx_destroy(c.handle) == _lib.TSNET_EINVAL
    assert b"free them first" in _lib.lib.tsnet_last_error()
    X = torch.zeros(50, 2, device="cuda")
    prob.grad(X)                      # the context is still intact
    torch.cuda.synchronize()
    c.close()                         # frees the problem first
    assert prob.handle is None and c.handle is None
