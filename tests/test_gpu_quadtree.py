"""GPU parity of the quadtree (Barnes-Hut) terms: BH-tsNET and FIt-tsNET.

The GPU builds the same tree as the oracle (the cells are computed in FP64 on
both sides, so the tree is identical) and walks it with the same test in
FP64; it sums the terms in FP32 and takes centres of mass from FP64 prefix
sums. Tolerances against the oracle's FP64 quadtree sums: F_rep and F_ent
2e-5 relative L2, Z_i and Z 1e-5 (FP32 sums; the opening test can only flip
where it is tied to rounding). With theta = 1e-4 no inner node is a summary
and the sums are the exact all-pairs sums. The gradient assembles those terms
with the exact sparse attraction; FIt-tsNET keeps the interpolated repulsion
bit for bit. Layouts: normal, clustered, rounded (many equal codes), a line,
coincident points, a bulk stretched by four far points (leaves below level
16), a batch with a one-vertex graph, and BA n = 1e6 on sampled vertices.
"""
import numpy as np
import pytest

from helpers import rel_l2, say
from oracle import affinities, gradient, quadtree as oq
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


def _terms(api, prob, X, prm):
    out = prob.grad_terms(torch.tensor(X, dtype=torch.float32, device="cuda"), prm)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _layouts(n, seed):
    rng = np.random.default_rng(seed)
    return {
        "normal": rng.normal(size=(n, 2)) * 4,
        "clustered": rng.normal(size=(n, 2)) * np.where(rng.random((n, 1)) < 0.7, 0.05, 5.0),
        "rounded": np.round(rng.normal(size=(n, 2)) * 3) / 3,
        "line": np.stack([np.linspace(-20, 20, n), np.zeros(n)], 1),
        "coincident": np.zeros((n, 2)),
        # four points 1e4 away: the bulk covers about 1e-4 of the square's side
        "stretched": np.vstack([[[1e4, 0], [-1e4, 0], [0, 1e4], [0, -1e4]], rng.normal(size=(n - 4, 2))]),
    }


def _check_qt(got, ref, label, tol=2e-5):
    zi, frep, fent, _ = ref
    e_rep = rel_l2(got["F_rep"], frep)
    e_ent = rel_l2(got["F_ent"], fent) if np.linalg.norm(fent) > 0 else np.abs(got["F_ent"]).max()
    e_zi = rel_l2(got["Z_i"], zi)
    say(f"[quadtree] {label}: F_rep {e_rep:.2e} F_ent {e_ent:.2e} Z_i {e_zi:.2e}")
    assert e_rep <= tol and e_ent <= tol and e_zi <= 1e-5, label


@pytest.mark.parametrize("theta", [0.5, 0.25])
def test_bh_terms_layouts(api, ctx, grid_problem, theta):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    prm = api.Params.variant("BH-tsNET", theta=theta)
    for name, X in _layouts(g.n, 11).items():
        X32 = X.astype(np.float32)
        got = _terms(api, prob, X32, prm)
        ref = oq.sums(X32, theta=theta, eps=0.05)
        _check_qt(got, ref, f"grid32 {name} theta {theta}")
        assert abs(got["Z"][0] - ref[0].sum()) <= 1e-5 * ref[0].sum()
        # the gradient: the quadtree terms with the exact attraction
        ex = gradient.grad_terms(X32.astype(np.float64), P, CostParams())
        G = gradient.assemble(ex.F_attr, ref[1], ref[2], X32.astype(np.float64), ref[0].sum(), g.n)
        assert rel_l2(got["G"], G) <= 1e-4, name


def test_tiny_theta_is_exact(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = (np.random.default_rng(3).normal(size=(g.n, 2)) * 2).astype(np.float32)
    got = _terms(api, prob, X, api.Params.variant("BH-tsNET", theta=1e-4))
    zi, frep, fent = gradient.pair_sums(X.astype(np.float64), 0.05)
    assert rel_l2(got["F_rep"], frep) <= 2e-5 and rel_l2(got["F_ent"], fent) <= 2e-5
    assert rel_l2(got["Z_i"], zi) <= 1e-5


def test_fit_variant_keeps_interpolated_repulsion(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = (np.random.default_rng(4).normal(size=(g.n, 2)) * 4).astype(np.float32)
    lt = _terms(api, prob, X, api.Params())
    fit = _terms(api, prob, X, api.Params.variant("FIt-tsNET"))
    assert np.array_equal(fit["F_rep"], lt["F_rep"]) and np.array_equal(fit["Z"], lt["Z"])
    assert np.array_equal(fit["Z_i"], lt["Z_i"]) and np.array_equal(fit["F_attr"], lt["F_attr"])
    ref = oq.sums(X, theta=0.5, eps=0.05)
    assert rel_l2(fit["F_ent"], ref[2]) <= 2e-5
    # both variants stay close to the exact entropy sums (approximation error)
    _, _, fent = gradient.pair_sums(X.astype(np.float64), 0.05)
    say(f"[quadtree] FIt entropy vs exact {rel_l2(fit['F_ent'], fent):.2e}, "
        f"interpolated {rel_l2(lt['F_ent'], fent):.2e}")
    assert rel_l2(fit["F_ent"], fent) <= 2e-2


def test_cost_with_quadtree_terms(api, ctx, grid_problem):
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = (np.random.default_rng(5).normal(size=(g.n, 2)) * 3).astype(np.float32)
    ex = gradient.cost_terms(X.astype(np.float64), P, CostParams())
    zi, _, _, lnv = oq.sums(X, theta=0.5, eps=0.05)
    Zex = gradient.pair_sums(X.astype(np.float64), 0.05)[0].sum()
    for name in ("BH-tsNET", "FIt-tsNET"):
        got = prob.cost(torch.tensor(X, device="cuda"), api.Params.variant(name)).cpu().numpy()[0]
        ent = -0.01 / (4.0 * g.n * g.n) * lnv.sum()
        assert abs(got[2] - ent) <= 1e-5 * abs(ent), name
        if name == "BH-tsNET":  # KL uses the quadtree Z (sum p = 1)
            kl = ex.kl[0] + np.log(zi.sum()) - np.log(Zex)
            assert abs(got[0] - kl) <= 1e-5 * abs(kl)
        say(f"[quadtree] cost {name}: {got}")


def test_batch_and_determinism(api, ctx):
    parts = [graphs.grid(12, 9), graphs.random_recursive_tree(500, 3),
             graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)),
             graphs.sbm([150, 150], 0.05, 0.01, 6)]
    b = graphs.concat_graphs(parts)
    P = affinities.build_P(b.indptr, b.indices, 10.0, seed=1, graph_offsets=b.graph_offsets)
    prob = _upload(api, ctx, P, b.graph_offsets)
    n = int(b.graph_offsets[-1])
    X = (np.random.default_rng(6).normal(size=(n, 2)) * 3).astype(np.float32)
    prm = api.Params.variant("BH-tsNET")
    got = _terms(api, prob, X, prm)
    ref = oq.sums(X, theta=0.5, eps=0.05, graph_offsets=b.graph_offsets)
    _check_qt(got, ref, "batch")
    off = b.graph_offsets
    for gi in range(len(parts)):
        zg = ref[0][off[gi]:off[gi + 1]].sum()
        assert abs(got["Z"][gi] - zg) <= 1e-5 * max(zg, 1e-30)
    again = _terms(api, prob, X, prm)
    for k in ("G", "F_rep", "F_ent", "Z_i", "Z"):
        assert np.array_equal(again[k], got[k]), k


def test_bad_theta_rejected(api, ctx, grid_problem):
    from paper_2509_19785_amd._lib import TsnetError
    g, P = grid_problem
    prob = _upload(api, ctx, P)
    X = torch.zeros((g.n, 2), device="cuda")
    for th in (0.0, 0.75):
        with pytest.raises(TsnetError):
            prob.grad(X, api.Params.variant("BH-tsNET", theta=th))


def test_ba1m_sampled(api, ctx):
    g = graphs.workload_ba1m()
    prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, seed=3)
    rng = np.random.default_rng(7)
    X = (rng.normal(size=(g.n, 2)) * np.where(rng.random((g.n, 1)) < 0.5, 2.0, 20.0)).astype(np.float32)
    got = _terms(api, prob, X, api.Params.variant("BH-tsNET"))
    rows = np.sort(rng.choice(g.n, 48, replace=False))
    say(f"[quadtree] BA n={g.n}: oracle tree and {len(rows)} sampled points")
    ref = oq.sums(X, theta=0.5, eps=0.05, rows=rows)
    sub = {k: got[k][rows] for k in ("F_rep", "F_ent", "Z_i")}
    _check_qt(sub, tuple(r[rows] for r in ref), "BA 1e6 sampled")
