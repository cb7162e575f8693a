"""GPU checks of the staged descent (tsnet_run) and of full-P tsNET at small n.

* tsnet_run enqueues the same kernels in the same order as calling
  tsnet_grad and tsnet_step per iteration, so its layout, update, gains,
  gradient and Z equal that loop's bit for bit, also across stages that
  switch between L-tsNET and BH-tsNET; the stage order matters; a stage of
  zero iterations changes nothing; a bad stage is named in the error.
* Full P (the original tsNET's affinities over every other vertex): the
  partial BFS with k = n - 1 reaches the whole component, so its support is
  every pair and is compared bit for bit with the oracle's (values within
  4 ulp), on the 32 x 32 grid (k = 1023) and a tree. On that P the FP64
  direct gradient, the exact O(n^2) gradient of tsNET, agrees with the
  oracle's to 1e-12.
"""
import numpy as np
import pytest

from helpers import P32, rel_l2, say, ulp_diff
from oracle import affinities, gradient
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
def grid_problem(api, ctx):
    g = graphs.workload_grid32()
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=0)
    return g, api.Problem.from_host(ctx, P.rowptr, P.col, P.val.astype(np.float32))


def _state(g, seed):
    X = torch.tensor(graphs.initial_layout(g.n, seed), device="cuda")
    return X, torch.zeros_like(X), torch.ones_like(X), torch.empty_like(X), torch.empty(1, dtype=torch.float64, device="cuda")


def _schedule(api):
    return [(12, api.Params(lambda_c=1.2, lambda_r=0.0)),
            (6, api.Params.variant("BH-tsNET", lambda_c=0.01, lambda_r=0.01)),
            (0, api.Params(lambda_c=7.0)),
            (8, api.Params(lambda_c=0.01, lambda_r=0.01))]


def test_run_equals_per_call_loop(api, ctx, grid_problem):
    g, prob = grid_problem
    sp = api.StepParams()
    X, U, Ga, G, Z = _state(g, 1)
    X2, U2, Ga2, G2, Z2 = (t.clone() for t in (X, U, Ga, G, Z))
    prob.run(X, U, Ga, G, _schedule(api), first_iter=240, sp=sp, Z=Z)
    it = 240
    for iters, prm in _schedule(api):
        for _ in range(iters):
            prob.grad(X2, prm, G=G2, Z=Z2)
            prob.step(X2, U2, Ga2, G2, it, sp)
            it += 1
    torch.cuda.synchronize()
    for a, b, name in ((X, X2, "X"), (U, U2, "update"), (Ga, Ga2, "gains"), (G, G2, "G"), (Z, Z2, "Z")):
        assert torch.equal(a, b), name
    say(f"[run] 26 iterations over 4 stages (240..265) equal the per-call loop; |X| {float(X.norm()):.4f}")


def test_stage_order_and_empty_stages(api, ctx, grid_problem):
    g, prob = grid_problem
    sched = _schedule(api)
    X, U, Ga, G, Z = _state(g, 2)
    Xb, Ub, Gab, Gb, Zb = (t.clone() for t in (X, U, Ga, G, Z))
    prob.run(X, U, Ga, G, sched)
    prob.run(Xb, Ub, Gab, Gb, [sched[3], sched[1], sched[0]])
    torch.cuda.synchronize()
    assert not torch.equal(X, Xb)
    X0 = X.clone()
    prob.run(X, U, Ga, G, [(0, api.Params()), (0, api.Params.variant("BH-tsNET"))])
    torch.cuda.synchronize()
    assert torch.equal(X, X0)


def test_bad_stage_rejected(api, ctx, grid_problem):
    from paper_2509_19785_amd import _lib
    from paper_2509_19785_amd._lib import TsnetError
    g, prob = grid_problem
    X, U, Ga, G, Z = _state(g, 3)
    X0 = X.clone()
    with pytest.raises(TsnetError, match="stage 1"):
        prob.run(X, U, Ga, G, [(5, api.Params()), (5, api.Params.variant("BH-tsNET", theta=0.9))])
    with pytest.raises(TsnetError):
        prob.run(X, U, Ga, G, [(-1, api.Params())])
    torch.cuda.synchronize()
    assert torch.equal(X, X0)  # nothing ran


@pytest.mark.parametrize("which", ["grid32", "tree"])
def test_full_P_and_exact_gradient(api, ctx, which):
    g = graphs.workload_grid32() if which == "grid32" else graphs.random_recursive_tree(700, 5)
    k = g.n - 1
    prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, k=k, seed=4)
    ex = prob.export()
    ref = affinities.build_P(g.indptr, g.indices, 40.0, k=k, seed=4)
    assert np.array_equal(ex["rowptr"], ref.rowptr) and np.array_equal(ex["col"], ref.col)
    assert np.all(np.diff(ex["rowptr"]) == g.n - 1)          # every other vertex
    ulp = ulp_diff(ex["val"], ref.val)
    assert ulp.max() <= 4
    X = graphs.initial_layout(g.n, 9, std=1.0).astype(np.float64)
    Gd, Zd = prob.grad_direct_f64(torch.tensor(X, device="cuda"))
    torch.cuda.synchronize()
    want = gradient.grad_terms(X, P32(ref), CostParams())
    assert abs(Zd.item() - want.Z[0]) <= 1e-12 * want.Z[0]
    assert rel_l2(Gd.cpu().numpy(), want.G) <= 1e-12
    say(f"[full P] {which}: n={g.n} k={k} nnz={len(ex['col'])}, max {ulp.max():.0f} ulp")
