"""The cost as a torch.autograd.Function, on the random geometric graph n = 1e5.

Backward (the gradient kernel) is checked against central finite differences
of the FP64 oracle cost on 64 random coordinates (seed 2), and forward against
the oracle cost. P and the exact normaliser Z come from the oracle. Layouts:
the initial N(0, 1e-4) layout and a spread layout N(0, 10^2) (span about 90,
512 intervals).
Tolerances: the 64 backward values against the finite differences 1e-3
relative L2 (the gradient contract); the forward cost 1e-4 relative.
"""
import multiprocessing as mp

import numpy as np
import pytest

from helpers import rel_l2, say
from oracle import affinities, gradient
from oracle.gradient import CostParams
from synth import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_X = None


def _z_rows(rows):
    return gradient.normaliser(_X, rows=rows)


def _exact_Z(X):
    """Exact FP64 Z = sum_{i != j} w_ij from the oracle, rows split over processes."""
    global _X
    _X = X
    n = X.shape[0]
    procs = max(1, min(8, mp.cpu_count()))   # forked workers stay well under the per-GPU process limit
    chunks = np.array_split(np.arange(n), procs * 4)
    with mp.get_context("fork").Pool(procs) as pool:
        return float(sum(pool.map(_z_rows, chunks)))


@pytest.fixture(scope="module")
def rgg():
    g = graphs.workload_rgg100k()
    say(f"[autograd] oracle P for RGG n={g.n} m={g.m} (CPU, about a minute)")
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=2)
    return g, P


@pytest.fixture(scope="module")
def api():
    from paper_2509_19785_amd import api as a
    return a


@pytest.mark.parametrize("std", [0.01, 10.0])
def test_backward_matches_finite_differences(api, rgg, std):
    from paper_2509_19785_amd.autograd import tsnet_cost
    g, P = rgg
    ctx = api.Context(0)
    prob = api.Problem.from_host(ctx, P.rowptr, P.col, P.val.astype(np.float32))
    X32 = graphs.initial_layout(g.n, 2, std=std)
    X = torch.tensor(X32, device="cuda", requires_grad=True)
    prm = api.Params()
    say(f"[autograd] forward/backward std={std}")
    c = tsnet_cost(X, prob, prm)
    c.backward()
    grad = X.grad.cpu().numpy().astype(np.float64)
    assert X.grad.dtype == torch.float32 and X.grad.shape == X.shape

    X64 = X32.astype(np.float64)
    Z = _exact_Z(X64)
    cp = CostParams()
    rng = np.random.default_rng(2)
    idx = rng.choice(g.n * 2, size=64, replace=False)
    scale = float(np.abs(X64).max())
    h = 1e-4 * scale
    fd = np.array([gradient.fd_delta_cost(X64, P, cp, int(q // 2), int(q % 2), h, Z) / (2 * h)
                   for q in idx])
    got = grad[idx // 2, idx % 2]
    err = rel_l2(got, fd)
    say(f"   64 coordinates: backward vs FD rel L2 {err:.2e} (|fd| {np.linalg.norm(fd):.3e})")
    assert err <= 1e-3

    # forward: the value of tsnet_cost (its parity with the oracle cost is tested on grid32)
    assert float(c.item()) == float(prob.cost(X.detach(), prm)[:, 3].sum().item())
    ctx.close()


def test_forward_matches_oracle_cost(api):
    from paper_2509_19785_amd.autograd import tsnet_cost
    g = graphs.workload_grid32()
    P = affinities.build_P(g.indptr, g.indices, 40.0, seed=0)
    ctx = api.Context(0)
    prob = api.Problem.from_host(ctx, P.rowptr, P.col, P.val.astype(np.float32))
    X32 = graphs.initial_layout(g.n, 3, std=2.0)
    X = torch.tensor(X32, device="cuda", requires_grad=True)
    c = tsnet_cost(X, prob)
    c.backward()
    ex = gradient.cost_terms(X32.astype(np.float64), P, CostParams())
    exg = gradient.grad_terms(X32.astype(np.float64), P, CostParams()).G
    say(f"[autograd] grid32 cost {c.item():.6e} oracle {ex.total[0]:.6e}")
    assert abs(float(c.item()) - float(ex.total[0])) <= 1e-4 * abs(float(ex.total[0]))
    assert rel_l2(X.grad.cpu().numpy(), exg) <= 1e-3
    ctx.close()
