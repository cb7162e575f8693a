"""The allocation-free FP64 direct gradient (tsnet_grad_direct_f64_static)
against the allocating entry point (tsnet_grad_direct_f64), through the C ABI.

Both run the same kernels in the same order, so G, Z and the per-row terms
must agree bit for bit. Two calls in a row on the static scratch, the second
with a smaller input (fewer vertices and a row subset), then a call past the
scratch's limit, which must fail on the host with TSNET_EINVAL.
"""
import ctypes

import numpy as np
import pytest

from helpers import say
from oracle import affinities
from synth import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _direct(fn, ctx, prob, X, prm, rows=None):
    n = prob.n
    nr = n if rows is None else int(rows.numel())
    G = torch.empty((nr, 2), dtype=torch.float64, device="cuda")
    Z = torch.empty(prob.num_graphs, dtype=torch.float64, device="cuda")
    T = torch.empty((nr, 7), dtype=torch.float64, device="cuda")
    c = prm.to_c()
    rc = fn(ctx.handle, prob.handle, X.data_ptr(), ctypes.byref(c), G.data_ptr(), Z.data_ptr(),
            None if rows is None else rows.data_ptr(), nr, T.data_ptr(),
            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return rc, G, Z, T


def test_static_direct_matches_allocating():
    from paper_2509_19785_amd import _lib, api
    lib = _lib.lib
    ctx = api.Context(0)
    prm = api.Params()
    cases = []
    g1 = graphs.sbm([700, 900, 1433], 0.012, 4e-4, 11)
    P1 = affinities.build_P(g1.indptr, g1.indices, 15.0, seed=3)
    X1 = graphs.bulk_with_far_points(g1.n, 2, n_far=30).astype(np.float64)
    cases.append(("SBM n=3033, every row", P1, X1, None))
    g2 = graphs.grid(20, 30)
    P2 = affinities.build_P(g2.indptr, g2.indices, 10.0, seed=1)
    X2 = graphs.initial_layout(g2.n, 5, std=2.0).astype(np.float64)
    rows2 = np.array([0, 7, 599, 300, 12, 7], dtype=np.int32)
    cases.append(("grid 20 x 30, 6 rows", P2, X2, rows2))
    for label, P, X, rows in cases:
        say(f"[no-alloc] {label}")
        prob = api.Problem.from_host(ctx, P.rowptr, P.col, P.val.astype(np.float32))
        Xt = torch.tensor(X, device="cuda")
        rt = None if rows is None else torch.tensor(rows, device="cuda")
        rc_s, Gs, Zs, Ts = _direct(lib.tsnet_grad_direct_f64_static, ctx, prob, Xt, prm, rt)
        assert rc_s == _lib.TSNET_OK, lib.tsnet_last_error()
        rc_a, Ga, Za, Ta = _direct(lib.tsnet_grad_direct_f64, ctx, prob, Xt, prm, rt)
        assert rc_a == _lib.TSNET_OK, lib.tsnet_last_error()
        say(f"   max |dG| {float((Gs - Ga).abs().max()):.3e}, Z {Zs.item():.17g} / {Za.item():.17g}")
        assert torch.equal(Gs, Ga) and torch.equal(Zs, Za) and torch.equal(Ts, Ta)
        assert bool(torch.isfinite(Gs).all())
        prob.free()
    # past the limit: 5 (n + nrows) > 2^21 is refused before anything runs
    prob = api.Problem.from_host(ctx, P2.rowptr, P2.col, P2.val.astype(np.float32))
    big = torch.zeros(420_000, dtype=torch.int32, device="cuda")
    rc, _, _, _ = _direct(lib.tsnet_grad_direct_f64_static, ctx, prob,
                          torch.tensor(X2, device="cuda"), prm, big)
    assert rc == _lib.TSNET_EINVAL
    assert b"static scratch" in lib.tsnet_last_error()
    prob.free()
    ctx.close()
