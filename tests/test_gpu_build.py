"""GPU parity of tsnet_build_P (partial BFS, Eq. 3 calibration, Eq. 2 symmetrisation).

Bar: selected neighbours, hop distances and row lengths bit-exact; row status
exact; beta such that the oracle's entropy at the GPU's beta is ln u within
1e-12 (the bisection decision near the root may flip on the last ulp);
support of P exact; values of P within 4 FP32 ulp of the oracle's FP64 values.
"""
import math

import numpy as np
import pytest

from helpers import say, ulp_diff
from oracle import affinities, perplexity
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


def _build(api, ctx, g, u, k=0, seed=0, mode="hash", goff=None):
    return api.Problem.build(ctx, g.indptr, g.indices, u, k=k, seed=seed, tie_mode=mode,
                             graph_offsets=goff)


def compare(api, ctx, g, u, k=0, seed=0, mode="hash", goff=None, label=""):
    say(f"[build parity] {label} n={g.indptr.shape[0] - 1} u={u} k={k} mode={mode}")
    prob = _build(api, ctx, g, u, k, seed, mode, goff)
    got = prob.export(conditional=True)
    oP = affinities.build_P(g.indptr, g.indices, u, k=k, seed=seed, tie_mode=mode, graph_offsets=goff)
    n = g.indptr.shape[0] - 1
    kk = prob.k
    # conditional rows, bit-exact
    olen = np.diff(oP.cond_ptr)
    assert np.array_equal(got["cond_len"], olen)
    for i in range(n):
        a, b = oP.cond_ptr[i], oP.cond_ptr[i + 1]
        L = b - a
        assert np.array_equal(got["cond_nbr"][i, :L], oP.cond_nbr[a:b]), i
        assert np.array_equal(got["cond_dist"][i, :L].astype(np.int32), oP.cond_dist[a:b]), i
    assert np.array_equal(got["status"], oP.status)
    # beta: the oracle's entropy at the GPU's beta hits ln u
    for i in np.nonzero(oP.status == perplexity.STATUS_OK)[0]:
        lv, ct = perplexity.level_histogram(oP.cond_dist[oP.cond_ptr[i]:oP.cond_ptr[i + 1]])
        deltas = lv.astype(float) ** 2 - float(lv[0]) ** 2
        h = perplexity.entropy_of_beta(got["beta"][i], deltas, ct)
        assert abs(h - math.log(u)) <= 1e-12, (i, h)
        assert abs(got["beta"][i] - oP.beta[i]) <= 1e-6 * oP.beta[i]
    assert np.all(np.isinf(got["beta"][oP.status == perplexity.STATUS_HIGH]))
    # symmetric P
    assert np.array_equal(got["rowptr"], oP.rowptr)
    assert np.array_equal(got["col"], oP.col)
    ud = ulp_diff(got["val"], oP.val)
    say(f"   nnz={prob.nnz} max ulp={int(ud.max()) if ud.size else 0} status={np.bincount(oP.status, minlength=4)}")
    assert ud.size == 0 or ud.max() <= 4
    return prob, got, oP


def test_grid32_id_ties(api, ctx):
    compare(api, ctx, graphs.workload_grid32(), 40.0, mode="id", label="grid32")


def test_grid32_hash_ties(api, ctx):
    compare(api, ctx, graphs.workload_grid32(), 40.0, seed=123, label="grid32")


def test_ba_hubs(api, ctx):
    # heavy-tailed degrees: HIGH rows (degree > u), long candidate lists at hubs
    compare(api, ctx, graphs.barabasi_albert(3000, 4, 3), 40.0, seed=3, label="BA 3000")


def test_sbm_with_isolated(api, ctx):
    g = graphs.sbm([400, 500, 357], 0.01, 1e-3, 5)
    assert (g.degrees() == 0).any()
    compare(api, ctx, g, 12.0, seed=9, label="sbm isolated")


def test_tree_many_levels(api, ctx):
    compare(api, ctx, graphs.random_recursive_tree(2500, 4), 40.0, seed=1, label="tree")


def test_path_long_levels(api, ctx):
    n = 700
    g = graphs.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    compare(api, ctx, g, 50.0, label="path")  # 150 levels of one vertex each


@pytest.mark.parametrize("k", [7, 200, 600])
def test_other_k(api, ctx, k):
    g = graphs.rgg(2000, graphs.rgg_radius_for_degree(2000, 9.0), 6)
    compare(api, ctx, g, k / 3.0, k=k, seed=2, label=f"rgg k={k}")


def test_batch(api, ctx):
    parts = [graphs.grid(20, 25), graphs.barabasi_albert(800, 3, 1), graphs.random_recursive_tree(600, 2),
             graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64))]
    b = graphs.concat_graphs(parts)
    compare(api, ctx, b, 10.0, seed=77, goff=b.graph_offsets, label="batch of 4")


def test_deterministic(api, ctx):
    g = graphs.barabasi_albert(5000, 4, 8)
    a = _build(api, ctx, g, 40.0, seed=5).export(conditional=True)
    b = _build(api, ctx, g, 40.0, seed=5).export(conditional=True)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_invalid_csr_rejected(api, ctx):
    from paper_2509_19785_amd._lib import TsnetError
    g = graphs.grid(4, 4)
    bad_cases = []
    ix = g.indices.copy()
    ix[0], ix[1] = ix[1], ix[0]                      # row 0 not ascending
    bad_cases.append((g.indptr, ix, "ascending"))
    ix = g.indices.copy()
    ix[0] = 0                                         # self loop in row 0
    bad_cases.append((g.indptr, ix, "self loop"))
    ix = g.indices.copy()
    ix[-1] = 99                                       # out of range
    bad_cases.append((g.indptr, ix, "out of range"))
    one_way = graphs.csr_from_edges(4, np.array([0]), np.array([1]))
    ip = one_way.indptr.copy()
    ip[2:] -= 1                                       # drop the arc 1 -> 0
    bad_cases.append((ip, np.array([1], np.int32), "symmetric"))
    ip = g.indptr.copy()
    ip[3] = ip[2] - 1                                 # decreasing row pointer
    bad_cases.append((ip, g.indices, "row pointers"))
    for ip, ix, why in bad_cases:
        with pytest.raises(TsnetError) as ei:
            api.Problem.build(ctx, ip, ix, 2.0)
        assert ei.value.code == -1, why
