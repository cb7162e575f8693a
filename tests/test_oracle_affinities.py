"""Pins for the oracle's Eq. (3) calibration and Eq. (2) symmetrisation (CPU only)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import affinities, perplexity
from synth import graphs


def _entropy_from_p(p):
    p = p[p > 0]
    return float(-np.sum(p * np.log(p)))


@pytest.mark.parametrize("u", [3.0, 7.5, 12.0, 40.0])
def test_calibrated_rows_reach_perplexity(u):
    g = graphs.rgg(600, graphs.rgg_radius_for_degree(600, 8), 3)
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(g.indptr, g.indices, u, seed=1)
    ok = 0
    for i in range(g.n):
        a, b = ptr[i], ptr[i + 1]
        if status[i] == perplexity.STATUS_OK:
            ok += 1
            row = p[a:b]
            assert abs(row.sum() - 1.0) < 1e-12
            # perplexity from the definition 2^{-sum p log2 p} of Sec. 2.1
            h2 = -np.sum(row[row > 0] * np.log2(row[row > 0]))
            assert abs(2.0 ** h2 - u) <= 1e-9 * u
            # Eq. (3) with the unshifted squared distances
            d2 = dist[a:b].astype(float) ** 2
            e = np.exp(-beta[i] * d2)
            assert np.allclose(row, e / e.sum(), rtol=1e-12, atol=0)
    assert ok > 0


def test_beta_matches_library_root_finder():
    g = graphs.barabasi_albert(800, 4, 2)
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(g.indptr, g.indices, 40.0, seed=3)
    checked = 0
    for i in range(0, g.n, 5):
        if status[i] != perplexity.STATUS_OK:
            continue
        lv, ct = perplexity.level_histogram(dist[ptr[i]:ptr[i + 1]])
        d2 = dist[ptr[i]:ptr[i + 1]].astype(float) ** 2

        def f(b):
            e = np.exp(-b * (d2 - d2.min()))
            q = e / e.sum()
            return _entropy_from_p(q) - math.log(40.0)

        hi = 1.0
        while f(hi) > 0:
            hi *= 2
        root = brentq(f, 0.0, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        assert abs(beta[i] - root) <= 1e-9 * root
        checked += 1
    assert checked > 10


def test_saturated_rows_closed_forms():
    # K5: every row has 4 neighbours on one level -> LOW, p = 1/4
    iu, ju = np.triu_indices(5, 1)
    k5 = graphs.csr_from_edges(5, iu, ju)
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(k5.indptr, k5.indices, 40.0)
    assert np.all(status == perplexity.STATUS_LOW) and np.allclose(p, 0.25)
    # broom: hub 0 with 50 leaves, leaf 1 carries a pendant vertex 51.
    u = np.concatenate([np.zeros(50, np.int64), [1]])
    v = np.concatenate([np.arange(1, 51), [51]])
    broom = graphs.csr_from_edges(52, u, v)
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(broom.indptr, broom.indices, 40.0)
    row = slice(ptr[0], ptr[1])
    assert status[0] == perplexity.STATUS_HIGH and math.isinf(beta[0])
    assert np.all(p[row][dist[row] == 1] == 1.0 / 50) and np.all(p[row][dist[row] == 2] == 0.0)
    # path P3, endpoint: 2 reachable vertices <= u -> LOW, p = 1/2
    p3 = graphs.csr_from_edges(3, np.array([0, 1]), np.array([1, 2]))
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(p3.indptr, p3.indices, 40.0)
    assert status[0] == perplexity.STATUS_LOW and np.allclose(p[ptr[0]:ptr[1]], 0.5)


def _dense_P(oP, n):
    D = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(oP.rowptr))
    D[rows, oP.col] = oP.val
    return D


def test_P_invariants_and_brute_force():
    g = graphs.sbm([30, 40], 0.2, 0.02, 4)
    oP = affinities.build_P(g.indptr, g.indices, 5.0, seed=2)
    n = g.n
    D = _dense_P(oP, n)
    assert np.array_equal(D, D.T)
    assert np.all(D >= 0)
    assert abs(D.sum() - 1.0) < 1e-14
    for i in range(n):
        cols = oP.col[oP.rowptr[i]:oP.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    # brute force: dense conditional matrix, Eq. (2) with n non-empty rows
    C = np.zeros((n, n))
    for i in range(n):
        a, b = oP.cond_ptr[i], oP.cond_ptr[i + 1]
        C[i, oP.cond_nbr[a:b]] = oP.cond_p[a:b]
    nonempty = int(np.sum(oP.status != 3))
    assert np.allclose(D, (C + C.T) / (2 * nonempty), rtol=1e-15, atol=0)
    g2 = graphs.grid(6, 7)
    p2 = affinities.build_P(g2.indptr, g2.indices, 5.0, seed=2)
    C2 = np.zeros((42, 42))
    for i in range(42):
        a, b = p2.cond_ptr[i], p2.cond_ptr[i + 1]
        C2[i, p2.cond_nbr[a:b]] = p2.cond_p[a:b]
    assert np.allclose(_dense_P(p2, 42), (C2 + C2.T) / (2 * 42), rtol=1e-15, atol=0)
    # the support is the union of selected pairs and their transposes
    sel = np.zeros((n, n), dtype=bool)
    for i in range(n):
        sel[i, oP.cond_nbr[oP.cond_ptr[i]:oP.cond_ptr[i + 1]]] = True
    want = sel | sel.T
    got = np.zeros((n, n), dtype=bool)
    got[np.repeat(np.arange(n), np.diff(oP.rowptr)), oP.col] = True
    assert np.array_equal(got, want)


def test_isolated_vertices_and_batches():
    a = graphs.csr_from_edges(6, np.array([0, 1, 2]), np.array([1, 2, 3]))   # 4, 5 isolated
    b = graphs.grid(3, 4)
    batch = graphs.concat_graphs([a, b])
    oP = affinities.build_P(batch.indptr, batch.indices, 2.0, seed=5,
                            graph_offsets=batch.graph_offsets)
    D = _dense_P(oP, batch.indptr.shape[0] - 1)
    assert abs(D[:6, :6].sum() - 1.0) < 1e-14 and abs(D[6:, 6:].sum() - 1.0) < 1e-14
    assert D[:6, 6:].sum() == 0 and D[4].sum() == 0 and D[5].sum() == 0
    assert list(oP.status[4:6]) == [3, 3]
    # each block equals the graph built alone
    pa = affinities.build_P(a.indptr, a.indices, 2.0, seed=5)
    pb = affinities.build_P(b.indptr, b.indices, 2.0, seed=5)
    assert np.array_equal(D[:6, :6], _dense_P(pa, 6))
    # tie keys use global ids, so only the support-free grid rows (no cut) compare
    Db = _dense_P(pb, 12)
    assert np.allclose(D[6:, 6:].sum(), Db.sum())
