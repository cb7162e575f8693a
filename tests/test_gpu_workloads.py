"""GPU parity at the sizes of the benchmark workloads.

Where the oracle cannot run the whole workload, outputs are checked on samples
it computes one by one, or through properties that hold at any size:

* SBM n = 2e4 (20 blocks of 1000): P bit-exact in support against the oracle's
  build, and the whole gradient against the exact O(n^2) oracle gradient.
* Barabasi-Albert n = 1e6 (m0 = 4, seed 3), built on the GPU in the launch
  configuration of the benchmark:
  - the selection and hop distances of 64 sampled rows are bit-exact against
    the oracle's partial BFS;
  - beta of those rows hits ln u;
  - P[i, j] for every j the oracle selects from i equals
    (p_{j|i} + p_{i|j}) / 2n from the oracle's conditional rows;
  - every stored entry of a sampled row is justified by a selection;
  - P is symmetric on those rows and sums to 1;
  - the repulsive and entropy sums and Z_i of 256 sampled vertices match the
    oracle's exact pair sums, and Z equals the sum of Z_i.
* A random sparse P with n = 1e6 and hub rows (the tiled attraction at full
  size): F_attr of 256 sampled rows against the oracle, and the tiled and row
  layouts against each other on all rows.
* The mixed batch of 256 graphs (n from 500 to 50000) in one problem: P rows
  and the gradient of sampled graphs against the oracle run on those graphs.
"""
import math

import numpy as np
import pytest

from helpers import P32, rel_l2, say
from oracle import affinities, gradient, interp, perplexity
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


def _ulps(a32, b64):
    ai = np.asarray(a32, np.float32).view(np.int32).astype(np.int64)
    bi = np.asarray(b64).astype(np.float32).view(np.int32).astype(np.int64)
    return np.abs(ai - bi)


def _terms(prob, X, prm):
    out = prob.grad_terms(X, prm)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


# --------------------------------------------------------------------- SBM 20k
def test_sbm20k_build_and_gradient(api, ctx):
    g = graphs.workload_sbm20k()
    say(f"[workload] SBM n={g.n} m={g.m}: oracle P")
    oP = affinities.build_P(g.indptr, g.indices, 40.0, seed=1)
    prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, seed=1)
    got = prob.export()
    assert np.array_equal(got["rowptr"], oP.rowptr)
    assert np.array_equal(got["col"], oP.col)
    assert _ulps(got["val"], oP.val).max() <= 4
    X32 = graphs.initial_layout(g.n, 1, std=3.0)
    t = _terms(prob, torch.tensor(X32, device="cuda"), api.Params())
    ex = gradient.grad_terms(X32.astype(np.float64), oP, CostParams())
    e = rel_l2(t["G"], ex.G)
    say(f"   gradient rel L2 {e:.2e}, Z {t['Z'][0]:.6e} vs {ex.Z[0]:.6e}")
    assert e <= 1e-3
    assert abs(t["Z"][0] - ex.Z[0]) <= 1e-4 * ex.Z[0]


# --------------------------------------------------------------------- BA 1e6
@pytest.fixture(scope="module")
def ba1m(api, ctx):
    g = graphs.workload_ba1m()
    say(f"[workload] BA n={g.n} m={g.m}: GPU build")
    prob = api.Problem.build(ctx, g.indptr, g.indices, 40.0, seed=3)
    return g, prob


def test_ba1m_build_sampled_rows(api, ba1m):
    g, prob = ba1m
    got = prob.export(conditional=True)
    n, k = g.n, prob.k
    rng = np.random.default_rng(3)
    rows = np.concatenate([np.arange(4), rng.choice(n, 60, replace=False)])  # 4 hubs + random
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(g.indptr, g.indices, 40.0, seed=3,
                                                                  rows=rows)
    u = 40.0
    for r, i in enumerate(rows):
        a, b = int(ptr[r]), int(ptr[r + 1])
        L = b - a
        assert int(got["cond_len"][i]) == L
        assert np.array_equal(got["cond_nbr"][i, :L], nbr[a:b]), i
        assert np.array_equal(got["cond_dist"][i, :L].astype(np.int32), dist[a:b]), i
        assert int(got["status"][i]) == int(status[r])
        if status[r] == perplexity.STATUS_OK:
            lv, ct = perplexity.level_histogram(dist[a:b])
            deltas = lv.astype(float) ** 2 - float(lv[0]) ** 2
            assert abs(perplexity.entropy_of_beta(got["beta"][i], deltas, ct) - math.log(u)) <= 1e-12
    rp, col, val = got["rowptr"], got["col"], got["val"]
    say(f"   nnz={prob.nnz} sum P={float(val.astype(np.float64).sum()):.9f}")
    assert abs(float(val.astype(np.float64).sum()) - 1.0) <= 1e-5
    # values of the selected pairs of 16 non-hub rows, from the oracle's conditional rows
    for r, i in enumerate(rows[4:20], start=4):
        a, b = int(ptr[r]), int(ptr[r + 1])
        js = nbr[a:b].astype(np.int64)
        jp, jn, jd, jpv, _, _ = affinities.conditional_rows(g.indptr, g.indices, 40.0, seed=3, rows=js)
        row_c = col[rp[i]:rp[i + 1]]
        row_v = val[rp[i]:rp[i + 1]]
        for q, j in enumerate(js):
            sel = jn[jp[q]:jp[q + 1]]
            hit = np.nonzero(sel == i)[0]
            p_ij = (p[a + q] + (jpv[jp[q] + hit[0]] if hit.size else 0.0)) / (2.0 * n)
            pos = np.searchsorted(row_c, j)
            assert pos < row_c.size and row_c[pos] == j, (i, j)
            assert _ulps(row_v[pos], p_ij)[()] <= 4, (i, j, row_v[pos], p_ij)
        # every stored entry is a selection of i or of j, and P is symmetric there
        extra = np.setdiff1d(row_c, js)
        if extra.size:
            ep, en_, _, _, _, _ = affinities.conditional_rows(g.indptr, g.indices, 40.0, seed=3,
                                                              rows=extra)
            for q in range(extra.size):
                assert i in en_[ep[q]:ep[q + 1]], (i, extra[q])
        for j, v in zip(row_c, row_v):
            rc = col[rp[j]:rp[j + 1]]
            pos = np.searchsorted(rc, i)
            assert pos < rc.size and rc[pos] == i and val[rp[j] + pos] == v


@pytest.mark.parametrize("std", [0.01, 8.0])
def test_ba1m_repulsion_sampled(api, ba1m, std):
    g, prob = ba1m
    X32 = graphs.initial_layout(g.n, 0, std=std)
    t = _terms(prob, torch.tensor(X32, device="cuda"), api.Params())
    rows = np.random.default_rng(5).choice(g.n, 256, replace=False)
    zi, frep, fent = gradient.pair_sums(X32.astype(np.float64), 0.05, rows=rows)
    e_rep = rel_l2(t["F_rep"][rows], frep)
    e_ent = rel_l2(t["F_ent"][rows], fent)
    e_zi = rel_l2(t["Z_i"][rows], zi)
    z_sum = float(t["Z_i"].astype(np.float64).sum())
    gi = prob.grid_info()
    say(f"[workload] BA 1e6 std={std} n_int={int(gi['n_intervals'][0])}: rep {e_rep:.2e} ent {e_ent:.2e}"
        f" Z_i {e_zi:.2e}; Z {t['Z'][0]:.6e} sum Z_i {z_sum:.6e}")
    assert e_rep <= 1e-3 and e_ent <= 1e-3 and e_zi <= 1e-3
    assert abs(t["Z"][0] - z_sum) <= 1e-5 * z_sum


def test_ba1m_bulk_with_far_points(api, ba1m):
    """The layout class of the benchmark descent: a dense bulk about a unit wide
    and ~100 far points out to tens of units that set the bounding box. Against
    the oracle: the far points and the grid; every vertex's interpolated sums
    (FP64 interpolation oracle); F_rep, F_ent, Z_i of 256 sampled vertices and
    the gradient of 16 of them against exact sums, each term within 1e-3."""
    g, prob = ba1m
    X32 = graphs.bulk_with_far_points(g.n, 3, n_far=100)
    X64 = X32.astype(np.float64)
    prm = api.Params()
    t = _terms(prob, torch.tensor(X32, device="cuda"), prm)
    gi = prob.grid_info()
    it = interp.interp_terms(X64, prm.eps_r, prm.interval_width, prm.min_intervals, prm.max_intervals)
    say(f"[workload] BA 1e6 bulk + far points: n_int {int(gi['n_intervals'][0])} (oracle "
        f"{it.grid.n_int}), far {int(gi['far_points'][0])} (oracle {int(it.far.sum())})")
    assert int(gi["n_intervals"][0]) == it.grid.n_int
    assert int(gi["far_points"][0]) == int(it.far.sum()) >= 100
    e_i = {k: rel_l2(t[k], getattr(it, k)) for k in ("F_rep", "F_ent", "Z_i")}
    say("   against the FP64 interpolation: " + " ".join(f"{k} {v:.2e}" for k, v in e_i.items()))
    assert max(e_i.values()) <= 2e-5
    # exact pair sums of sampled vertices: every far point and 156 others
    rng = np.random.default_rng(6)
    far_ids = np.nonzero(it.far)[0]
    rows = np.concatenate([far_ids, rng.choice(np.nonzero(~it.far)[0], 256 - far_ids.size, replace=False)])
    zi, frep, fent = gradient.pair_sums(X64, 0.05, rows=rows)
    e_rep = rel_l2(t["F_rep"][rows], frep)
    e_ent = rel_l2(t["F_ent"][rows], fent)
    e_zi = rel_l2(t["Z_i"][rows], zi)
    # the oracle's interpolated Z_i of the same rows, to vouch for its Z below
    e_zi_oracle = rel_l2(it.Z_i[rows], zi)
    say(f"   against exact sums of {rows.size} vertices: rep {e_rep:.2e} ent {e_ent:.2e} Z_i {e_zi:.2e}"
        f" (oracle interpolation Z_i {e_zi_oracle:.2e})")
    assert e_rep <= 1e-3 and e_ent <= 1e-3 and e_zi <= 1e-3
    assert e_zi_oracle <= 1e-6
    assert abs(t["Z"][0] - it.Z) <= 1e-5 * it.Z
    # the gradient of 16 sampled rows whose P entries the oracle derives from
    # its own conditional rows (each entry (p_j|i + p_i|j) / 2n)
    got = prob.export()
    n = g.n
    Grows = rows[::16]
    ptr, nbr, dist, p, beta, status = affinities.conditional_rows(g.indptr, g.indices, 40.0, seed=3,
                                                                  rows=Grows)
    fa = np.zeros((Grows.size, 2))
    for r, i in enumerate(Grows):
        cols = got["col"][got["rowptr"][i]:got["rowptr"][i + 1]].astype(np.int64)
        sel = nbr[ptr[r]:ptr[r + 1]].astype(np.int64)
        assert np.isin(sel, cols).all(), i
        cp, cn, _, cpv, _, _ = affinities.conditional_rows(g.indptr, g.indices, 40.0, seed=3, rows=cols)
        vals = np.zeros(cols.size)
        for q, j in enumerate(cols):
            back = cn[cp[q]:cp[q + 1]]
            hit = np.nonzero(back == i)[0]
            fwd = np.nonzero(sel == j)[0]
            assert hit.size or fwd.size, (i, j)     # every stored entry is a selection
            vals[q] = ((p[ptr[r] + fwd[0]] if fwd.size else 0.0) +
                       (cpv[cp[q] + hit[0]] if hit.size else 0.0)) / (2.0 * n)
        d = X64[i] - X64[cols]
        w = 1.0 / (1.0 + (d ** 2).sum(1))
        fa[r] = ((vals * w)[:, None] * d).sum(0)
    k = np.arange(0, rows.size, 16)  # positions of Grows in rows
    Gx = 4.0 * (fa - frep[k] / it.Z) + 1.2 / n * X64[Grows] - 0.01 / n ** 2 * fent[k]
    e_G = rel_l2(t["G"][Grows], Gx)
    say(f"   gradient of {Grows.size} rows: rel L2 {e_G:.2e}")
    assert e_G <= 1e-3


# --------------------------------------------------------------------- random 1e6
def test_random1m_tiled_attraction(api, ctx):
    n = 1_000_000
    rowptr, col, val = graphs.random_affinity(n, 60.0, 11, hub_rows=8, hub_len=40000, empty_frac=0.01)
    say(f"[workload] random P n={n} nnz={col.size}")
    prob = api.Problem.from_host(ctx, rowptr, col, val.astype(np.float32))
    X = torch.tensor(graphs.initial_layout(n, 11, std=5.0), device="cuda")
    prm_t = api.Params(attract_layout=2, max_intervals=64)
    prm_r = api.Params(attract_layout=1, max_intervals=64)
    t = _terms(prob, X, prm_t)
    r = _terms(prob, X, prm_r)
    e_layouts = rel_l2(t["F_attr"], r["F_attr"])
    rows = np.concatenate([np.arange(8), np.random.default_rng(11).choice(n, 248, replace=False)])

    class _P:
        pass
    Pc = _P()
    Pc.rowptr, Pc.col, Pc.val = rowptr, col, val
    fa = gradient.attraction(X.cpu().numpy().astype(np.float64), rowptr, col, P32(Pc).val, rows=rows)
    e = rel_l2(t["F_attr"][rows], fa)
    say(f"   sampled F_attr rel L2 {e:.2e}; tiled vs rows {e_layouts:.2e}")
    assert e <= 1e-6 and e_layouts <= 1e-6


# --------------------------------------------------------------------- mixed batch
def _oracle_interp(args):
    """The oracle's interpolated sums of one graph (runs in a worker process)."""
    from oracle import interp as oi
    X64, eps = args
    it = oi.interp_terms(X64, eps)
    return it.F_rep, it.F_ent, it.Z_i, it.grid.n_int, int(it.far.sum())


def _oracle_graph_exact(args):
    """One graph of the batch: its P from the oracle's conditional rows (global
    ids, as the batch was built), then the exact gradient terms of sampled rows
    and the exact Z (runs in a worker process)."""
    from oracle import affinities as oa, gradient as og
    indptr, indices, a, e, X64, rows = args
    ng = e - a
    ptr, nbr, dist, p, beta, status = oa.conditional_rows(indptr, indices, 40.0, seed=4,
                                                          rows=np.arange(a, e))
    rp, cl, vl = oa.symmetrize(ng, ptr, nbr.astype(np.int64) - a, p, status,
                               np.array([0, ng], dtype=np.int64))
    zi, frep, fent = og.pair_sums(X64, 0.05, rows=rows)
    fa = og.attraction(X64, rp, cl, vl.astype(np.float32).astype(np.float64), rows=rows)
    Z = og.normaliser(X64)
    return rp, cl, vl, zi, frep, fent, fa, Z


def _pool(k):
    import multiprocessing as mp
    import os
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return mp.get_context("spawn").Pool(max(1, min(k, 16, usable)))


def test_mixed256_all_graphs(api, ctx):
    """The 256-graph batch at the default settings, one launch per stage for all
    graphs, on layouts of both classes (a dense bulk with far points in the
    even graphs, N(0, 2^2) in the odd ones): every graph's F_rep, F_ent and Z_i
    against the FP64 interpolation oracle, its grid and far points the
    oracle's; the gradient of the 5 largest graphs against the exact oracle on
    256 sampled rows each, with P from the oracle's conditional rows."""
    b = graphs.workload_mixed256()
    off = b.graph_offsets.astype(np.int64)
    sizes = np.diff(off)
    n = int(off[-1])
    say(f"[workload] mixed batch: {b.num_graphs} graphs, n={n}")
    prob = api.Problem.build(ctx, b.indptr, b.indices, 40.0, seed=4, graph_offsets=off)
    got = prob.export()
    X32 = np.empty((n, 2), np.float32)
    for g in range(b.num_graphs):
        a, e = int(off[g]), int(off[g + 1])
        X32[a:e] = (graphs.bulk_with_far_points(e - a, 40 + g, n_far=max(4, (e - a) // 500), r_min=5.0)
                    if g % 2 == 0 else graphs.initial_layout(e - a, 40 + g, std=2.0))
    prm = api.Params()
    t = _terms(prob, torch.tensor(X32, device="cuda"), prm)
    gi = prob.grid_info()
    X64 = X32.astype(np.float64)
    with _pool(16) as pool:
        res = pool.map(_oracle_interp, [(X64[off[g]:off[g + 1]], 0.05) for g in range(b.num_graphs)])
    worst = 0.0
    for g, (frep, fent, zi, nint, nfar) in enumerate(res):
        a, e = int(off[g]), int(off[g + 1])
        assert int(gi["n_intervals"][g]) == nint, g
        assert int(gi["far_points"][g]) == nfar, g
        assert (nfar > 0) == (g % 2 == 0), g
        err = max(rel_l2(t["F_rep"][a:e], frep), rel_l2(t["F_ent"][a:e], fent), rel_l2(t["Z_i"][a:e], zi))
        worst = max(worst, err)
        assert err <= 2e-5, (g, err)
        assert abs(t["Z"][g] - zi.sum()) <= 1e-5 * zi.sum(), g
    say(f"   every graph against the FP64 interpolation: worst term {worst:.2e}; far points "
        f"{int(gi['far_points'].sum())} in {int((gi['far_points'] > 0).sum())} graphs, "
        f"intervals {sorted(set(gi['n_intervals'].tolist()))}")
    big = np.argsort(sizes, kind="stable")[-5:]
    rng = np.random.default_rng(4)
    jobs = []
    for g in big:
        a, e = int(off[g]), int(off[g + 1])
        jobs.append((b.indptr, b.indices, a, e, X64[a:e], np.sort(rng.choice(e - a, 256, replace=False))))
    with _pool(5) as pool:
        ex = pool.map(_oracle_graph_exact, jobs)
    for g, job, (rp, cl, vl, zi, frep, fent, fa, Z) in zip(big, jobs, ex):
        a, e, rows = job[2], job[3], job[5]
        ng = e - a
        # P of the graph: support bit-exact, values within 4 ulp
        grp = got["rowptr"][a:e + 1] - got["rowptr"][a]
        assert np.array_equal(grp, rp)
        assert np.array_equal(got["col"][got["rowptr"][a]:got["rowptr"][e]] - a, cl)
        assert _ulps(got["val"][got["rowptr"][a]:got["rowptr"][e]], vl).max() <= 4
        Xg = X64[a:e]
        Gx = 4.0 * (fa - frep / Z) + 1.2 / ng * Xg[rows] - 0.01 / ng ** 2 * fent
        eg = rel_l2(t["G"][a + rows], Gx)
        e_terms = max(rel_l2(t["F_rep"][a + rows], frep), rel_l2(t["F_ent"][a + rows], fent),
                      rel_l2(t["Z_i"][a + rows], zi))
        say(f"   graph {g} ({b.kinds[g]}, n={ng}, far {int(gi['far_points'][g])}): gradient rel L2 {eg:.2e}, "
            f"terms {e_terms:.2e}, Z {abs(t['Z'][g] - Z) / Z:.2e}")
        assert eg <= 1e-3 and e_terms <= 1e-3
        assert abs(t["Z"][g] - Z) <= 1e-4 * Z
