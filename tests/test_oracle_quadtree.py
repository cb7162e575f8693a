"""Pins of the oracle's quadtree (Barnes-Hut) sums (no GPU).

* With theta near 0 no inner node is a summary and every pair is summed one by
  one: the sums equal the exact all-pairs sums of ``gradient.pair_sums`` and a
  direct sum of ln(eps + r^2).
* Tree invariants: children partition their parent's range in code order,
  counts add up, leaves hold one point or sit at the deepest level (32),
  centres of mass are means; a layout whose bulk covers a tiny corner of the
  square (a few far points) still gets a leaf per distinct point.
* A single point facing a far cluster sees the cluster as one summary at its
  centre of mass (closed form).
* The error against the exact sums shrinks with theta; coincident points;
  a batch gives every graph its sums alone; theta out of range is rejected.
"""
import numpy as np
import pytest

from oracle import gradient, quadtree


def _walk(node, out):
    out.append(node)
    for c in node.children:
        _walk(c, out)
    return out


def test_tiny_theta_is_exact():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(120, 2)).astype(np.float32)
    zi, frep, fent, lnv = quadtree.sums(X, theta=1e-9, eps=0.05)
    z2, r2, e2 = gradient.pair_sums(X.astype(np.float64), 0.05)
    assert np.allclose(zi, z2, rtol=1e-13, atol=0)
    assert np.allclose(frep, r2, rtol=1e-12, atol=1e-15)
    assert np.allclose(fent, e2, rtol=1e-12, atol=1e-15)
    X64 = X.astype(np.float64)
    d = X64[:, None, :] - X64[None, :, :]
    L = np.log(0.05 + (d ** 2).sum(-1))
    np.fill_diagonal(L, 0.0)
    assert np.allclose(lnv, L.sum(1), rtol=1e-12)


def test_tree_invariants():
    rng = np.random.default_rng(1)
    X = (rng.normal(size=(300, 2)) * np.where(rng.random((300, 1)) < 0.5, 1e-3, 1.0)).astype(np.float32)
    X[7] = X[8]          # two coincident points
    root, order, codes, side = quadtree.build(X)
    assert np.all(np.diff(codes) >= 0)
    pts = X.astype(np.float64)[order]
    nodes = _walk(root, [])
    for nd in nodes:
        assert np.isclose(nd.cx, pts[nd.start:nd.start + nd.count, 0].mean(), rtol=0, atol=1e-12)
        if nd.children:
            assert nd.count > 1 and nd.level < quadtree.LEVELS
            assert sum(c.count for c in nd.children) == nd.count
            assert nd.children[0].start == nd.start
            for c0, c1 in zip(nd.children, nd.children[1:]):
                assert c0.start + c0.count == c1.start
            assert all(c.level == nd.level + 1 for c in nd.children)
        else:
            assert nd.count == 1 or nd.level == quadtree.LEVELS
    leaves = [nd for nd in nodes if not nd.children]
    assert sum(nd.count for nd in leaves) == len(X)
    # the two coincident points share a leaf at the deepest level
    assert any(nd.count == 2 and nd.level == quadtree.LEVELS for nd in leaves)


def test_stretched_square_keeps_points_apart():
    # 2000 points of spread 1 and four points 1e4 away: the bulk covers about
    # 1e-4 of the square's side, finer than 2^-16 of it, so the leaves lie
    # below level 16; every leaf still holds one point, except the one pair of
    # coincident points
    rng = np.random.default_rng(5)
    X = rng.normal(size=(2000, 2)).astype(np.float32)
    X[:4] = np.array([[1e4, 0], [-1e4, 0], [0, 1e4], [0, -1e4]], np.float32)
    X[10] = X[11]
    root, order, codes, side = quadtree.build(X)
    leaves = [nd for nd in _walk(root, []) if not nd.children]
    assert sum(nd.count for nd in leaves) == len(X)
    shared = [nd for nd in leaves if nd.count > 1]
    assert len(shared) == 1 and shared[0].count == 2 and shared[0].level == quadtree.LEVELS
    assert max(nd.level for nd in leaves if nd.count == 1) > 16
    # theta near 0: the exact all-pairs sums, also at this depth
    zi, frep, fent, _ = quadtree.sums(X, theta=1e-6, eps=0.05)
    ez, er, ee = gradient.pair_sums(X.astype(np.float64), 0.05)
    assert np.allclose(zi, ez, rtol=1e-12, atol=0)
    assert np.allclose(frep, er, rtol=1e-9, atol=1e-15)
    assert np.allclose(fent, ee, rtol=1e-9, atol=1e-15)


def test_far_cluster_is_one_summary():
    rng = np.random.default_rng(2)
    B = np.array([100.0, 100.0]) + rng.normal(size=(30, 2)) * 1e-2
    X = np.vstack([[0.0, 0.0], B]).astype(np.float32)
    zi, frep, fent, lnv = quadtree.sums(X, theta=0.5, eps=0.05)
    c = X[1:].astype(np.float64).mean(0)
    d = -c
    r2 = float(d @ d)
    z = 1.0 / (1.0 + r2)
    assert zi[0] == pytest.approx(30 * z, rel=1e-14)
    assert np.allclose(frep[0], 30 * z * z * d, rtol=1e-13)
    assert np.allclose(fent[0], 30 * d / (0.05 + r2), rtol=1e-13)
    assert lnv[0] == pytest.approx(30 * np.log(0.05 + r2), rel=1e-14)


def test_error_shrinks_with_theta():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(400, 2)).astype(np.float32) * 3
    _, r_ex, e_ex = gradient.pair_sums(X.astype(np.float64), 0.05)
    errs = []
    for th in (0.2, 0.4, 0.7):
        _, fr, fe, _ = quadtree.sums(X, theta=th)
        errs.append((np.linalg.norm(fr - r_ex) / np.linalg.norm(r_ex),
                     np.linalg.norm(fe - e_ex) / np.linalg.norm(e_ex)))
    assert errs[0][0] < errs[1][0] < errs[2][0] < 0.05
    assert errs[0][1] < errs[1][1] < errs[2][1] < 0.05


def test_coincident_points_and_batch():
    X = np.zeros((9, 2), np.float32)
    zi, frep, fent, lnv = quadtree.sums(X, theta=0.5)
    assert np.all(zi == 8.0) and np.all(frep == 0.0) and np.all(fent == 0.0)
    assert np.allclose(lnv, 8 * np.log(0.05))
    rng = np.random.default_rng(4)
    parts = [rng.normal(size=(n, 2)).astype(np.float32) * s for n, s in ((50, 1.0), (1, 1.0), (80, 20.0))]
    Xb = np.vstack(parts)
    off = np.cumsum([0] + [len(p) for p in parts])
    got = quadtree.sums(Xb, theta=0.5, graph_offsets=off)
    for gi, p in enumerate(parts):
        alone = quadtree.sums(p, theta=0.5)
        for a, b in zip(got, alone):
            assert np.array_equal(a[off[gi]:off[gi + 1]], b)
    with pytest.raises(ValueError):
        quadtree.sums(Xb, theta=0.75)
