"""Pins for the oracle's exact cost, gradient and finite-difference helper (CPU only)."""
import numpy as np
import pytest

from oracle import affinities, gradient
from oracle.gradient import CostParams
from synth import graphs


def _problem(n=40, seed=0, scale=1.0):
    g = graphs.sbm([n // 2, n - n // 2], 0.3, 0.05, seed)
    oP = affinities.build_P(g.indptr, g.indices, 4.0, seed=seed)
    X = np.random.default_rng(seed).normal(0, scale, (n, 2))
    return g, oP, X


def _cost(X, oP, prm):
    return float(gradient.cost_terms(X, oP, prm).total[0])


@pytest.mark.parametrize("scale", [0.05, 1.0, 4.0])
def test_gradient_matches_central_differences(scale):
    _, oP, X = _problem(30, 1, scale)
    prm = CostParams(lambda_kl=1.0, lambda_c=1.2, lambda_r=0.3, eps_r=0.05)
    G = gradient.grad_terms(X, oP, prm).G
    h = 1e-5 * max(scale, 0.1)
    fd = np.zeros_like(X)
    for i in range(X.shape[0]):
        for a in range(2):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            fd[i, a] = (_cost(Xp, oP, prm) - _cost(Xm, oP, prm)) / (2 * h)
    assert np.linalg.norm(fd - G) <= 1e-6 * np.linalg.norm(G)


def test_fd_delta_cost_equals_cost_difference():
    _, oP, X = _problem(36, 2, 1.0)
    prm = CostParams(lambda_r=0.2)
    Z = gradient.normaliser(X)
    for (i, a, h) in [(0, 0, 1e-3), (5, 1, 0.1), (20, 0, 0.7)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[i, a] += h
        Xm[i, a] -= h
        want = _cost(Xp, oP, prm) - _cost(Xm, oP, prm)
        got = gradient.fd_delta_cost(X, oP, prm, i, a, h, Z, psum=float(oP.val.sum()))
        assert abs(got - want) <= 1e-9 * max(abs(want), 1e-12)


def test_fd_delta_cost_gives_gradient():
    _, oP, X = _problem(200, 3, 2.0)
    prm = CostParams()
    G = gradient.grad_terms(X, oP, prm).G
    Z = gradient.normaliser(X)
    h = 1e-4
    for i, a in [(0, 0), (17, 1), (150, 0), (199, 1)]:
        d = gradient.fd_delta_cost(X, oP, prm, i, a, h, Z, psum=float(oP.val.sum()))
        assert abs(d / (2 * h) - G[i, a]) <= 1e-6 * np.abs(G).max()


def test_brute_force_pair_sums():
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (6, 2))
    eps = 0.05
    zi, frep, fent = gradient.pair_sums(X, eps)
    for i in range(6):
        z, r, e = 0.0, np.zeros(2), np.zeros(2)
        for j in range(6):
            if i == j:
                continue
            d = X[i] - X[j]
            r2 = d[0] * d[0] + d[1] * d[1]
            w = 1.0 / (1.0 + r2)
            z += w
            r += w * w * d
            e += d / (eps + r2)
        assert abs(zi[i] - z) < 1e-14 and np.allclose(frep[i], r, atol=1e-15)
        assert np.allclose(fent[i], e, rtol=1e-14)


def test_zero_sum_and_symmetries():
    _, oP, X = _problem(50, 5, 1.5)
    prm = CostParams()
    T = gradient.grad_terms(X, oP, prm)
    for F in (T.F_attr, T.F_rep, T.F_ent):
        assert np.linalg.norm(F.sum(axis=0)) <= 1e-12 * np.abs(F).sum()
    # translation: the KL and entropy parts do not change
    shift = np.array([3.0, -1.5])
    T2 = gradient.grad_terms(X + shift, oP, prm)
    assert np.allclose(T2.F_attr, T.F_attr, atol=1e-12) and np.allclose(T2.F_ent, T.F_ent, atol=1e-9)
    assert abs(T2.Z[0] - T.Z[0]) < 1e-9 * T.Z[0]
    # rotation: the whole gradient rotates with the layout
    c, s = np.cos(0.7), np.sin(0.7)
    R = np.array([[c, -s], [s, c]])
    T3 = gradient.grad_terms(X @ R.T, oP, prm)
    assert np.allclose(T3.G, T.G @ R.T, atol=1e-12 * np.abs(T.G).max() * 100)


def test_two_vertices_closed_form():
    g = graphs.csr_from_edges(2, np.array([0]), np.array([1]))
    oP = affinities.build_P(g.indptr, g.indices, 1.0)
    assert np.allclose(oP.val, 0.5)
    X = np.array([[0.3, -0.2], [1.1, 0.4]])
    prm = CostParams(lambda_kl=1.0, lambda_c=0.0, lambda_r=0.0)
    T = gradient.grad_terms(X, oP, prm)
    assert np.allclose(T.G, 0.0, atol=1e-15)           # P equals Q
    C = gradient.cost_terms(X, oP, prm)
    assert abs(C.kl[0]) < 1e-15
    # entropy alone: -(lambda_r / 4) d / (eps + r^2) on vertex 0
    prm = CostParams(lambda_kl=0.0, lambda_c=0.0, lambda_r=1.0, eps_r=0.05)
    d = X[0] - X[1]
    want = -(1.0 / 4.0) * d / (0.05 + d @ d)
    assert np.allclose(gradient.grad_terms(X, oP, prm).G[0], want, rtol=1e-14)


def test_kl_nonnegative_and_entropy_forms_agree_as_eps_vanishes():
    _, oP, X = _problem(40, 6, 1.0)
    assert gradient.cost_terms(X, oP).kl[0] >= 0
    for eps in (1e-3, 1e-6):
        prm = CostParams(eps_r=eps)
        a = gradient.cost_terms(X, oP, prm, entropy="kernel").ent[0]
        b = gradient.cost_terms(X, oP, prm, entropy="literal").ent[0]
        assert abs(a - b) <= 50 * eps * abs(b)


def test_single_vertex():
    g = graphs.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    oP = affinities.build_P(g.indptr, g.indices, 5.0)
    X = np.array([[0.4, -2.0]])
    T = gradient.grad_terms(X, oP, CostParams(lambda_c=1.2))
    assert T.Z[0] == 0 and np.allclose(T.G, 1.2 * X)
