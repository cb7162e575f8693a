"""Pins for the oracle's FFT-accelerated interpolation (CPU only)."""
import numpy as np
import pytest

from oracle import gradient, interp


def test_lagrange_basis_nodal_and_partition_of_unity():
    L = interp.lagrange_weights(interp.NODE_OFFSETS)
    assert np.allclose(L, np.eye(3), atol=1e-15)
    s = np.linspace(0, 1, 101)
    W = interp.lagrange_weights(s)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-14)
    # quadratics are reproduced exactly
    for f in (lambda t: t * t, lambda t: 3 - 2 * t):
        assert np.allclose(W @ f(interp.NODE_OFFSETS), f(s), atol=1e-14)


def test_grid_rule():
    X = np.array([[0.0, 0.0], [2.0, 0.5]])
    g = interp.make_grid(X, 0.25, 2, 64)
    assert g.n_int == 8 and abs(g.h - 0.25) < 1e-15
    assert abs(g.x0 - 0.0) < 1e-15 and abs(g.y0 - (0.25 - 1.0)) < 1e-15
    g = interp.make_grid(X, 0.25, 50, 256)
    assert g.n_int == 64
    g = interp.make_grid(X * 100, 0.25, 50, 256)
    assert g.n_int == 256 and abs(g.h - 200 / 256) < 1e-12


def test_fft_convolution_equals_direct_sum():
    rng = np.random.default_rng(0)
    X = rng.normal(0, 1, (40, 2))
    grid = interp.make_grid(X, 0.25, 2, 4)
    w = rng.normal(size=(grid.n_nodes, grid.n_nodes))
    st = interp.kernel_stencil("Ke", grid, 0.05)
    a = interp.convolve(w, st, "fft")
    b = interp.convolve(w, st, "direct")
    assert np.allclose(a, b, rtol=1e-11, atol=1e-11 * np.abs(b).max())


def _exact_sums(X, name, eps):
    d = X[:, None, :] - X[None, :, :]
    r2 = (d ** 2).sum(-1)
    K = interp.kernel_values(name, r2, eps)
    q = np.stack([np.ones(X.shape[0]), X[:, 0], X[:, 1]])
    return K @ q.T     # includes j = i


@pytest.mark.parametrize("name", ["quad", "one"])
def test_low_degree_kernels_are_exact(name):
    # K = r^2 is quadratic in each coordinate, K = 1 constant: the tensor
    # Lagrange interpolation reproduces both exactly.
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1.5, (120, 2))
    grid = interp.make_grid(X, 0.5, 4, 16)
    pot = interp.potentials(X, grid, [name], 0.05)[name]
    want = _exact_sums(X, name, 0.05)
    want[:, 1] -= grid.cx * want[:, 0]
    want[:, 2] -= grid.cy * want[:, 0]
    assert np.allclose(pot, want, rtol=1e-10, atol=1e-10 * np.abs(want).max())


def test_error_falls_with_interval_width():
    rng = np.random.default_rng(2)
    X = rng.normal(0, 2.0, (500, 2))
    zi, frep, fent = gradient.pair_sums(X, 0.05)
    errs = []
    for nint in (16, 32, 64):
        t = interp.interp_terms(X, 0.05, h_target=1e-9, min_intervals=1, max_intervals=nint)
        assert t.grid.n_int == nint
        errs.append(np.linalg.norm(t.F_ent - fent) / np.linalg.norm(fent))
        rep_err = np.linalg.norm(t.F_rep - frep) / np.linalg.norm(frep)
        assert rep_err < 3 * errs[-1] + 1e-6
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4


def test_default_settings_meet_tolerance():
    rng = np.random.default_rng(3)
    X = rng.normal(0, 1.0, (800, 2))
    zi, frep, fent = gradient.pair_sums(X, 0.05)
    t = interp.interp_terms(X, 0.05, with_ln=True)
    assert np.linalg.norm(t.F_rep - frep) <= 1e-3 * np.linalg.norm(frep)
    assert np.linalg.norm(t.F_ent - fent) <= 1e-3 * np.linalg.norm(fent)
    assert abs(t.Z - zi.sum()) <= 1e-5 * zi.sum()
    d = X[:, None, :] - X[None, :, :]
    r2 = (d ** 2).sum(-1)
    lsum = np.log(0.05 + r2).sum() - X.shape[0] * np.log(0.05)
    assert abs(t.ln_sum - lsum) <= 1e-5 * abs(lsum)
