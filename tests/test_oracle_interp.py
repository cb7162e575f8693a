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
    pot = interp.potentials(X, grid, [name], 0.05)[0][name]
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


# ----------------------------------------------------------------- far points
def _bulk_with_outliers(n, n_out, seed, std=0.15, far=30.0):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, std, (n, 2))
    X[:n_out] = rng.normal(0, far, (n_out, 2))
    return X


def _split_by_sorting(X, far_trim):
    """The far-point rule written with sorted coordinates instead of histograms:
    lo / hi are the bins of the (t+1)-th smallest / largest coordinate."""
    n = X.shape[0]
    t = min(far_trim, n // 64)
    lo, hi, bins = [], [], []
    for a in range(2):
        v = X[:, a]
        vmin, w = v.min(), v.max() - v.min()
        b = np.minimum(np.floor((v - vmin) * (2048 / w)).astype(np.int64), 2047)
        sb = np.sort(b)
        lo.append(sb[t])
        hi.append(sb[n - 1 - t])
        bins.append(b)
    far = np.zeros(n, dtype=bool)
    for a in range(2):
        far |= (bins[a] < lo[a]) | (bins[a] > hi[a])
    return t, far, lo, hi


@pytest.mark.parametrize("n,n_out,seed", [(3000, 12, 0), (5000, 40, 1), (20000, 3, 2)])
def test_split_matches_sorted_definition(n, n_out, seed):
    X = _bulk_with_outliers(n, n_out, seed)
    sp = interp.split(X)
    t, far, lo, hi = _split_by_sorting(X, interp.FAR_TRIM)
    assert sp.trimmed
    assert np.array_equal(sp.far, far)
    assert far.sum() <= 4 * t
    assert far[:n_out].all()                     # every planted outlier is set apart
    # at most t points lie beyond each bound, more than t at or beyond it
    for a in range(2):
        v = X[:, a]
        assert np.sum(v < sp.region[2 * a]) <= t and np.sum(v <= sp.region[2 * a + 1]) >= n - t
    # the region is the union of the core bins: it holds every core point
    core = X[~sp.far]
    assert (core[:, 0] >= sp.region[0]).all() and (core[:, 0] <= sp.region[1] + 1e-12).all()
    assert (core[:, 1] >= sp.region[2]).all() and (core[:, 1] <= sp.region[3] + 1e-12).all()


def test_split_not_used_without_far_points():
    rng = np.random.default_rng(4)
    for X in (rng.uniform(-5, 5, (4000, 2)), rng.normal(0, 3, (4000, 2)),
              np.zeros((500, 2)), rng.normal(0, 1, (63, 2))):
        sp = interp.split(X)
        assert not sp.trimmed and not sp.far.any()
        g = interp.grid_over(*sp.region, 0.25, 50, 512)
        assert g == interp.make_grid(X, 0.25, 50, 512)
    # far_trim = 0 switches the rule off
    assert not interp.split(_bulk_with_outliers(3000, 10, 5), far_trim=0).trimmed


def _exact_all(X, name, eps, self_term):
    d = X[:, None, :] - X[None, :, :]
    K = interp.kernel_values(name, (d ** 2).sum(-1), eps)
    if not self_term:
        np.fill_diagonal(K, 0.0)
    q = np.stack([np.ones(X.shape[0]), X[:, 0], X[:, 1]])
    return K @ q.T


@pytest.mark.parametrize("name", ["quad", "one"])
def test_far_point_sums_exact_for_low_degree_kernels(name):
    # Between a far point and the core the kernel is interpolated in the core
    # point's argument only: quadratic and constant kernels are reproduced
    # exactly in both directions.
    X = _bulk_with_outliers(1500, 10, 6)
    sp = interp.split(X)
    assert sp.trimmed and sp.far.sum() >= 10
    grid = interp.grid_over(*sp.region, 0.05, 4, 64)
    core, fs = interp.potentials(X, grid, [name], 0.05, far=sp.far)
    for rows, got, self_term in ((~sp.far, core[name], True), (sp.far, fs[name], False)):
        want = _exact_all(X, name, 0.05, self_term)[rows]
        want[:, 1] -= grid.cx * want[:, 0]
        want[:, 2] -= grid.cy * want[:, 0]
        assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


def test_far_split_error_falls_with_interval_width():
    X = _bulk_with_outliers(2000, 15, 7)
    zi, frep, fent = gradient.pair_sums(X, 0.05)
    errs = []
    for nint in (8, 16, 32):
        t = interp.interp_terms(X, 0.05, h_target=1e-9, min_intervals=1, max_intervals=nint)
        assert t.grid.n_int == nint and t.far.sum() >= 15
        errs.append(np.linalg.norm(t.F_ent - fent) / np.linalg.norm(fent))
        assert abs(t.Z - zi.sum()) <= 10 * errs[-1] * zi.sum()
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4


def test_dense_bulk_with_far_points_meets_tolerance():
    # the layout class of the early descent from a small random start: a dense
    # bulk and a few points far out that set the bounding box
    X = _bulk_with_outliers(6000, 25, 8, std=0.2, far=40.0)
    zi, frep, fent = gradient.pair_sums(X, 0.05)
    t = interp.interp_terms(X, 0.05, with_ln=True)
    assert t.far.sum() >= 25
    for got, want in ((t.F_rep, frep), (t.F_ent, fent)):
        assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)
    assert abs(t.Z - zi.sum()) <= 1e-6 * zi.sum()
    d = X[:, None, :] - X[None, :, :]
    lsum = np.log(0.05 + (d ** 2).sum(-1)).sum() - X.shape[0] * np.log(0.05)
    assert abs(t.ln_sum - lsum) <= 1e-6 * abs(lsum)
    # the same layout with the rule switched off misses the tolerance: the bulk
    # falls into a handful of boxes
    t0 = interp.interp_terms(X, 0.05, far_trim=0)
    assert np.linalg.norm(t0.F_ent - fent) > 1e-3 * np.linalg.norm(fent)
