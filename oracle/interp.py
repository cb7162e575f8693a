"""FFT-accelerated interpolation of the kernel sums, in FP64 (oracle side).

Sec. 2.3 and Sec. 3.3: the drawing area is cut into intervals, each holding P
interpolation points; the kernel between the points is replaced by its values
between interpolation nodes, and the node-to-node sums are a convolution that
an FFT evaluates. L-tsNET (Algorithm 3) applies this to the KL repulsion and to
the entropy sums h1, h2, h3 of Eq. (8).

The paper fixes neither the interval count nor the node placement, nor which
part of the drawing the grid covers. Reading used on both sides (oracle and
GPU):

* the region (``split``): normally the bounding box of the graph's layout.
  When a few far points stretch it, they are set apart: per axis, the
  coordinates are put in ``TRIM_BINS`` equal bins over the bounding box
  (bin = floor((v - v_min) * (TRIM_BINS / w)) in FP64, the last bin closed);
  lo is the bin of the (t+1)-th smallest coordinate and hi the bin of the
  (t+1)-th largest, t = min(far_trim, floor(n / 64)). The core is the set of
  points whose bins lie in [lo, hi] on both axes, its region the union of
  those bins. When that region's larger side is at most half the bounding
  box's larger side (and t >= 1), the grid covers the core region and the
  other points (at most 4 t) are far points; otherwise the grid covers the
  bounding box and no point is far;
* square boxes over that region; span = its larger side (at least
  ``SPAN_FLOOR``); n_int = ceil(span / h_target) clamped to
  [min_intervals, max_intervals] and rounded up to a power of two; box side
  h = span / n_int; the grid is centred on the region's centre c;
* P = 3 nodes per box and axis at local offsets (t + 1/2) / 3, t = 0, 1, 2, so
  the N_g = 3 n_int nodes per axis are equispaced with spacing h / 3;
* a core point with local coordinates (s, t) in [0, 1]^2 of its box is spread
  to and gathered from the 3 x 3 nodes of that box with Lagrange weights
  L_a(s) L_b(t);
* charges 1, x - c_x, y - c_y; kernels
  K2 = (1 + r^2)^-2, K1 = (1 + r^2)^-1, Ke = (eps + r^2)^-1, Kln = ln(eps + r^2).

With phi[K, q](i) the interpolated sum_j K(X_i - X_j) q_j over the core points
(the j = i term included):
    F_rep,i = (x_i - c) phi[K2, 1] - phi[K2, x]     (self term cancels)
    F_ent,i = (x_i - c) phi[Ke, 1] - phi[Ke, x]     (Eq. 8; self term cancels)
    Z_i     = phi[K1, 1] - 1                         (K1(0) = 1)
    sum_{j!=i} ln(eps + r_ij^2) = phi[Kln, 1] - ln(eps)
The node-to-node step is a linear convolution; here it is done with a library
FFT convolution (or a direct sum on tiny grids).

A far point o is never interpolated on its own side: between o and a core
point the kernel is interpolated in the core point's argument only,
K(X_o - X_j) ~ sum_b K(X_o - y_b) L_b(X_j) (y_b the nodes), so o adds
K(y_a - X_o) q(o) to the potential of every node a before the gather, and o's
own sums are sum_b K(X_o - y_b) w_b over the node charges w plus the exact
sums over the other far points (no self term).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SPAN_FLOOR = 1e-4
NODES = 3
NODE_OFFSETS = (np.arange(NODES) + 0.5) / NODES     # 1/6, 1/2, 5/6
TRIM_BINS = 2048      # bins per axis of the far-point rule
FAR_TRIM = 64         # default t: at most t points set apart per side and axis
TRIM_MIN_POINTS = 64  # t is also at most floor(n / TRIM_MIN_POINTS)


@dataclass
class Grid:
    n_int: int
    h: float           # box side
    x0: float          # lower-left corner of the box grid
    y0: float
    cx: float          # charge centre
    cy: float
    span: float

    @property
    def n_nodes(self) -> int:
        return NODES * self.n_int

    @property
    def spacing(self) -> float:
        return self.h / NODES


def next_pow2(v: int) -> int:
    p = 1
    while p < v:
        p *= 2
    return p


def grid_over(xlo: float, xhi: float, ylo: float, yhi: float, h_target: float,
              min_intervals: int, max_intervals: int) -> Grid:
    """The square box grid over the region [xlo, xhi] x [ylo, yhi]."""
    span = max(xhi - xlo, yhi - ylo, SPAN_FLOOR)
    n_int = int(np.ceil(span / h_target))
    n_int = min(max(n_int, min_intervals), max_intervals)
    n_int = min(next_pow2(n_int), max_intervals)
    h = span / n_int
    cx, cy = 0.5 * (xlo + xhi), 0.5 * (ylo + yhi)
    return Grid(n_int, h, cx - 0.5 * n_int * h, cy - 0.5 * n_int * h, cx, cy, span)


def make_grid(X: np.ndarray, h_target: float, min_intervals: int, max_intervals: int) -> Grid:
    """The grid over the bounding box of X (no point set apart)."""
    X = np.asarray(X, dtype=np.float64)
    xmin, ymin = X.min(axis=0)
    xmax, ymax = X.max(axis=0)
    return grid_over(xmin, xmax, ymin, ymax, h_target, min_intervals, max_intervals)


@dataclass
class Split:
    far: np.ndarray     # bool [n]: points set apart
    region: tuple       # (xlo, xhi, ylo, yhi) the grid covers
    trimmed: bool


def trim_count(n: int, far_trim: int) -> int:
    return min(far_trim, n // TRIM_MIN_POINTS)


def axis_bins(v: np.ndarray, vmin: float, w: float) -> np.ndarray:
    """Bin of every coordinate among TRIM_BINS equal bins over [vmin, vmin + w]."""
    if not w > 0:
        return np.zeros(v.shape[0], dtype=np.int64)
    b = np.floor((np.asarray(v, dtype=np.float64) - vmin) * (TRIM_BINS / w)).astype(np.int64)
    return np.minimum(b, TRIM_BINS - 1)


def _trim_bounds(bins: np.ndarray, t: int):
    """lo = bin of the (t+1)-th smallest value, hi = bin of the (t+1)-th largest."""
    cnt = np.bincount(bins, minlength=TRIM_BINS)
    lo = int(np.searchsorted(np.cumsum(cnt), t + 1))
    hi = TRIM_BINS - 1 - int(np.searchsorted(np.cumsum(cnt[::-1]), t + 1))
    return lo, hi


def split(X: np.ndarray, far_trim: int = FAR_TRIM) -> Split:
    """Which points the grid covers and which are set apart (module docstring)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    xmin, ymin = X.min(axis=0)
    xmax, ymax = X.max(axis=0)
    wx, wy = xmax - xmin, ymax - ymin
    box = (xmin, xmax, ymin, ymax)
    none = Split(np.zeros(n, dtype=bool), box, False)
    t = trim_count(n, far_trim)
    span = max(wx, wy)
    if t < 1 or not span > 0:
        return none
    bx, by = axis_bins(X[:, 0], xmin, wx), axis_bins(X[:, 1], ymin, wy)
    lox, hix = _trim_bounds(bx, t)
    loy, hiy = _trim_bounds(by, t)
    qx, qy = wx / TRIM_BINS, wy / TRIM_BINS
    cw, ch = (hix - lox + 1) * qx, (hiy - loy + 1) * qy
    if not 2.0 * max(cw, ch) <= span:
        return none
    far = (bx < lox) | (bx > hix) | (by < loy) | (by > hiy)
    region = (xmin + lox * qx, xmin + (hix + 1) * qx, ymin + loy * qy, ymin + (hiy + 1) * qy)
    return Split(far, region, True)


def lagrange_weights(s: np.ndarray) -> np.ndarray:
    """[len(s), 3] Lagrange basis at local coordinate s for nodes NODE_OFFSETS."""
    s = np.asarray(s, dtype=np.float64)
    out = np.ones((s.shape[0], NODES))
    for a in range(NODES):
        for b in range(NODES):
            if a != b:
                out[:, a] *= (s - NODE_OFFSETS[b]) / (NODE_OFFSETS[a] - NODE_OFFSETS[b])
    return out


def locate(X: np.ndarray, grid: Grid):
    """Box indices (bx, by) and local coordinates (s, t) of every point."""
    fx = (X[:, 0] - grid.x0) / grid.h
    fy = (X[:, 1] - grid.y0) / grid.h
    bx = np.clip(np.floor(fx), 0, grid.n_int - 1).astype(np.int64)
    by = np.clip(np.floor(fy), 0, grid.n_int - 1).astype(np.int64)
    return bx, by, fx - bx, fy - by


def spread(X: np.ndarray, grid: Grid, charges: np.ndarray) -> np.ndarray:
    """Node charges w[c, ay, ax] = sum_points L_tx(s) L_ty(t) q_c (one box per point)."""
    bx, by, s, t = locate(X, grid)
    lx, ly = lagrange_weights(s), lagrange_weights(t)
    ng = grid.n_nodes
    w = np.zeros((charges.shape[0], ng, ng))
    for ty in range(NODES):
        for tx in range(NODES):
            wt = ly[:, ty] * lx[:, tx]
            ay = NODES * by + ty
            ax = NODES * bx + tx
            for c in range(charges.shape[0]):
                np.add.at(w[c], (ay, ax), wt * charges[c])
    return w


def kernel_values(name: str, r2: np.ndarray, eps: float) -> np.ndarray:
    if name == "K2":
        return 1.0 / (1.0 + r2) ** 2
    if name == "K1":
        return 1.0 / (1.0 + r2)
    if name == "Ke":
        return 1.0 / (eps + r2)
    if name == "Kln":
        return np.log(eps + r2)
    if name == "one":
        return np.ones_like(r2)
    if name == "quad":
        return r2
    raise ValueError(name)


def kernel_stencil(name: str, grid: Grid, eps: float) -> np.ndarray:
    """K at every node offset (dy, dx) in [-(N_g-1), N_g-1]^2."""
    ng = grid.n_nodes
    off = np.arange(-(ng - 1), ng) * grid.spacing
    r2 = off[:, None] ** 2 + off[None, :] ** 2
    return kernel_values(name, r2, eps)


def node_coords(grid: Grid):
    """x and y of the node columns and rows (equispaced, spacing h / 3)."""
    k = np.arange(grid.n_nodes) + 0.5
    return grid.x0 + k * grid.spacing, grid.y0 + k * grid.spacing


def convolve(w: np.ndarray, stencil: np.ndarray, method: str = "fft") -> np.ndarray:
    """phi[by, bx] = sum_{ay, ax} K[by - ay, bx - ax] w[ay, ax] (linear convolution)."""
    ng = w.shape[0]
    if method == "fft":
        from scipy.signal import fftconvolve
        full = fftconvolve(w, stencil, mode="full")
        return full[ng - 1:2 * ng - 1, ng - 1:2 * ng - 1]
    if method == "direct":
        out = np.zeros_like(w)
        for by in range(ng):
            for bx in range(ng):
                k = stencil[by - np.arange(ng)[:, None] + ng - 1, bx - np.arange(ng)[None, :] + ng - 1]
                out[by, bx] = np.sum(k * w)
        return out
    raise ValueError(method)


def gather(X: np.ndarray, grid: Grid, phi: np.ndarray) -> np.ndarray:
    """Interpolate node potentials phi[..., ny, nx] back to every point."""
    bx, by, s, t = locate(X, grid)
    lx, ly = lagrange_weights(s), lagrange_weights(t)
    out = np.zeros((X.shape[0],) + phi.shape[:-2])
    for ty in range(NODES):
        for tx in range(NODES):
            vals = phi[..., NODES * by + ty, NODES * bx + tx]   # [..., n]
            out += (ly[:, ty] * lx[:, tx])[:, None] * np.moveaxis(vals, -1, 0).reshape(X.shape[0], -1)
    return out


def _far_node_kernel(name: str, grid: Grid, Xf: np.ndarray, eps: float) -> np.ndarray:
    """K(y_a - X_o) for every far point o and node a: [F, N_g, N_g]."""
    nx, ny = node_coords(grid)
    dx = nx[None, None, :] - Xf[:, 0, None, None]
    dy = ny[None, :, None] - Xf[:, 1, None, None]
    return kernel_values(name, dx * dx + dy * dy, eps)


def potentials(X, grid: Grid, kernels, eps: float, method: str = "fft", far=None):
    """phi[K, q] for each kernel name in ``kernels`` and charges (1, x - cx, y - cy).

    Returns (core, far_sums): core[name] is [n_core, 3] at the core points
    (interpolated, the j = i term included), far_sums[name] is [F, 3] at the
    far points (no self term). With ``far`` None every point is a core point.
    """
    X = np.asarray(X, dtype=np.float64)
    far = np.zeros(X.shape[0], dtype=bool) if far is None else np.asarray(far, dtype=bool)
    Xc, Xf = X[~far], X[far]
    q = np.stack([np.ones(X.shape[0]), X[:, 0] - grid.cx, X[:, 1] - grid.cy])
    qc, qf = q[:, ~far], q[:, far]
    w = spread(Xc, grid, qc)
    core, fsum = {}, {}
    for name in kernels:
        st = kernel_stencil(name, grid, eps)
        phi = np.stack([convolve(w[c], st, method) for c in range(3)])
        if Xf.shape[0]:
            Kf = _far_node_kernel(name, grid, Xf, eps)             # [F, ng, ng]
            phi = phi + np.einsum("fyx,cf->cyx", Kf, qf)            # far charges at the nodes
            d = Xf[:, None, :] - Xf[None, :, :]
            Kff = kernel_values(name, (d ** 2).sum(-1), eps)
            np.fill_diagonal(Kff, 0.0)
            fsum[name] = np.einsum("fyx,cyx->fc", Kf, w) + Kff @ qf.T
        else:
            fsum[name] = np.zeros((0, 3))
        core[name] = gather(Xc, grid, phi)                          # [n_core, 3]
    return core, fsum


@dataclass
class InterpTerms:
    grid: Grid
    F_rep: np.ndarray
    F_ent: np.ndarray
    Z_i: np.ndarray
    Z: float
    ln_sum: float | None = None
    far: np.ndarray | None = None   # bool [n]: the points set apart


def interp_terms(X, eps: float, h_target: float = 0.25, min_intervals: int = 50,
                 max_intervals: int = 512, method: str = "fft", with_ln: bool = False,
                 far_trim: int = FAR_TRIM) -> InterpTerms:
    """Interpolated F_rep, F_ent, Z_i and Z for one graph (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    sp = split(X, far_trim)
    grid = grid_over(*sp.region, h_target, min_intervals, max_intervals)
    names = ["K2", "K1", "Ke"] + (["Kln"] if with_ln else [])
    core, fs = potentials(X, grid, names, eps, method, far=sp.far)
    xt = np.stack([X[:, 0] - grid.cx, X[:, 1] - grid.cy], axis=1)
    frep = np.zeros((n, 2))
    fent = np.zeros((n, 2))
    zi = np.zeros(n)
    c, f = ~sp.far, sp.far
    frep[c] = xt[c] * core["K2"][:, :1] - core["K2"][:, 1:]
    fent[c] = xt[c] * core["Ke"][:, :1] - core["Ke"][:, 1:]
    zi[c] = core["K1"][:, 0] - 1.0
    frep[f] = xt[f] * fs["K2"][:, :1] - fs["K2"][:, 1:]
    fent[f] = xt[f] * fs["Ke"][:, :1] - fs["Ke"][:, 1:]
    zi[f] = fs["K1"][:, 0]
    if n == 1:
        frep[:] = 0.0
        fent[:] = 0.0
        zi[:] = 0.0
    ln_sum = None
    if with_ln:
        ln_sum = float(np.sum(core["Kln"][:, 0]) - int(c.sum()) * np.log(eps) + np.sum(fs["Kln"][:, 0]))
    return InterpTerms(grid, frep, fent, zi, float(zi.sum()), ln_sum, sp.far)
