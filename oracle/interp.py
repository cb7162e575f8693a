"""FFT-accelerated interpolation of the kernel sums, in FP64 (oracle side).

Sec. 2.3 and Sec. 3.3: the drawing area is cut into intervals, each holding P
interpolation points; the kernel between the points is replaced by its values
between interpolation nodes, and the node-to-node sums are a convolution that
an FFT evaluates. L-tsNET (Algorithm 3) applies this to the KL repulsion and to
the entropy sums h1, h2, h3 of Eq. (8).

The paper fixes neither the interval count nor the node placement. Reading
used on both sides (oracle and GPU):

* square boxes over the bounding box of the graph's layout; span = the larger
  side (at least ``SPAN_FLOOR``); n_int = ceil(span / h_target) clamped to
  [min_intervals, max_intervals] and rounded up to a power of two; box side
  h = span / n_int; the grid is centred on the bounding-box centre c;
* P = 3 nodes per box and axis at local offsets (t + 1/2) / 3, t = 0, 1, 2, so
  the N_g = 3 n_int nodes per axis are equispaced with spacing h / 3;
* a point with local coordinates (s, t) in [0, 1]^2 of its box is spread to and
  gathered from the 3 x 3 nodes of that box with Lagrange weights
  L_a(s) L_b(t);
* charges 1, x - c_x, y - c_y; kernels
  K2 = (1 + r^2)^-2, K1 = (1 + r^2)^-1, Ke = (eps + r^2)^-1, Kln = ln(eps + r^2).

With phi[K, q](i) the interpolated sum_j K(X_i - X_j) q_j (the j = i term
included):
    F_rep,i = (x_i - c) phi[K2, 1] - phi[K2, x]     (self term cancels)
    F_ent,i = (x_i - c) phi[Ke, 1] - phi[Ke, x]     (Eq. 8; self term cancels)
    Z_i     = phi[K1, 1] - 1                         (K1(0) = 1)
    sum_{j!=i} ln(eps + r_ij^2) = phi[Kln, 1] - ln(eps)
The node-to-node step is a linear convolution; here it is done with a library
FFT convolution (or a direct sum on tiny grids).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SPAN_FLOOR = 1e-4
NODES = 3
NODE_OFFSETS = (np.arange(NODES) + 0.5) / NODES     # 1/6, 1/2, 5/6


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


def make_grid(X: np.ndarray, h_target: float, min_intervals: int, max_intervals: int) -> Grid:
    X = np.asarray(X, dtype=np.float64)
    xmin, ymin = X.min(axis=0)
    xmax, ymax = X.max(axis=0)
    span = max(xmax - xmin, ymax - ymin, SPAN_FLOOR)
    n_int = int(np.ceil(span / h_target))
    n_int = min(max(n_int, min_intervals), max_intervals)
    n_int = min(next_pow2(n_int), max_intervals)
    h = span / n_int
    cx, cy = 0.5 * (xmin + xmax), 0.5 * (ymin + ymax)
    return Grid(n_int, h, cx - 0.5 * n_int * h, cy - 0.5 * n_int * h, cx, cy, span)


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


def potentials(X, grid: Grid, kernels, eps: float, method: str = "fft"):
    """phi[K, q](i) for each kernel name in ``kernels`` and charges (1, x - cx, y - cy)."""
    X = np.asarray(X, dtype=np.float64)
    q = np.stack([np.ones(X.shape[0]), X[:, 0] - grid.cx, X[:, 1] - grid.cy])
    w = spread(X, grid, q)
    out = {}
    for name in kernels:
        st = kernel_stencil(name, grid, eps)
        phi = np.stack([convolve(w[c], st, method) for c in range(3)])
        out[name] = gather(X, grid, phi)            # [n, 3]
    return out


@dataclass
class InterpTerms:
    grid: Grid
    F_rep: np.ndarray
    F_ent: np.ndarray
    Z_i: np.ndarray
    Z: float
    ln_sum: float | None = None


def interp_terms(X, eps: float, h_target: float = 0.25, min_intervals: int = 50,
                 max_intervals: int = 256, method: str = "fft", with_ln: bool = False) -> InterpTerms:
    """Interpolated F_rep, F_ent, Z_i and Z for one graph (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    grid = make_grid(X, h_target, min_intervals, max_intervals)
    names = ["K2", "K1", "Ke"] + (["Kln"] if with_ln else [])
    pot = potentials(X, grid, names, eps, method)
    xt = np.stack([X[:, 0] - grid.cx, X[:, 1] - grid.cy], axis=1)
    frep = xt * pot["K2"][:, :1] - pot["K2"][:, 1:]
    fent = xt * pot["Ke"][:, :1] - pot["Ke"][:, 1:]
    zi = pot["K1"][:, 0] - 1.0
    n = X.shape[0]
    if n == 1:
        frep[:] = 0.0
        fent[:] = 0.0
        zi[:] = 0.0
    ln_sum = None
    if with_ln:
        ln_sum = float(np.sum(pot["Kln"][:, 0]) - n * np.log(eps))
    return InterpTerms(grid, frep, fent, zi, float(zi.sum()), ln_sum)
