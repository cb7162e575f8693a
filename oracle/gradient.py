"""Exact FP64 cost and gradient of the tsNET objective (oracle side).

Cost, Eq. (1):  C = C_KL + C_CMP + C_ENT with
    C_KL  = lambda_KL * sum_{i!=j} p_ij ln(p_ij / q_ij),   q_ij = w_ij / Z,
            w_ij = (1 + ||X_i - X_j||^2)^-1,  Z = sum_{k!=l} w_kl   (Sec. 2.1)
    C_CMP = lambda_c / (2n) * sum_i ||X_i||^2
    C_ENT = -lambda_r / (4 n^2) * sum_{i!=j} ln(eps + ||X_i - X_j||^2)

Reading of the entropy term. Eq. (1) writes ln(||X_i - X_j|| + eps), while the
L-tsNET gradient (Sec. 3.3, Eq. 8) uses the kernel 1 / (eps + ||X_k - X_i||^2).
The form above is the cost whose exact gradient is that kernel sum; it equals
Eq. (1) at eps = 0. The literal form is kept as ``entropy="literal"`` for
comparison only. The gradient sign is the true derivative (a descent step
pushes vertices apart); the printed signs of Eq. (5) and Eq. (8) disagree with
each other.

Gradient (Eq. 6 for the KL part, written with the attraction/repulsion split
of Sec. 2.2, Eq. 8 for the entropy part, plus the compression derivative):
    F_attr,i = sum_j p_ij w_ij (X_i - X_j)
    F_rep,i  = sum_{j!=i} w_ij^2 (X_i - X_j)
    F_ent,i  = sum_{j!=i} (X_i - X_j) / (eps + ||X_i - X_j||^2)
    dC/dX_i  = 4 lambda_KL (F_attr,i - F_rep,i / Z) + (lambda_c / n) X_i
               - (lambda_r / n^2) F_ent,i
With n = 1 there are no pairs: Z = 0 and the F_rep / Z term is taken as 0.
Every graph of a batch is its own problem, with its own n and Z.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CostParams:
    lambda_kl: float = 1.0
    lambda_c: float = 1.2
    lambda_r: float = 0.01
    eps_r: float = 0.05


def _row_block(n: int) -> int:
    return max(1, (1 << 22) // max(n, 1))


def pair_sums(X: np.ndarray, eps: float, rows=None):
    """Exact all-pairs sums for rows of one graph: Z_i, F_rep,i, F_ent,i (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    zi = np.zeros(rows.shape[0])
    frep = np.zeros((rows.shape[0], 2))
    fent = np.zeros((rows.shape[0], 2))
    bs = _row_block(n)
    for s in range(0, rows.shape[0], bs):
        r = rows[s:s + bs]
        d = X[r, None, :] - X[None, :, :]                  # [b, n, 2]
        r2 = d[..., 0] ** 2 + d[..., 1] ** 2
        w = 1.0 / (1.0 + r2)
        ke = 1.0 / (eps + r2)
        self_mask = r[:, None] == np.arange(n)[None, :]
        w[self_mask] = 0.0
        ke[self_mask] = 0.0
        zi[s:s + bs] = w.sum(axis=1)
        frep[s:s + bs] = np.einsum("bj,bjc->bc", w * w, d)
        fent[s:s + bs] = np.einsum("bj,bjc->bc", ke, d)
    return zi, frep, fent


def attraction(X: np.ndarray, rowptr, col, val, rows=None) -> np.ndarray:
    """F_attr,i = sum_j p_ij w_ij (X_i - X_j) over the sparse support (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.zeros((rows.shape[0], 2))
    for t, i in enumerate(rows):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        j = col[a:b]
        d = X[i] - X[j]
        w = 1.0 / (1.0 + (d * d).sum(axis=1))
        out[t] = ((val[a:b] * w)[:, None] * d).sum(axis=0)
    return out


def attraction_all(X: np.ndarray, rowptr, col, val) -> np.ndarray:
    """Vectorised F_attr for every row (same sums as ``attraction``)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    d = X[rows] - X[col]
    w = 1.0 / (1.0 + (d * d).sum(axis=1))
    contrib = (val * w)[:, None] * d
    out = np.zeros((n, 2))
    np.add.at(out, rows, contrib)
    return out


@dataclass
class GradTerms:
    F_attr: np.ndarray   # [n, 2]
    F_rep: np.ndarray    # [n, 2]
    F_ent: np.ndarray    # [n, 2]
    Z_i: np.ndarray      # [n]
    Z: np.ndarray        # [G] per graph
    G: np.ndarray        # [n, 2]


def grad_terms(X, P, params: CostParams = CostParams(), graph_offsets=None) -> GradTerms:
    """All terms of dC/dX at X for every graph of the batch (exact, FP64).

    ``P`` is any object with ``rowptr``, ``col``, ``val`` (global vertex ids).
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    offs = np.array([0, n]) if graph_offsets is None else np.asarray(graph_offsets)
    fattr = attraction_all(X, P.rowptr, P.col, P.val)
    frep = np.zeros((n, 2))
    fent = np.zeros((n, 2))
    zi = np.zeros(n)
    Z = np.zeros(offs.shape[0] - 1)
    G = np.zeros((n, 2))
    for g in range(offs.shape[0] - 1):
        a, b = int(offs[g]), int(offs[g + 1])
        ng = b - a
        if ng == 0:
            continue
        zi[a:b], frep[a:b], fent[a:b] = pair_sums(X[a:b], params.eps_r)
        Z[g] = zi[a:b].sum()
        rep_over_z = frep[a:b] / Z[g] if Z[g] > 0 else np.zeros((ng, 2))
        G[a:b] = (4.0 * params.lambda_kl * (fattr[a:b] - rep_over_z)
                  + (params.lambda_c / ng) * X[a:b]
                  - (params.lambda_r / (ng * ng)) * fent[a:b])
    return GradTerms(fattr, frep, fent, zi, Z, G)


def assemble(fattr, frep, fent, X, Z: float, n: int, params: CostParams = CostParams()):
    """dC/dX_i from its terms for rows of one graph with n vertices and normaliser Z."""
    X = np.asarray(X, dtype=np.float64)
    rep_over_z = frep / Z if Z > 0 else np.zeros_like(frep)
    return (4.0 * params.lambda_kl * (fattr - rep_over_z) + (params.lambda_c / n) * X
            - (params.lambda_r / (n * n)) * fent)


@dataclass
class CostTerms:
    kl: np.ndarray
    cmp: np.ndarray
    ent: np.ndarray

    @property
    def total(self) -> np.ndarray:
        return self.kl + self.cmp + self.ent


def cost_terms(X, P, params: CostParams = CostParams(), graph_offsets=None,
               entropy: str = "kernel") -> CostTerms:
    """C_KL, C_CMP, C_ENT of Eq. (1) per graph (exact, FP64)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    offs = np.array([0, n]) if graph_offsets is None else np.asarray(graph_offsets)
    G = offs.shape[0] - 1
    kl, cmp_, ent = np.zeros(G), np.zeros(G), np.zeros(G)
    rows = np.repeat(np.arange(n), np.diff(P.rowptr))
    for g in range(G):
        a, b = int(offs[g]), int(offs[g + 1])
        ng = b - a
        if ng == 0:
            continue
        Xg = X[a:b]
        zsum, lnsum = 0.0, 0.0
        bs = _row_block(ng)
        for s in range(0, ng, bs):
            d = Xg[s:s + bs, None, :] - Xg[None, :, :]
            r2 = d[..., 0] ** 2 + d[..., 1] ** 2
            off = np.ones_like(r2, dtype=bool)
            idx = np.arange(s, min(s + bs, ng))
            off[idx - s, idx] = False
            zsum += (1.0 / (1.0 + r2))[off].sum()
            if entropy == "kernel":
                lnsum += np.log(params.eps_r + r2[off]).sum()
            elif entropy == "literal":
                lnsum += np.log(np.sqrt(r2[off]) + params.eps_r).sum()
            else:
                raise ValueError(entropy)
        sel = (rows >= a) & (rows < b) & (P.val > 0)
        i, j, p = rows[sel], P.col[sel], P.val[sel]
        dd = X[i] - X[j]
        w = 1.0 / (1.0 + (dd * dd).sum(axis=1))
        if zsum > 0:
            kl[g] = params.lambda_kl * np.sum(p * np.log(p * zsum / w))
        cmp_[g] = params.lambda_c / (2.0 * ng) * np.sum(Xg * Xg)
        if entropy == "kernel":
            ent[g] = -params.lambda_r / (4.0 * ng * ng) * lnsum
        else:
            ent[g] = -params.lambda_r / (2.0 * ng * ng) * lnsum
    return CostTerms(kl, cmp_, ent)


def normaliser(X, rows=None) -> float:
    """Z = sum_{k!=l} w_kl for one graph (exact, FP64)."""
    zi, _, _ = pair_sums(X, 1.0, rows)
    return float(zi.sum())


def fd_delta_cost(X, P, params: CostParams, i: int, axis: int, h: float, Z: float,
                  graph_range=None, psum: float = 1.0) -> float:
    """C(X + h e) - C(X - h e) for e the unit vector of coordinate (i, axis).

    Only the pairs that involve vertex i change, so the difference is summed
    pair by pair, each written without cancellation:
      r_+^2 - r_-^2 = 4 h (X_i - X_j)_axis for every j,
      ln w_+ - ln w_- = -log1p((r_+^2 - r_-^2) / (1 + r_-^2)),
      w_+ - w_- = -w_+ w_- (r_+^2 - r_-^2),
    and Z(X - h e) = Z + 2 sum_j (w_- - w). ``Z`` is the normaliser at X (one
    O(n^2) sum shared by all coordinates) and ``psum`` the sum of p over the
    graph (1 up to rounding). P is symmetric, so the entries (i, j) and (j, i)
    of the support contribute equally. Uses the kernel entropy form.
    """
    X = np.asarray(X, dtype=np.float64)
    a, b = (0, X.shape[0]) if graph_range is None else graph_range
    n = b - a
    Xg = X[a:b]
    li = i - a
    d = Xg[li] - Xg                                   # X_i - X_j at X
    mask = np.ones(n, dtype=bool)
    mask[li] = False
    dm = d.copy()
    dm[:, axis] -= h
    dp = d.copy()
    dp[:, axis] += h
    r2 = (d * d).sum(axis=1)
    r2m = (dm * dm).sum(axis=1)
    r2p = (dp * dp).sum(axis=1)
    diff = 4.0 * h * d[:, axis]                       # r_+^2 - r_-^2
    wp, wm, w0 = 1.0 / (1.0 + r2p), 1.0 / (1.0 + r2m), 1.0 / (1.0 + r2)
    z_minus = Z + 2.0 * np.sum(((-wm * w0) * (r2m - r2))[mask])
    dz = 2.0 * np.sum((-wp * wm * diff)[mask])        # Z(+) - Z(-)
    ra, rb = int(P.rowptr[i]), int(P.rowptr[i + 1])
    cols = P.col[ra:rb].astype(np.int64) - a
    pv = P.val[ra:rb]
    dlnw = -np.log1p(diff[cols] / (1.0 + r2m[cols]))  # ln w_+ - ln w_-
    d_kl = params.lambda_kl * (-2.0 * np.sum(pv * dlnw) + psum * np.log1p(dz / z_minus))
    d_cmp = params.lambda_c / (2.0 * n) * 4.0 * h * Xg[li, axis]
    d_ent = -params.lambda_r / (4.0 * n * n) * 2.0 * np.sum(
        np.log1p(diff / (params.eps_r + r2m))[mask])
    return float(d_kl + d_cmp + d_ent)
