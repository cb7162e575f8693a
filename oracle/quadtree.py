"""Quadtree (Barnes-Hut) approximation of the repulsion and entropy sums (oracle side).

BH-tsNET (Algorithm 1, Sec. 3.1) computes the repulsive part of the KL
gradient with the quadtree of BH-SNE (Sec. 2.2), and both BH-tsNET and
FIt-tsNET (Algorithm 2, Sec. 3.2) compute the entropy gradient with a
quadtree: a node N whose points are far enough from X_i stands for all of
them, at its centre of mass with its point count as weight (Eq. 7). The
paper gives neither the tree nor the test for "far enough"; the readings
below are this project's, shared with the GPU path. Per graph [a, b):

1. Tree. x0, y0 = the smallest coordinates; side = max(x_max - x0, y_max - y0)
   in FP64 from the FP32 coordinates (1 if it is 0). Each point gets the cell
   q = min(2^32 - 1, floor((x - x0) * 2^32 / side)) per axis, computed in
   FP64 one operation at a time; its 64-bit code interleaves the bits of qy
   and qx (2 bits per level, y above x, level 1 first). Points are ordered by
   (code, id). The root holds all points at level 0; a node with more than
   one point below level 32 has one child per non-empty next 2-bit digit, in
   digit order. Nodes with one point, or at level 32, are leaves. (32 levels
   keep leaves small when a few far points stretch the square: then the bulk
   of the layout covers a tiny corner of it.) A node of
   level l has width w = side / 2^l, and its centre of mass is the FP64 mean
   of its points.
2. Traversal for point i, depth first from the root in child order: a leaf
   contributes its points one by one (i itself left out); an inner node with
   w^2 < theta^2 ||X_i - c||^2 contributes its point count times the terms
   at its centre of mass c and is not opened; other inner nodes are opened.
   theta is at most 0.7, so a node holding i is never a summary.
3. Terms at distance d = X_i - X (a point or a centre), r2 = ||d||^2:
   z = 1 / (1 + r2); F_rep += z^2 d; F_ent += d / (eps + r2);
   L += ln(eps + r2) (the cost's entropy sum). All in FP64.

Library primitives: numpy's lexicographic sort. Everything else is written
out below.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LEVELS = 32
THETA_MAX = 0.7


@dataclass
class Node:
    level: int
    start: int          # first position in the graph's sorted order
    count: int
    cx: float
    cy: float
    children: list


def _codes(X64: np.ndarray):
    x0, y0 = X64[:, 0].min(), X64[:, 1].min()
    side = max(X64[:, 0].max() - x0, X64[:, 1].max() - y0)
    if not side > 0:
        side = 1.0
    scale = float(1 << LEVELS) / side
    lim = float((1 << LEVELS) - 1)
    qx = np.minimum(np.floor((X64[:, 0] - x0) * scale), lim).astype(np.uint64)
    qy = np.minimum(np.floor((X64[:, 1] - y0) * scale), lim).astype(np.uint64)
    code = np.zeros(len(X64), dtype=np.uint64)
    one = np.uint64(1)
    for b in range(LEVELS):        # bit b of each axis -> digit LEVELS-1-b of the code
        code |= ((qy >> np.uint64(b)) & one) << np.uint64(2 * b + 1)
        code |= ((qx >> np.uint64(b)) & one) << np.uint64(2 * b)
    return code, side


def build(X) -> tuple:
    """The tree of one graph's layout: (root, order, codes in order, side)."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    code, side = _codes(X64)
    order = np.lexsort((np.arange(len(code)), code))
    sc = code[order]
    pts = X64[order]

    def make(level: int, s: int, e: int) -> Node:
        node = Node(level, s, e - s, float(pts[s:e, 0].mean()), float(pts[s:e, 1].mean()), [])
        if e - s > 1 and level < LEVELS:
            shift = 2 * (LEVELS - level - 1)
            digits = (sc[s:e] >> np.uint64(shift)) & np.uint64(3)
            for d in range(4):
                idx = np.nonzero(digits == d)[0]
                if idx.size:
                    node.children.append(make(level + 1, s + int(idx[0]), s + int(idx[-1]) + 1))
        return node

    return make(0, 0, len(code)), order, sc, side


def _terms(dx, dy, eps, cnt, acc):
    r2 = dx * dx + dy * dy
    z = 1.0 / (1.0 + r2)
    u = 1.0 / (eps + r2)
    acc[0] += cnt * z
    acc[1] += cnt * z * z * dx
    acc[2] += cnt * z * z * dy
    acc[3] += cnt * u * dx
    acc[4] += cnt * u * dy
    acc[5] += cnt * np.log(eps + r2)


def sums(X, theta: float = 0.5, eps: float = 0.05, graph_offsets=None, rows=None):
    """Per vertex (z_i, F_rep,i, F_ent,i, L_i) by the quadtree rule, FP64.
    With rows (vertex ids), only those vertices are evaluated (others stay 0)."""
    if not 0.0 < theta <= THETA_MAX:
        raise ValueError("theta must be in (0, 0.7]")
    X = np.asarray(X, dtype=np.float32)
    n = X.shape[0]
    off = np.array([0, n]) if graph_offsets is None else np.asarray(graph_offsets, np.int64)
    zi = np.zeros(n)
    frep = np.zeros((n, 2))
    fent = np.zeros((n, 2))
    lnv = np.zeros(n)
    th2 = theta * theta
    want = None if rows is None else set(int(r) for r in rows)
    for g in range(len(off) - 1):
        a, b = int(off[g]), int(off[g + 1])
        if want is not None and not any(a <= r < b for r in want):
            continue
        root, order, _, side = build(X[a:b])
        pts = X[a:b].astype(np.float64)[order]
        for p in range(b - a):
            if want is not None and a + int(order[p]) not in want:
                continue
            xi, yi = pts[p]
            acc = [0.0] * 6
            stack = [root]
            while stack:
                nd = stack.pop()
                if not nd.children:                      # leaf: its points one by one
                    for q in range(nd.start, nd.start + nd.count):
                        if q != p:
                            _terms(xi - pts[q, 0], yi - pts[q, 1], eps, 1.0, acc)
                    continue
                dx, dy = xi - nd.cx, yi - nd.cy
                w = side / float(1 << nd.level)
                if w * w < th2 * (dx * dx + dy * dy):
                    _terms(dx, dy, eps, float(nd.count), acc)
                else:
                    stack.extend(reversed(nd.children))  # visit in child order
            v = a + int(order[p])
            zi[v] = acc[0]
            frep[v] = acc[1:3]
            fent[v] = acc[3:5]
            lnv[v] = acc[5]
    return zi, frep, fent, lnv
