"""Conditional probabilities p_{j|i} calibrated to a perplexity (oracle side).

Eq. (3): p_{j|i} = exp(-d_ij^2 / (2 sigma_i^2)) / sum_k exp(-d_ik^2 / (2 sigma_i^2)),
with sigma_i chosen so that the perplexity 2^{H_2(P_i)} equals u. As in the
sparse t-SNE the method builds on (Sec. 2.2), the sums run over the selected
neighbours N_k(i) only, and d is the hop distance.

Written with beta = 1 / (2 sigma^2) and with the row grouped into distance
levels (d_l, c_l): the shift delta_l = d_l^2 - d_1^2 cancels in the ratio, so

    S(beta) = sum_l c_l exp(-beta delta_l),    A(beta) = sum_l c_l delta_l exp(-beta delta_l)
    H(beta) = ln S + beta A / S                (entropy in nats; target ln u)

H falls monotonically from ln K (beta = 0, K = |N_k(i)|) to ln c_1
(beta -> inf). Rows whose target lies outside that range cannot reach the
perplexity; they take the limiting distribution and a status flag:

* LOW  (one level, or u >= K):   beta = 0, uniform over the row;
* HIGH (u <= c_1):               beta = inf, uniform over level 1, zero elsewhere;
* EMPTY (isolated vertex):       no entries.

Otherwise beta is found by bisection: beta_hi doubles from 1 until
H(beta_hi) < ln u, then [0, beta_hi] is halved until its width is at most
1e-14 * beta_hi or 200 halvings are done; beta is the final midpoint.
"""
from __future__ import annotations

import math

import numpy as np

STATUS_OK = 0
STATUS_LOW = 1
STATUS_HIGH = 2
STATUS_EMPTY = 3

BISECT_RTOL = 1e-14
BISECT_MAX_STEPS = 200


def level_histogram(dist: np.ndarray):
    """Distinct hop distances of a row and their counts, ascending."""
    levels, counts = np.unique(np.asarray(dist, dtype=np.int64), return_counts=True)
    return levels, counts


def entropy_of_beta(beta: float, deltas: np.ndarray, counts: np.ndarray) -> float:
    """H(beta) in nats over a level histogram."""
    e = np.exp(-beta * deltas)
    s = float(np.sum(counts * e))
    a = float(np.sum(counts * deltas * e))
    return math.log(s) + beta * a / s


def solve_beta(levels: np.ndarray, counts: np.ndarray, perplexity: float):
    """(beta, status) for one row's level histogram."""
    total = int(np.sum(counts))
    if total == 0:
        return 0.0, STATUS_EMPTY
    if levels.shape[0] == 1 or perplexity >= total:
        return 0.0, STATUS_LOW
    if perplexity <= counts[0]:
        return math.inf, STATUS_HIGH
    deltas = levels.astype(np.float64) ** 2 - float(levels[0]) ** 2
    target = math.log(perplexity)
    hi = 1.0
    while entropy_of_beta(hi, deltas, counts) >= target:
        hi *= 2.0
    lo = 0.0
    for _ in range(BISECT_MAX_STEPS):
        if hi - lo <= BISECT_RTOL * hi:
            break
        mid = 0.5 * (lo + hi)
        if entropy_of_beta(mid, deltas, counts) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi), STATUS_OK


def row_probabilities(dist: np.ndarray, perplexity: float):
    """(p_{j|i} FP64 aligned with ``dist``, beta, status) for one row."""
    dist = np.asarray(dist, dtype=np.int64)
    if dist.shape[0] == 0:
        return np.zeros(0), 0.0, STATUS_EMPTY
    levels, counts = level_histogram(dist)
    beta, status = solve_beta(levels, counts, perplexity)
    if status == STATUS_LOW:
        return np.full(dist.shape[0], 1.0 / dist.shape[0]), beta, status
    if status == STATUS_HIGH:
        p = np.where(dist == levels[0], 1.0 / counts[0], 0.0)
        return p, beta, status
    deltas = levels.astype(np.float64) ** 2 - float(levels[0]) ** 2
    s = float(np.sum(counts * np.exp(-beta * deltas)))
    d2 = dist.astype(np.float64) ** 2 - float(levels[0]) ** 2
    return np.exp(-beta * d2) / s, beta, status
