"""The vertex move of the gradient loop, in FP64 (oracle side).

Algorithm 3 ends each iteration by moving every vertex along the gradient of C;
the paper names no optimiser. Reading: the standard t-SNE update with momentum
and per-coordinate gains (van der Maaten and Hinton, JMLR 2008), which the
t-SNE codes the method builds on use:

    gains <- gains + 0.2   where sign(g) differs from sign(update)
             gains * 0.8   elsewhere,       then floored at min_gain (0.01)
    update <- mu_t * update - eta * gains * g
    X      <- X + update

with mu_t = 0.5 for t < 250 and 0.8 afterwards, and eta = max(200, n / 12) per
graph (the n/12 rule of Belkina et al., Nat. Commun. 2019). "sign differs" is
(g > 0) != (update > 0), evaluated per coordinate.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class StepParams:
    eta: float = 0.0              # <= 0 selects max(200, n/12) per graph
    momentum_early: float = 0.5
    momentum_late: float = 0.8
    momentum_switch_iter: int = 250
    min_gain: float = 0.01
    gain_up: float = 0.2
    gain_down: float = 0.8


def learning_rate(n: int, sp: StepParams) -> float:
    return sp.eta if sp.eta > 0 else max(200.0, n / 12.0)


def step(X, update, gains, G, it: int, sp: StepParams = StepParams(), graph_offsets=None):
    """Return (X, update, gains) after one move; inputs are not modified."""
    X = np.array(X, dtype=np.float64)
    update = np.array(update, dtype=np.float64)
    gains = np.array(gains, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n = X.shape[0]
    offs = np.array([0, n]) if graph_offsets is None else np.asarray(graph_offsets)
    mu = sp.momentum_early if it < sp.momentum_switch_iter else sp.momentum_late
    flip = (G > 0) != (update > 0)
    gains = np.where(flip, gains + sp.gain_up, gains * sp.gain_down)
    gains = np.maximum(gains, sp.min_gain)
    eta = np.zeros((n, 1))
    for g in range(offs.shape[0] - 1):
        a, b = int(offs[g]), int(offs[g + 1])
        eta[a:b] = learning_rate(b - a, sp)
    update = mu * update - eta * gains * G
    return X + update, update, gains
