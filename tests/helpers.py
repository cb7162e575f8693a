"""Shared helpers of the GPU parity tests (inputs and error measures only)."""
from __future__ import annotations

import sys

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def say(*args):
    """Print and flush, so a failing GPU step names its case."""
    print(*args, flush=True)
    sys.stdout.flush()


def f32_round(P):
    """Host CSR (rowptr, col, FP32 values) of an oracle P for tsnet_P_from_host."""
    return P.rowptr, P.col, P.val.astype(np.float32)


class P32:
    """The same P with FP32-rounded values, as the GPU sees it (FP64 arithmetic)."""

    def __init__(self, P):
        self.rowptr = P.rowptr
        self.col = P.col
        self.val = P.val.astype(np.float32).astype(np.float64)


def ulp_diff(a32, b64):
    """Distance in FP32 ulps between GPU values and the oracle's FP64 values."""
    b32 = np.asarray(b64).astype(np.float32)
    ai = np.asarray(a32, dtype=np.float32).view(np.int32).astype(np.int64)
    bi = b32.view(np.int32).astype(np.int64)
    return np.abs(ai - bi)
