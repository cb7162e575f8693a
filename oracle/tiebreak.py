"""Reproducible tie-breaking for the partial BFS (oracle side).

The partial BFS stops after k vertices and breaks ties among vertices at the
same hop distance "randomly" (Sec. 3.1). A random choice cannot be compared
bit for bit, so the tie order is fixed by a counter-based hash of the pair
(source i, candidate j): smaller key first, then smaller j.

The hash is the SplitMix64 output function (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), applied twice:
key(i, j) = mix(seed XOR mix(i * 2^32 + j)). With ``mode == "id"`` the key is
simply j, which makes hand-checked cases easy.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
TIE_HASH = "hash"
TIE_ID = "id"


def mix64(z: int) -> int:
    """SplitMix64 finaliser on a Python int (reference form, one value)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def mix64_array(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser over a uint64 array (wrap-around products)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def tie_keys(i: int, js: np.ndarray, seed: int, mode: str = TIE_HASH) -> np.ndarray:
    """uint64 tie keys of candidates ``js`` seen from source ``i``."""
    js = np.asarray(js, dtype=np.int64)
    if mode == TIE_ID:
        return js.astype(np.uint64)
    if mode != TIE_HASH:
        raise ValueError(f"unknown tie mode {mode!r}")
    counter = (np.uint64(i) << np.uint64(32)) | js.astype(np.uint64)
    return mix64_array(np.uint64(seed & MASK64) ^ mix64_array(counter))
