"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) and the bath-vector rule built on it.

Test infrastructure only (see ``oracle/__init__``).

``sm64(x)`` is one SplitMix64 output taken from state ``x``: add the golden
gamma 0x9E3779B97F4A7C15, then apply the published 64-bit finaliser (xor-shift
30, multiply 0xBF58476D1CE4E5B9, xor-shift 27, multiply 0x94D049BB133111EB,
xor-shift 31).  A generator seeded with 0 therefore yields sm64(0) first.

Bath vector rule (the estimator's random start vectors, Section "Block
stochastic Lanczos quadrature"; real Rademacher entries normalised to unit
norm, so that the expectation of v v^T is I/d_b):

    key_j  = sm64(seed XOR sm64(j))
    word   = sm64(key_j XOR (b >> 6))
    bit    = (word >> (b & 63)) & 1
    v_j[b] = (1 - 2*bit) * sqrt(2^-n_b)
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def sm64(x: int) -> int:
    """One SplitMix64 output from state x (pure Python integers)."""
    z = (x + GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def sm64_stream(seed: int, n: int):
    """The first n outputs of a SplitMix64 generator seeded with ``seed``."""
    out = []
    s = seed & MASK64
    for _ in range(n):
        out.append(sm64(s))
        s = (s + GAMMA) & MASK64
    return out


def _sm64_np(x: np.ndarray) -> np.ndarray:
    """Vectorised sm64 over a uint64 array (wrap-around arithmetic)."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        return z ^ (z >> np.uint64(31))


def bath_key(seed: int, j: int) -> int:
    return sm64((seed & MASK64) ^ sm64(j))


def rademacher_signs(seed: int, j: int, n_b: int) -> np.ndarray:
    """Signs (+1/-1 as int8) of bath vector j over the 2^n_b bath basis states."""
    d_b = 1 << n_b
    key = np.uint64(bath_key(seed, j))
    b = np.arange(d_b, dtype=np.uint64)
    words = _sm64_np(key ^ (b >> np.uint64(6)))
    bits = (words >> (b & np.uint64(63))) & np.uint64(1)
    return (1 - 2 * bits.astype(np.int64)).astype(np.int8)


def bath_vector(seed: int, j: int, n_b: int) -> np.ndarray:
    """Unit-norm real Rademacher bath vector v_j (FP64)."""
    return rademacher_signs(seed, j, n_b).astype(np.float64) * np.sqrt(2.0 ** (-n_b))


def bath_vectors(seed: int, n_v: int, n_b: int) -> np.ndarray:
    """(d_b, n_v) matrix whose columns are v_0..v_{n_v-1}."""
    return np.stack([bath_vector(seed, j, n_b) for j in range(n_v)], axis=1)
