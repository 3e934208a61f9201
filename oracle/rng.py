"""Oracle: splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), written from its published definition.
Test infrastructure only.

One step on a 64-bit input x:
    z = x + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    return z ^ (z >> 31)                       (all mod 2^64)
It is used as a counter-based generator: value i of stream `seed` is
splitmix64(seed XOR i), mapped to [0, 1) by (z >> 11) * 2^-53.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def uniform01(seed: int, n: int) -> np.ndarray:
    """u[i] = (splitmix64(seed ^ i) >> 11) * 2^-53 for i < n (pure Python ints)."""
    out = np.empty(n)
    for i in range(n):
        out[i] = (splitmix64(seed ^ i) >> 11) * 2.0 ** -53
    return out


def splitmix64_vec(seed: int, n: int) -> np.ndarray:
    """splitmix64(seed ^ i) for i < n as uint64 (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.bitwise_xor(np.uint64(seed), np.arange(n, dtype=np.uint64))
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform01_vec(seed: int, n: int) -> np.ndarray:
    """Same values as `uniform01`, vectorised with wrapping uint64 arithmetic."""
    return (splitmix64_vec(seed, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
