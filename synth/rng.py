"""Counter-based SplitMix64 streams (Steele, Lea & Flood 2014), vectorised in numpy.

Value i of a stream with key s is the SplitMix64 output mixer applied to
s + (i + 1) * 0x9E3779B97F4A7C15 (mod 2**64).  Uniform doubles take the top 53 bits:
u = (z >> 11) * 2**-53, so u lies in [0, 1).

Every seeded input of the package (point clouds, physical fields, model counts) is
drawn from these streams, so a (seed, tag) pair names one input exactly.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64(key: int, start: int, n: int) -> np.ndarray:
    """Outputs start .. start+n-1 of the stream with 64-bit key ``key``."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(key & 0xFFFFFFFFFFFFFFFF) + ctr * _GOLDEN
        return _mix(z)


def stream_key(seed: int, tag: str) -> int:
    """Derive an independent 64-bit key from a seed and a text tag."""
    h = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for ch in tag.encode():
            h = _mix(np.array([h ^ np.uint64(ch)], dtype=np.uint64))[0]
    return int(h)


class Stream:
    """A sequential reader over one SplitMix64 stream."""

    def __init__(self, seed: int, tag: str):
        self.key = stream_key(seed, tag)
        self.pos = 0

    def bits(self, n: int) -> np.ndarray:
        out = splitmix64(self.key, self.pos, n)
        self.pos += n
        return out

    def uniform(self, n: int) -> np.ndarray:
        return (self.bits(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, n: int) -> np.ndarray:
        """Box-Muller pairs; 1 - u keeps the logarithm finite."""
        m = (n + 1) // 2
        u1 = 1.0 - self.uniform(m)
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
        return z[:n]
