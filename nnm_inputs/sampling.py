"""Counter-based sampling of box points (splitmix64).

The same sequence as the library's device sampler for nesting thresholds
(nnm_sup_abs_diff): splitmix64 (Steele, Lea and Flood, 2014, with Vigna's
published finaliser) at stream position k = 4 i + c for coordinate c of point
i, u = top 24 bits / 2^24, x_c = float32(lo + (hi - lo) u) evaluated in float64,
and t = float32(u) of c = 3.  Reproduced here, from that definition, so tests
can evaluate the very points the device drew.
"""

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_at(seed: int, k: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def box_points(seed: int, n: int, lo: float, hi: float, first: int = 0):
    """Points first .. first+n-1 of the sequence: (x [n, 3] float32, t [n] float32)."""
    i = np.arange(first, first + n, dtype=np.uint64)
    u = [(splitmix64_at(seed, np.uint64(4) * i + np.uint64(c)) >> np.uint64(40)).astype(np.float64) / 16777216.0
         for c in range(4)]
    lo64, hi64 = np.float64(np.float32(lo)), np.float64(np.float32(hi))
    x = np.stack([(lo64 + (hi64 - lo64) * u[c]).astype(np.float32) for c in range(3)], axis=1)
    return np.ascontiguousarray(x), u[3].astype(np.float32)
