"""Regular grids of sample points.

Node (i, j, k) of a res^3 grid over [lo, hi]^3 sits at coordinates
float32(lo + (hi - lo) i / (res - 1)) (evaluated in float64, left to right, and
rounded once), with linear index (k res + j) res + i -- x fastest.  The
library's grid evaluator computes the same coordinates on the device.
"""

import numpy as np


def grid_axis(res: int, lo: float, hi: float) -> np.ndarray:
    lo64, hi64 = np.float64(np.float32(lo)), np.float64(np.float32(hi))
    i = np.arange(res, dtype=np.float64)
    return (lo64 + (hi64 - lo64) * i / np.float64(res - 1)).astype(np.float32)


def grid_nodes(res: int, lo: float, hi: float) -> np.ndarray:
    """float32 [res^3, 3] node coordinates in linear-index order."""
    a = grid_axis(res, lo, hi)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
