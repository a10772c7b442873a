"""Training data for the fitting workload: an analytic torus SDF.

Torus with axis z, major radius R = 0.5 and minor radius r = 0.2:
    sdf(x) = sqrt((sqrt(x^2 + y^2) - R)^2 + z^2) - r.
Surface points are area-uniform: u ~ U[0, 2 pi) and v drawn by rejection with
density proportional to R + r cos v (the torus area element), with analytic unit
normals.  Uniform points are drawn in [-1, 1]^3 with their exact sdf.
Each fitting step uses its own stream ``default_rng([seed, step])``.
"""

import numpy as np

R_MAJOR = 0.5
R_MINOR = 0.2


def torus_sdf(x: np.ndarray, R: float = R_MAJOR, r: float = R_MINOR) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    q = np.sqrt(x[:, 0] ** 2 + x[:, 1] ** 2) - R
    return np.sqrt(q * q + x[:, 2] ** 2) - r


def torus_surface_samples(rng, n: int, R: float = R_MAJOR, r: float = R_MINOR):
    """n area-uniform surface points and their unit normals (float64)."""
    u = rng.uniform(0.0, 2.0 * np.pi, size=n)
    v = np.empty(n)
    filled = 0
    while filled < n:
        m = max(2 * (n - filled), 64)
        cand = rng.uniform(0.0, 2.0 * np.pi, size=m)
        acc = rng.uniform(0.0, R + r, size=m) < (R + r * np.cos(cand))
        take = cand[acc][: n - filled]
        v[filled:filled + take.size] = take
        filled += take.size
    cu, su, cv, sv = np.cos(u), np.sin(u), np.cos(v), np.sin(v)
    pts = np.stack([(R + r * cv) * cu, (R + r * cv) * su, r * sv], axis=1)
    nrm = np.stack([cv * cu, cv * su, sv], axis=1)
    return pts, nrm


def torus_uniform_samples(rng, n: int, lo: float = -1.0, hi: float = 1.0):
    pts = rng.uniform(lo, hi, size=(n, 3))
    return pts, torus_sdf(pts)


def torus_batch(step: int, n_surf: int, n_unif: int, seed: int = 7):
    """Float32 batch for one fitting step: (surf_x, surf_n, unif_x, unif_sdf)."""
    rng = np.random.default_rng([seed, step])
    sp, sn = torus_surface_samples(rng, n_surf)
    up, us = torus_uniform_samples(rng, n_unif)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)  # noqa: E731
    return f32(sp), f32(sn), f32(up), f32(us)
