"""Pinhole camera rays (input generation for every rendering workload).

Camera: centre at (0, 0, 2.5) looking at the origin (view along -z), +y up,
vertical field of view 45 degrees, aspect = width / height, pixel centres at
(col + 1/2, row + 1/2), rays stored row major starting from the top row.
Directions are normalised in float64 and rounded once to float32; origins are
the camera centre (no near plane).
"""

import numpy as np

CAM_POS = (0.0, 0.0, 2.5)
FOV_Y_DEG = 45.0


def pinhole_rays(width: int, height: int, cam_pos=CAM_POS, fov_y_deg: float = FOV_Y_DEG,
                 rows=None):
    """Return (o[n,3], v[n,3]) float32 for a width x height image.

    ``rows`` optionally selects a subset of image rows (e.g. every k-th row);
    the rays are identical to the corresponding rays of the full image.
    """
    if width <= 0 or height <= 0:
        return np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32)
    row_idx = np.arange(height) if rows is None else np.asarray(rows, dtype=np.int64)
    tan_half = np.tan(np.deg2rad(fov_y_deg) * 0.5)
    aspect = width / height
    cols = (np.arange(width, dtype=np.float64) + 0.5) / width
    rws = (row_idx.astype(np.float64) + 0.5) / height
    px = (2.0 * cols - 1.0) * aspect * tan_half
    py = (1.0 - 2.0 * rws) * tan_half
    X, Y = np.meshgrid(px, py)  # [rows, cols]
    d = np.stack([X, Y, -np.ones_like(X)], axis=-1).reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    v = d.astype(np.float32)
    o = np.broadcast_to(np.asarray(cam_pos, np.float32), v.shape).copy()
    return np.ascontiguousarray(o), np.ascontiguousarray(v)
