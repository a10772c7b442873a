"""Triangle-mesh side of neural normal mapping (test infrastructure; see
oracle/__init__.py).

* ``marching_tets``  -- ctypes wrapper of ``mesh_oracle.c``: the coarse mesh
  extracted from a grid of float32 values (the extraction reading is stated in
  that file's header).
* ``unit_normals``   -- neural normal mapping onto arbitrary points (Sec. 5, the
  triangle-mesh example): the unit gradient of a finer scene function, in
  float64, from the oracle's analytic gradient.
"""

import ctypes

import numpy as np

from . import tracing as T

_ready = False


def _lib():
    global _ready
    lib = T._load()
    if not _ready:
        P = ctypes.c_void_p
        lib.orc_marching_tets.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_float, P, P,
                                          ctypes.c_int64, ctypes.c_int64, P]
        lib.orc_marching_tets.restype = ctypes.c_int
        _ready = True
    return lib


def marching_tets(values, lo, hi, iso=0.0):
    """values: float32 [res, res, res] indexed [k, j, i] (x fastest).

    Returns (verts float64 [nv, 3], tris int32 [nt, 3])."""
    v = np.ascontiguousarray(values, dtype=np.float32)
    res = v.shape[0]
    assert v.shape == (res, res, res)
    counts = np.zeros(2, np.int64)
    lib = _lib()
    rc = lib.orc_marching_tets(T._ptr(v), res, float(np.float32(lo)), float(np.float32(hi)), float(iso), None,
                               None, 0, 0, T._ptr(counts))
    if rc != 0:
        raise RuntimeError("orc_marching_tets failed")
    nv, nt = int(counts[0]), int(counts[1])
    verts = np.empty((max(nv, 1), 3))
    tris = np.empty((max(nt, 1), 3), np.int32)
    rc = lib.orc_marching_tets(T._ptr(v), res, float(np.float32(lo)), float(np.float32(hi)), float(iso),
                               T._ptr(verts), T._ptr(tris), nv, nt, T._ptr(counts))
    if rc != 0:
        raise RuntimeError("orc_marching_tets failed")
    return verts[:nv], tris[:nt]


def unit_normals(scene, level, x, t=None, threads=0):
    """grad f_level / |grad f_level| at float32 points x[n, 3] (0 where the gradient vanishes)."""
    x64 = np.asarray(x, dtype=np.float32).astype(np.float64)
    tt = None if t is None else np.asarray(t, dtype=np.float32).astype(np.float64)
    _, g = T.scene_eval(scene, level, x64, tt, grad=True, threads=threads)
    n = np.linalg.norm(g, axis=1, keepdims=True)
    return np.where(n > 0, g / np.where(n > 0, n, 1.0), 0.0)
