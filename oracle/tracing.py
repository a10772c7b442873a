"""ctypes wrapper of the C oracle (test infrastructure; see oracle/__init__.py).

Scenes come from ``nnm_inputs`` (levels with SIREN weights, amplitudes, deltas).
Levels are 0-based.  All results are float64 numpy arrays.
"""

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int64, c_uint8

import numpy as np

from .build import build_oracle, oracle_lib_path

ST_HIT, ST_FAR, ST_BUDGET, ST_NEG_STEP, ST_NONFINITE = 1, 2, 4, 8, 16


class _LevelDesc(ctypes.Structure):
    _fields_ = [("d_in", c_int), ("width", c_int), ("n_sine", c_int), ("follow_center", c_int),
                ("amplitude", c_double), ("delta", c_double), ("params", POINTER(c_float))]


class _BaseDesc(ctypes.Structure):
    _fields_ = [("sphere", c_int), ("r0", c_double), ("rho", c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = oracle_lib_path()
        if not os.path.exists(path):
            build_oracle()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.orc_max_threads.restype = c_int
        lib.orc_net_eval.argtypes = [c_int, c_int, c_int, P, c_int64, P, P, P, c_int]
        lib.orc_scene_eval.argtypes = [P, P, c_int64, P, P, P, P, c_int]
        lib.orc_trace.argtypes = [c_int, P, P, c_double, c_double, c_double, c_int, c_int, c_int,
                                  c_int64, P, P, P, P, P, P, P, P, c_int]
        lib.orc_trace_iters.argtypes = [c_int, P, P, c_double, c_double, c_double, c_int, P, c_int, c_int,
                                        c_int64, P, P, P, P, P, P, P, P, c_int]
        lib.orc_trace_log.argtypes = [c_int, P, P, c_double, c_double, c_double, c_int, c_int, P, P,
                                      c_double, c_int, P, P, P, P, P]
        lib.orc_first_root.argtypes = [P, P, c_int64, P, P, P, c_double, c_double, c_double, c_double,
                                       P, c_int]
        for f in (lib.orc_net_eval, lib.orc_scene_eval, lib.orc_trace, lib.orc_trace_iters, lib.orc_trace_log,
                  lib.orc_first_root):
            f.restype = c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return _load().orc_max_threads()


class _Levels:
    """Keeps the float32 parameter arrays alive while the C descriptors are used."""

    def __init__(self, levels):
        self.params = [np.ascontiguousarray(l.net.flat(), dtype=np.float32) for l in levels]
        arr = (_LevelDesc * len(levels))()
        for j, l in enumerate(levels):
            arr[j].d_in = l.net.d_in
            arr[j].width = l.net.width
            arr[j].n_sine = l.net.n_sine
            arr[j].follow_center = int(bool(l.follow_center))
            arr[j].amplitude = float(l.amplitude)
            arr[j].delta = float(l.delta)
            arr[j].params = self.params[j].ctypes.data_as(POINTER(c_float))
        self.arr = arr
        self.m = len(levels)

    def ptr(self, j=0):
        return ctypes.cast(ctypes.byref(self.arr, j * ctypes.sizeof(_LevelDesc)), ctypes.c_void_p)


def _base(scene):
    b = _BaseDesc()
    b.sphere = 1 if scene.base_sphere else 0
    b.r0 = float(scene.r0)
    b.rho = float(scene.rho)
    return b


def net_eval(net, x, grad=True, threads=0):
    """Raw SIREN N(x) and grad N (spatial) at x[n, d_in] (float64 inputs)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    params = np.ascontiguousarray(net.flat(), dtype=np.float32)
    val = np.empty(n)
    g = np.empty((n, 3)) if grad else None
    rc = _load().orc_net_eval(net.d_in, net.width, net.n_sine, _ptr(params), n, _ptr(x), _ptr(val),
                              _ptr(g), threads)
    if rc != 0:
        raise RuntimeError(f"orc_net_eval failed ({rc})")
    return (val, g) if grad else val


def scene_eval(scene, level, x, t=None, grad=True, threads=0):
    """f_level and grad_x f_level at x[n, 3] (times t[n] or None)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    lv = _Levels([scene.levels[level]])
    tt = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
    val = np.empty(n)
    g = np.empty((n, 3)) if grad else None
    base = _base(scene)
    rc = _load().orc_scene_eval(lv.ptr(0), ctypes.cast(ctypes.byref(base), ctypes.c_void_p), n, _ptr(x),
                                _ptr(tt), _ptr(val), _ptr(g), threads)
    if rc != 0:
        raise RuntimeError(f"orc_scene_eval failed ({rc})")
    return (val, g) if grad else val


def trace(scene, o, v, t=None, final_level=None, normal_level=None, want_normal=True, threads=0,
          iterations=None):
    """Multiscale sphere tracing of the rays (Algorithm 1) with normals.

    ``iterations``: None for eps-terminated tracing, else the number of steps
    of each traced level (fixed-iteration mode, as in the paper's experiments).
    Returns dict(depth, hit, normal, steps[n, m], status)."""
    m = len(scene.levels)
    final_level = m - 1 if final_level is None else final_level
    normal_level = final_level if normal_level is None else normal_level
    o = np.ascontiguousarray(o, dtype=np.float32)
    v = np.ascontiguousarray(v, dtype=np.float32)
    tt = None if t is None else np.ascontiguousarray(t, dtype=np.float32)
    n = o.shape[0]
    lv = _Levels(scene.levels)
    base = _base(scene)
    depth = np.empty(n)
    hit = np.empty(n, np.uint8)
    normal = np.empty((n, 3)) if want_normal else None
    steps = np.empty((n, m), np.uint8)
    status = np.empty(n, np.uint8)
    its = None
    if iterations is not None:
        its = np.zeros(8, np.int32)
        its[:len(iterations)] = iterations
    rc = _load().orc_trace_iters(m, lv.ptr(0), ctypes.cast(ctypes.byref(base), ctypes.c_void_p),
                                 scene.step_scale, scene.eps, scene.far, scene.max_steps, _ptr(its),
                                 final_level, normal_level, n, _ptr(o), _ptr(v), _ptr(tt), _ptr(depth),
                                 _ptr(hit), _ptr(normal), _ptr(steps), _ptr(status), threads)
    if rc != 0:
        raise RuntimeError(f"orc_trace failed ({rc})")
    return {"depth": depth, "hit": hit, "normal": normal, "steps": steps, "status": status}


def trace_log(scene, o, v, t=0.0, final_level=None, cap=4096):
    """Step log of one ray: (tau_before[k], d[k], level[k], tau_end, status)."""
    m = len(scene.levels)
    final_level = m - 1 if final_level is None else final_level
    lv = _Levels(scene.levels)
    base = _base(scene)
    o = np.ascontiguousarray(o, dtype=np.float32).reshape(3)
    v = np.ascontiguousarray(v, dtype=np.float32).reshape(3)
    lt = np.empty(cap)
    ld = np.empty(cap)
    ll = np.empty(cap, np.int32)
    tau = np.empty(1)
    st = np.empty(1, np.int32)
    k = _load().orc_trace_log(m, lv.ptr(0), ctypes.cast(ctypes.byref(base), ctypes.c_void_p),
                              scene.step_scale, scene.eps, scene.far, scene.max_steps, final_level,
                              _ptr(o), _ptr(v), float(t), cap, _ptr(lt), _ptr(ld), _ptr(ll), _ptr(tau),
                              _ptr(st))
    if k < 0:
        raise RuntimeError(f"orc_trace_log failed ({k})")
    return lt[:k], ld[:k], ll[:k], float(tau[0]), int(st[0])


def first_root(scene, level, o, v, t=None, lip=1.03, h_min=1e-6, tol=1e-13, threads=0):
    """Brute-force first zero crossing of f_level along each ray (+inf if none)."""
    o = np.ascontiguousarray(o, dtype=np.float32)
    v = np.ascontiguousarray(v, dtype=np.float32)
    tt = None if t is None else np.ascontiguousarray(t, dtype=np.float32)
    n = o.shape[0]
    lv = _Levels([scene.levels[level]])
    base = _base(scene)
    root = np.empty(n)
    rc = _load().orc_first_root(lv.ptr(0), ctypes.cast(ctypes.byref(base), ctypes.c_void_p), n, _ptr(o),
                                _ptr(v), _ptr(tt), scene.far, lip, h_min, tol, _ptr(root), threads)
    if rc != 0:
        raise RuntimeError(f"orc_first_root failed ({rc})")
    return root
