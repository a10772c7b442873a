"""ctypes marshalling of libnnm's C ABI (include/nnm.h).  No computation here."""

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_void_p
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DEFAULT_LIB = os.path.join(_HERE, "libnnm.so")
_LIB_PATH = _DEFAULT_LIB

PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
ST_HIT, ST_FAR, ST_BUDGET, ST_NEG_STEP, ST_NONFINITE = 1, 2, 4, 8, 16
_ERRORS = {-1: "E_INVAL", -2: "E_FORMAT", -3: "E_NONFINITE", -4: "E_LIPSCHITZ", -5: "E_NESTING",
           -6: "E_NOMEM", -7: "E_DEVICE", -8: "E_UNSUPPORTED", -9: "E_IO"}


class NnmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _LevelDesc(ctypes.Structure):
    _fields_ = [("d_in", c_int32), ("width", c_int32), ("n_sine", c_int32), ("follow_center", c_int32),
                ("amplitude", c_float), ("delta", c_float), ("params", POINTER(c_float))]


class _StackDesc(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("base_sphere", c_int32), ("r0", c_float), ("rho", c_float),
                ("lipschitz_max", c_float), ("reserved", c_int32), ("levels", POINTER(_LevelDesc))]


class _TraceParams(ctypes.Structure):
    _fields_ = [("step_scale", c_float), ("eps", c_float), ("far", c_float), ("max_steps", c_int32),
                ("final_level", c_int32), ("normal_level", c_int32), ("mode", c_int32),
                ("kernels", c_int32), ("profiler", c_void_p), ("iterations", c_int32 * 8)]


class _RefSdf(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("a", c_float), ("b", c_float), ("reserved", c_int32)]


KERNELS = {"auto": 0, "streaming": 1}
REF_SHAPES = {"sphere": 1, "torus": 2}


_PROF_MAX = 32


class _ProfileReport(ctypes.Structure):
    _fields_ = [("n_entries", c_int32), ("kind", c_int32 * _PROF_MAX), ("level", c_int32 * _PROF_MAX),
                ("width", c_int32 * _PROF_MAX), ("launches", c_int64 * _PROF_MAX),
                ("total_ms", c_double * _PROF_MAX), ("variant", c_int32 * _PROF_MAX)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library(path: Optional[str] = None):
    """Load libnnm.so (raises NnmError when it has not been built).

    ``path`` names another build of the same library (a tuning variant); it
    must be given before the first call into the library, and a later call
    naming a different file raises."""
    global _lib, _LIB_PATH
    if path is not None and os.path.abspath(path) != os.path.abspath(_LIB_PATH):
        if _lib is not None:
            raise NnmError(-1, f"{_LIB_PATH} is already loaded; cannot switch to {path}")
        _LIB_PATH = os.path.abspath(path)
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise NnmError(-7, f"{_LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    P = c_void_p
    sig = {
        "nnm_validate_stack": ([P, c_int], c_int),
        "nnm_level_lipschitz_bound": ([P, c_int, P], c_int),
        "load_siren_stack": ([P, c_int, c_int, P], c_int),
        "free_siren_stack": ([P], None),
        "nnm_stack_levels": ([P], c_int),
        "nnm_stack_precision": ([P], c_int),
        "trace_rays": ([P, P, c_int64, P, P, P, P, P, P, P, P, P], c_int),
        "trace_rays_noalloc": ([P, P, c_int64, P, P, P, P, P, P, P, P, P], c_int),
        "analytic_normal": ([P, c_int, c_int64, P, P, P, P, P], c_int),
        "nnm_net_eval": ([P, c_int, c_int64, P, P, P, P, P], c_int),
        "nnm_sup_abs_diff": ([P, c_int, c_int, c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_float, P, P], c_int),
        "nnm_sup_abs_err": ([P, c_int, P, c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_float, P, P], c_int),
        "nnm_nesting_thresholds": ([c_int, c_int32, P, c_double, P], c_int),
        "neural_normal_map": ([P, c_int, c_int64, P, P, P, P], c_int),
        "nnm_grid_values": ([P, c_int, c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P], c_int),
        "nnm_mesh_extract": ([P, c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_int64, c_int64, P, P, P,
                              P], c_int),
        "nnm_read_net_file": ([ctypes.c_char_p, P, P, P, P, P], c_int),
        "nnm_write_net_file": ([ctypes.c_char_p, c_int32, c_int32, c_int32, P, c_int64], c_int),
        "fit_export": ([P, ctypes.c_char_p], c_int),
        "nnm_free": ([P], None),
        "nnm_param_count": ([c_int32, c_int32, c_int32], c_int64),
        "nnm_sync": ([P], c_int),
        "nnm_last_error": ([], ctypes.c_char_p),
        "nnm_version": ([], ctypes.c_char_p),
        "siren_workspace_bytes": ([P, c_int64], c_int64),
        "siren_forward_tangent": ([P, P, c_int64, P, P, P, P], c_int),
        "siren_backward": ([P, P, c_int64, P, P, P, P, P, P, c_int64, P], c_int),
        "fit_create": ([P, P, c_int, c_int64, P], c_int),
        "fit_free": ([P], None),
        "fit_step": ([P, P, P, P, P], c_int),
        "fit_loss_grad": ([P, P, P, P, P], c_int),
        "fit_state": ([P, P, P, P, P], c_int),
        "fit_get_step": ([P], c_int64),
        "fit_read_state": ([P, P, P, P], c_int),
        "fit_write_state": ([P, P, P, P], c_int),
        "fit_set_step": ([P, c_int64], c_int),
        "nnm_profiler_create": ([P], c_int),
        "nnm_profiler_free": ([P], None),
        "nnm_profiler_reset": ([P], c_int),
        "nnm_profiler_report": ([P, P], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = load_library().nnm_last_error().decode(errors="replace")
        raise NnmError(rc, msg)


# ------------------------------------------------------------------ descriptors

@dataclass
class LevelSpec:
    """One level: network shape, float32 parameters (file order), scene terms."""
    d_in: int
    width: int
    n_sine: int
    params: np.ndarray
    amplitude: float
    delta: float = 0.0
    follow_center: bool = False


def levels_from_scene(scene) -> List[LevelSpec]:
    """LevelSpecs of an ``nnm_inputs`` scene (duck-typed: level.net, .amplitude, ...)."""
    out = []
    for l in scene.levels:
        out.append(LevelSpec(l.net.d_in, l.net.width, l.net.n_sine,
                             np.ascontiguousarray(l.net.flat(), dtype=np.float32),
                             float(l.amplitude), float(l.delta), bool(l.follow_center)))
    return out


class _Desc:
    """Keeps parameter arrays alive while the C descriptor is in use."""

    def __init__(self, levels: List[LevelSpec], base_sphere: bool, r0: float, rho: float,
                 lipschitz_max: float):
        self.params = [np.ascontiguousarray(l.params, dtype=np.float32) for l in levels]
        arr = (_LevelDesc * max(len(levels), 1))()
        for j, l in enumerate(levels):
            arr[j].d_in = int(l.d_in)
            arr[j].width = int(l.width)
            arr[j].n_sine = int(l.n_sine)
            arr[j].follow_center = 1 if l.follow_center else 0
            arr[j].amplitude = float(l.amplitude)
            arr[j].delta = float(l.delta)
            arr[j].params = self.params[j].ctypes.data_as(POINTER(c_float))
        self.arr = arr
        self.desc = _StackDesc(len(levels), 1 if base_sphere else 0, float(r0), float(rho),
                               float(lipschitz_max), 0, ctypes.cast(arr, POINTER(_LevelDesc)))

    def ptr(self):
        return ctypes.cast(ctypes.byref(self.desc), c_void_p)


def _prec(precision) -> int:
    if isinstance(precision, str):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        return PRECISIONS[precision]
    return int(precision)


def nnm_validate_stack(levels: List[LevelSpec], precision="fp32", base_sphere=True, r0=0.6, rho=0.0,
                       lipschitz_max=1.03) -> int:
    """Host-only validation; returns the C return code (0 = valid)."""
    d = _Desc(levels, base_sphere, r0, rho, lipschitz_max)
    return load_library().nnm_validate_stack(d.ptr(), _prec(precision))


def nnm_level_lipschitz_bound(level: LevelSpec, base_sphere=True) -> float:
    d = _Desc([level], base_sphere, 0.6, 0.0, 0.0)
    out = c_double()
    _check(load_library().nnm_level_lipschitz_bound(ctypes.cast(d.arr, c_void_p), 1 if base_sphere else 0,
                                                    ctypes.cast(ctypes.byref(out), c_void_p)))
    return out.value


class Stack:
    """A loaded (immutable) nested sequence of networks on one device."""

    def __init__(self, handle, m: int, precision: int, device: int):
        self._h = handle
        self.m = m
        self.precision = precision
        self.device = device

    @property
    def handle(self):
        if not self._h:
            raise NnmError(-1, "stack has been freed")
        return self._h

    def close(self):
        if self._h:
            load_library().free_siren_stack(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load_siren_stack(levels, precision="fp32", device: int = 0, base_sphere=True, r0=0.6, rho=0.0,
                     lipschitz_max=1.03) -> Stack:
    """Validate, pack and upload a nested sequence (list of LevelSpec or a scene)."""
    if not isinstance(levels, (list, tuple)):
        scene = levels
        levels = levels_from_scene(scene)
        base_sphere, r0, rho = scene.base_sphere, scene.r0, scene.rho
    d = _Desc(list(levels), base_sphere, r0, rho, lipschitz_max)
    h = c_void_p()
    p = _prec(precision)
    _check(load_library().load_siren_stack(d.ptr(), p, int(device), ctypes.cast(ctypes.byref(h), c_void_p)))
    return Stack(h, len(levels), p, int(device))


def free_siren_stack(stack: Stack):
    stack.close()


class Profiler:
    """HIP-event timing of every kernel launched by trace_rays while attached."""

    def __init__(self):
        h = c_void_p()
        _check(load_library().nnm_profiler_create(ctypes.cast(ctypes.byref(h), c_void_p)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def reset(self):
        _check(load_library().nnm_profiler_reset(self._h))

    def report(self):
        """List of dicts (kind 'trace'/'normal'/'order', level, width, kernel, variant, launches,
        total_ms); 'order' is the sort of level `level`'s output queue."""
        r = _ProfileReport()
        _check(load_library().nnm_profiler_report(self._h, ctypes.cast(ctypes.byref(r), c_void_p)))
        names = {("trace", 0): "k_trace_level", ("trace", 1): "k_trace_ws",
                 ("normal", 0): "k_normal", ("normal", 1): "k_normal_ws", ("order", 0): "k_queue_order"}
        out = []
        for i in range(r.n_entries):
            kind = ("trace", "normal", "order")[r.kind[i]]
            out.append({"kind": kind, "level": r.level[i], "width": r.width[i],
                        "kernel": names[(kind, r.variant[i])], "variant": int(r.variant[i]),
                        "launches": int(r.launches[i]), "total_ms": float(r.total_ms[i])})
        return out

    def close(self):
        if self._h:
            load_library().nnm_profiler_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class TraceParams:
    step_scale: float = 0.9
    eps: float = 1e-4
    far: float = 5.0
    max_steps: int = 64
    final_level: int = -1    # -1: last level
    normal_level: int = -1   # -1: final_level
    mode: int = 0
    profiler: Optional[Profiler] = None
    iterations: Optional[Sequence[int]] = None  # fixed-iteration mode (mode 1): steps per traced level
    kernels: str = "auto"  # "auto" (weight-stationary where available) or "streaming"

    def c(self, m: int) -> _TraceParams:
        fl = m - 1 if self.final_level < 0 else self.final_level
        nl = fl if self.normal_level < 0 else self.normal_level
        prof = self.profiler.handle if self.profiler is not None else None
        mode = self.mode
        its = (c_int32 * 8)()
        if self.iterations is not None:
            mode = 1
            for j, k in enumerate(self.iterations):
                its[j] = int(k)
        return _TraceParams(self.step_scale, self.eps, self.far, self.max_steps, fl, nl, mode,
                            KERNELS[self.kernels], prof, its)


def _dev_ptr(t, dtype, shape, name, device, allow_none=True):
    """Validate a torch tensor argument and return its device pointer (marshalling only)."""
    if t is None:
        if allow_none:
            return None
        raise NnmError(-1, f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise NnmError(-1, f"{name} must be a torch tensor")
    if t.device.type != "cuda" or (t.device.index if t.device.index is not None else 0) != device:
        raise NnmError(-1, f"{name} must live on cuda:{device}")
    if t.dtype != dtype:
        raise NnmError(-1, f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise NnmError(-1, f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise NnmError(-1, f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return c_void_p(t.data_ptr()) if t.numel() else c_void_p(0)


def _stream_ptr(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return c_void_p(stream.cuda_stream)


def trace_rays(stack: Stack, params: TraceParams, o, v, t, depth, hit, normal=None, steps=None, status=None,
               stream=None):
    """Multiscale sphere tracing into caller-allocated tensors (see include/nnm.h)."""
    _trace_call("trace_rays", stack, params, o, v, t, depth, hit, normal, steps, status, stream)


def trace_rays_noalloc(stack: Stack, params: TraceParams, o, v, t, depth, hit, normal=None, steps=None,
                       status=None, stream=None):
    """trace_rays with the library's static per-GPU scratch: no device allocation
    (at most NNM_NOALLOC_MAX_RAYS rays; calls that overlap on one GPU race)."""
    _trace_call("trace_rays_noalloc", stack, params, o, v, t, depth, hit, normal, steps, status, stream)


NOALLOC_MAX_RAYS = 1 << 21


def _trace_call(entry, stack, params, o, v, t, depth, hit, normal, steps, status, stream):
    import torch
    n = int(o.shape[0]) if hasattr(o, "shape") else 0
    dev = stack.device
    args = [
        _dev_ptr(o, torch.float32, (n, 3), "o", dev, False),
        _dev_ptr(v, torch.float32, (n, 3), "v", dev, False),
        _dev_ptr(t, torch.float32, (n,), "t", dev),
        _dev_ptr(depth, torch.float32, (n,), "depth", dev, False),
        _dev_ptr(hit, torch.uint8, (n,), "hit", dev, False),
        _dev_ptr(normal, torch.float32, (n, 3), "normal", dev),
        _dev_ptr(steps, torch.uint8, (n, stack.m), "steps", dev),
        _dev_ptr(status, torch.uint8, (n,), "status", dev),
    ]
    cp = params.c(stack.m)
    fn = getattr(load_library(), entry)
    _check(fn(stack.handle, ctypes.cast(ctypes.byref(cp), c_void_p), n, *args, _stream_ptr(stream, dev)))


def analytic_normal(stack: Stack, level: int, x, t, value, grad, stream=None):
    import torch
    n = int(x.shape[0])
    dev = stack.device
    _check(load_library().analytic_normal(
        stack.handle, int(level), n, _dev_ptr(x, torch.float32, (n, 3), "x", dev, False),
        _dev_ptr(t, torch.float32, (n,), "t", dev), _dev_ptr(value, torch.float32, (n,), "value", dev),
        _dev_ptr(grad, torch.float32, (n, 3), "grad", dev, False), _stream_ptr(stream, dev)))


def nnm_net_eval(stack: Stack, level: int, x, t, value, grad, stream=None):
    import torch
    n = int(x.shape[0])
    dev = stack.device
    _check(load_library().nnm_net_eval(
        stack.handle, int(level), n, _dev_ptr(x, torch.float32, (n, 3), "x", dev, False),
        _dev_ptr(t, torch.float32, (n,), "t", dev), _dev_ptr(value, torch.float32, (n,), "value", dev),
        _dev_ptr(grad, torch.float32, (n, 3), "grad", dev), _stream_ptr(stream, dev)))


def nnm_sup_abs_diff(stack: Stack, level_a: int, level_b: int, n: int, seed: int = 0, lo: float = -1.5,
                     hi: float = 1.5, out=None, stream=None) -> float:
    """Sampled sup |f_a - f_b| over [lo, hi]^3 (nnm_sup_abs_diff); returns it as a float."""
    import torch
    dev = torch.device("cuda", stack.device)
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=dev)
    _check(load_library().nnm_sup_abs_diff(stack.handle, int(level_a), int(level_b), ctypes.c_int64(int(n)),
                                           ctypes.c_uint64(int(seed)), ctypes.c_float(lo), ctypes.c_float(hi),
                                           _dev_ptr(out, torch.float32, (1,), "out", stack.device, False),
                                           _stream_ptr(stream, stack.device)))
    return float(out.item())


def nnm_sup_abs_err(stack: Stack, level: int, shape: str, a: float, b: float = 0.0, n: int = 1 << 24,
                    seed: int = 0, lo: float = -1.0, hi: float = 1.0, out=None, stream=None) -> float:
    """Sampled sup |f - f_level| against a reference SDF ("sphere": radius a;
    "torus": major radius a, minor radius b, axis z) over [lo, hi]^3
    (nnm_sup_abs_err); returns it as a float."""
    import torch
    dev = torch.device("cuda", stack.device)
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=dev)
    if shape not in REF_SHAPES:
        raise NnmError(-1, f"reference shape {shape!r} (sphere or torus)")
    ref = _RefSdf(REF_SHAPES[shape], float(a), float(b), 0)
    _check(load_library().nnm_sup_abs_err(stack.handle, int(level), ctypes.byref(ref), ctypes.c_int64(int(n)),
                                          ctypes.c_uint64(int(seed)), ctypes.c_float(lo), ctypes.c_float(hi),
                                          _dev_ptr(out, torch.float32, (1,), "out", stack.device, False),
                                          _stream_ptr(stream, stack.device)))
    return float(out.item())


def nnm_nesting_thresholds(proposition: int, sup: Sequence[float], margin: float = 0.0) -> List[float]:
    """Thresholds delta[0 .. m-1] from sampled bounds by Proposition 1 or 2
    (nnm_nesting_thresholds; for proposition 1, sup[0] is not read)."""
    m = len(sup)
    arr = (c_double * max(m, 1))(*[float(x) for x in sup])
    out = (c_double * max(m, 1))()
    _check(load_library().nnm_nesting_thresholds(int(proposition), m, arr, float(margin), out))
    return [out[i] for i in range(m)]


def nesting_thresholds(stack: Stack, n: int = 1 << 24, seed: int = 0, lo: float = -1.5, hi: float = 1.5,
                       margin: float = 1e-4):
    """Proposition 1 thresholds from sampled bounds sup |f_i - f_{i-1}| (i = 1 .. m-1):
    nnm_sup_abs_diff for each pair, then nnm_nesting_thresholds.
    Returns (deltas[m], sups[m-1])."""
    sups = [nnm_sup_abs_diff(stack, i, i - 1, n, seed + i, lo, hi) for i in range(1, stack.m)]
    return nnm_nesting_thresholds(1, [0.0] + sups, margin), sups


def capacity_thresholds(stack: Stack, shape: str, a: float, b: float = 0.0, n: int = 1 << 24, seed: int = 0,
                        lo: float = -1.0, hi: float = 1.0, margin: float = 1e-4):
    """Proposition 2 thresholds for levels that approximate one known SDF:
    nnm_sup_abs_err for each level, then nnm_nesting_thresholds.
    Returns (deltas[m], sups[m])."""
    sups = [nnm_sup_abs_err(stack, i, shape, a, b, n, seed, lo, hi) for i in range(stack.m)]
    return nnm_nesting_thresholds(2, sups, margin), sups


def neural_normal_map(stack: Stack, level: int, x, t=None, normal=None, stream=None):
    """Unit normals of f_level at points x[n, 3] (neural_normal_map); returns the normal tensor."""
    import torch
    n = int(x.shape[0])
    dev = stack.device
    if normal is None:
        normal = torch.empty((n, 3), dtype=torch.float32, device=torch.device("cuda", dev))
    _check(load_library().neural_normal_map(
        stack.handle, int(level), n, _dev_ptr(x, torch.float32, (n, 3), "x", dev, False),
        _dev_ptr(t, torch.float32, (n,), "t", dev), _dev_ptr(normal, torch.float32, (n, 3), "normal", dev, False),
        _stream_ptr(stream, dev)))
    return normal


def nnm_grid_values(stack: Stack, level: int, res: int, lo: float = -1.0, hi: float = 1.0, t: float = 0.0,
                    values=None, stream=None):
    """f_level at the res^3 grid nodes (nnm_grid_values); returns values[res, res, res] indexed [k, j, i]."""
    import torch
    dev = stack.device
    if values is None:
        values = torch.empty((res, res, res), dtype=torch.float32, device=torch.device("cuda", dev))
    _check(load_library().nnm_grid_values(
        stack.handle, int(level), int(res), ctypes.c_float(lo), ctypes.c_float(hi), ctypes.c_float(t),
        _dev_ptr(values, torch.float32, (res, res, res), "values", dev, False), _stream_ptr(stream, dev)))
    return values


def nnm_mesh_extract(values, lo: float = -1.0, hi: float = 1.0, iso: float = 0.0, verts=None, tris=None,
                     counts=None, stream=None):
    """Marching tetrahedra into caller-allocated verts[max_v, 3] / tris[max_t, 3] (nnm_mesh_extract).

    Asynchronous; counts (int64 [2], allocated when None) receives the totals,
    which exceed the capacities when the arrays were too small.  Returns counts."""
    import torch
    res = int(values.shape[0])
    dev = values.device.index if values.device.index is not None else 0
    if counts is None:
        counts = torch.empty(2, dtype=torch.int64, device=values.device)
    max_v = 0 if verts is None else int(verts.shape[0])
    max_t = 0 if tris is None else int(tris.shape[0])
    with torch.cuda.device(dev):
        _check(load_library().nnm_mesh_extract(
            _dev_ptr(values, torch.float32, (res, res, res), "values", dev, False), res, ctypes.c_float(lo),
            ctypes.c_float(hi), ctypes.c_float(iso), max_v, max_t,
            _dev_ptr(verts, torch.float32, (max_v, 3), "verts", dev), _dev_ptr(tris, torch.int32, (max_t, 3), "tris", dev),
            _dev_ptr(counts, torch.int64, (2,), "counts", dev, False), _stream_ptr(stream, dev)))
    return counts


def extract_mesh(values, lo: float = -1.0, hi: float = 1.0, iso: float = 0.0, capacity=(1 << 20, 1 << 21),
                 stream=None):
    """nnm_mesh_extract with allocation: (verts[nv, 3], tris[nt, 3]), calling again with exact
    capacities when the first guess was too small (one host synchronisation per call)."""
    import torch
    dev = values.device
    max_v, max_t = capacity
    for _ in range(2):
        verts = torch.empty((max_v, 3), dtype=torch.float32, device=dev)
        tris = torch.empty((max_t, 3), dtype=torch.int32, device=dev)
        counts = nnm_mesh_extract(values, lo, hi, iso, verts, tris, stream=stream)
        nv, nt = (int(c) for c in counts.cpu())
        if nv <= max_v and nt <= max_t:
            return verts[:nv], tris[:nt]
        max_v, max_t = max(nv, 1), max(nt, 1)
    raise NnmError(-7, "mesh counts changed between calls")


def mesh_neural_normal_map(stack: Stack, coarse_level: int, fine_level: int, res: int, lo: float = -1.0,
                           hi: float = 1.0, iso: float = 0.0, t: float = 0.0, stream=None):
    """The triangle-mesh form of neural normal mapping: the coarse mesh of f_coarse by
    nnm_grid_values + nnm_mesh_extract, with the normals of f_fine at its vertices
    (neural_normal_map).  Returns (verts, tris, normals)."""
    values = nnm_grid_values(stack, coarse_level, res, lo, hi, t, stream=stream)
    verts, tris = extract_mesh(values, lo, hi, iso, stream=stream)
    tt = None
    if t != 0.0:
        import torch
        tt = torch.full((verts.shape[0],), float(t), dtype=torch.float32, device=verts.device)
    normals = neural_normal_map(stack, fine_level, verts, tt, stream=stream) if verts.shape[0] else verts.clone()
    return verts, tris, normals


def nnm_sync(stream=None, device: int = 0):
    _check(load_library().nnm_sync(_stream_ptr(stream, device)))


def nnm_write_net_file(path: str, d_in: int, width: int, n_sine: int, params) -> None:
    """Write float32 host parameters as a network file (nnm_write_net_file)."""
    flat = np.ascontiguousarray(params, dtype=np.float32).ravel()
    _check(load_library().nnm_write_net_file(str(path).encode(), int(d_in), int(width), int(n_sine),
                                              flat.ctypes.data_as(c_void_p), flat.size))


def nnm_read_net_file(path: str):
    """(d_in, width, n_sine, float32 params) parsed by the library."""
    lib = load_library()
    d_in, width, n_sine = c_int32(), c_int32(), c_int32()
    buf = ctypes.POINTER(c_float)()
    npar = c_int64()
    _check(lib.nnm_read_net_file(str(path).encode(), ctypes.cast(ctypes.byref(d_in), c_void_p),
                                 ctypes.cast(ctypes.byref(width), c_void_p),
                                 ctypes.cast(ctypes.byref(n_sine), c_void_p),
                                 ctypes.cast(ctypes.byref(buf), c_void_p),
                                 ctypes.cast(ctypes.byref(npar), c_void_p)))
    try:
        arr = np.ctypeslib.as_array(buf, shape=(npar.value,)).copy()
    finally:
        lib.nnm_free(ctypes.cast(buf, c_void_p))
    return d_in.value, width.value, n_sine.value, arr


def render(stack: Stack, o, v, t=None, params: Optional[TraceParams] = None, want_normal=True, stream=None):
    """Allocate outputs on the stack's device and trace; returns a dict of tensors."""
    import torch
    params = params or TraceParams()
    n = int(o.shape[0])
    dev = torch.device("cuda", stack.device)
    out = {
        "depth": torch.empty(n, dtype=torch.float32, device=dev),
        "hit": torch.empty(n, dtype=torch.uint8, device=dev),
        "normal": torch.empty((n, 3), dtype=torch.float32, device=dev) if want_normal else None,
        "steps": torch.empty((n, stack.m), dtype=torch.uint8, device=dev),
        "status": torch.empty(n, dtype=torch.uint8, device=dev),
    }
    trace_rays(stack, params, o, v, t, out["depth"], out["hit"], out["normal"], out["steps"], out["status"],
               stream)
    return out


# ------------------------------------------------------------------ fitting

class _NetShape(ctypes.Structure):
    _fields_ = [("d_in", c_int32), ("width", c_int32), ("n_sine", c_int32), ("reserved", c_int32)]


class _FitBatch(ctypes.Structure):
    _fields_ = [("n_surf", c_int64), ("n_unif", c_int64), ("surf_x", c_void_p), ("surf_n", c_void_p),
                ("unif_x", c_void_p), ("unif_sdf", c_void_p)]


class _Adam(ctypes.Structure):
    _fields_ = [("lr", c_float), ("beta1", c_float), ("beta2", c_float), ("eps", c_float)]


def _shape(d_in, width, n_sine):
    return _NetShape(int(d_in), int(width), int(n_sine), 0)


def _byref(x):
    return ctypes.cast(ctypes.byref(x), c_void_p)


def siren_workspace_bytes(d_in, width, n_sine, n) -> int:
    sh = _shape(d_in, width, n_sine)
    return int(load_library().siren_workspace_bytes(_byref(sh), int(n)))


def siren_forward_tangent(d_in, width, n_sine, params, x, value=None, grad=None, stream=None):
    """N(x) and grad_x N for a flat float32 parameter vector (device tensors)."""
    import torch
    n = int(x.shape[0])
    dev = x.device.index or 0
    sh = _shape(d_in, width, n_sine)
    if value is None:
        value = torch.empty(n, dtype=torch.float32, device=x.device)
    if grad is None:
        grad = torch.empty((n, 3), dtype=torch.float32, device=x.device)
    _check(load_library().siren_forward_tangent(
        _byref(sh), _dev_ptr(params, torch.float32, tuple(params.shape), "params", dev, False), n,
        _dev_ptr(x, torch.float32, (n, d_in), "x", dev, False), _dev_ptr(value, torch.float32, (n,), "value", dev),
        _dev_ptr(grad, torch.float32, (n, 3), "grad", dev), _stream_ptr(stream, dev)))
    return value, grad


def siren_backward(d_in, width, n_sine, params, x, dvalue, dgrad, dparams=None, dx=None, workspace=None,
                   stream=None):
    """dL/dparams (and dL/dx) from upstream dL/dN and dL/dgrad N (device tensors)."""
    import torch
    n = int(x.shape[0])
    dev = x.device.index or 0
    sh = _shape(d_in, width, n_sine)
    if dparams is None:
        dparams = torch.empty_like(params)
    need = siren_workspace_bytes(d_in, width, n_sine, n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    _check(load_library().siren_backward(
        _byref(sh), _dev_ptr(params, torch.float32, tuple(params.shape), "params", dev, False), n,
        _dev_ptr(x, torch.float32, (n, d_in), "x", dev, n > 0),
        _dev_ptr(dvalue, torch.float32, (n,), "dvalue", dev), _dev_ptr(dgrad, torch.float32, (n, 3), "dgrad", dev),
        _dev_ptr(dparams, torch.float32, tuple(params.shape), "dparams", dev, False),
        _dev_ptr(dx, torch.float32, (n, d_in), "dx", dev), c_void_p(workspace.data_ptr()), int(workspace.numel()),
        _stream_ptr(stream, dev)))
    return dparams, dx


class Fit:
    """Fitting state on one device: parameters, Adam moments, step counter."""

    def __init__(self, d_in, width, n_sine, params: np.ndarray, device: int = 0, max_points: int = 1 << 19):
        self.shape = (int(d_in), int(width), int(n_sine))
        self.device = int(device)
        p = np.ascontiguousarray(params, dtype=np.float32)
        sh = _shape(*self.shape)
        h = c_void_p()
        _check(load_library().fit_create(_byref(sh), p.ctypes.data_as(c_void_p), self.device, int(max_points),
                                         _byref(h)))
        self._h = h
        self.n_params = p.size

    def params(self) -> np.ndarray:
        """Copy of the parameters (synchronises the device)."""
        out = np.empty(self.n_params, np.float32)
        _check(load_library().fit_read_state(self._h, out.ctypes.data_as(c_void_p), None, None))
        return out

    def export(self, path: str) -> None:
        """Write the current parameters as a network file (fit_export)."""
        _check(load_library().fit_export(self._h, str(path).encode()))

    def state(self):
        """(params, m, v, step) as numpy arrays (synchronises): a checkpoint."""
        arrs = [np.empty(self.n_params, np.float32) for _ in range(3)]
        _check(load_library().fit_read_state(self._h, *[a.ctypes.data_as(c_void_p) for a in arrs]))
        return arrs[0], arrs[1], arrs[2], self.step

    def load_state(self, params, m, v, step):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, m, v)]
        for a in arrs:
            if a.size != self.n_params:
                raise NnmError(-1, f"state arrays need {self.n_params} entries")
        _check(load_library().fit_write_state(self._h, *[a.ctypes.data_as(c_void_p) for a in arrs]))
        _check(load_library().fit_set_step(self._h, int(step)))

    @property
    def step(self) -> int:
        return int(load_library().fit_get_step(self._h))

    def _batch(self, surf_x, surf_n, unif_x, unif_sdf):
        import torch
        dev = self.device
        ns, nu = int(surf_x.shape[0]), int(unif_x.shape[0])
        b = _FitBatch(ns, nu, _dev_ptr(surf_x, torch.float32, (ns, 3), "surf_x", dev, False),
                      _dev_ptr(surf_n, torch.float32, (ns, 3), "surf_n", dev, False),
                      _dev_ptr(unif_x, torch.float32, (nu, 3), "unif_x", dev, False),
                      _dev_ptr(unif_sdf, torch.float32, (nu,), "unif_sdf", dev, False))
        return b

    def step_adam(self, surf_x, surf_n, unif_x, unif_sdf, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, loss4=None,
                  stream=None):
        """One fitting step (fit_step); loss4: optional device [4] tensor."""
        import torch
        b = self._batch(surf_x, surf_n, unif_x, unif_sdf)
        opt = _Adam(lr, beta1, beta2, eps)
        lp = _dev_ptr(loss4, torch.float32, (4,), "loss4", self.device)
        _check(load_library().fit_step(self._h, _byref(b), _byref(opt), lp, _stream_ptr(stream, self.device)))

    def loss_grad(self, surf_x, surf_n, unif_x, unif_sdf, loss4, dparams, stream=None):
        import torch
        b = self._batch(surf_x, surf_n, unif_x, unif_sdf)
        _check(load_library().fit_loss_grad(
            self._h, _byref(b), _dev_ptr(loss4, torch.float32, (4,), "loss4", self.device),
            _dev_ptr(dparams, torch.float32, (self.n_params,), "dparams", self.device, False),
            _stream_ptr(stream, self.device)))

    def close(self):
        if getattr(self, "_h", None):
            load_library().fit_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
