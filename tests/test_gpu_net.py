"""GPU parity of the fused SIREN evaluator (net level) against the FP64 oracle.

Raw N and grad N at points uniform in [-1.5, 1.5]^3 and in a shell around the
sphere, for every network of the workload scenes and every precision form;
the scene function f and its raw gradient (analytic_normal); ragged and
empty inputs.  Gates: relative L2 error of N and of grad N <= 1e-5 (fp32),
3e-2 (bf16), 5e-3 (fp16).
"""

import numpy as np
import pytest

import nnm_inputs as ni
from oracle import tracing as orc
from tests.parity import NET_REL_L2, rel_l2, sample_points

pytestmark = pytest.mark.gpu

CASES = [("single_64x1_128sq", 0), ("stack3_512sq", 0), ("stack3_512sq", 1), ("stack3_512sq", 2),
         ("anim16_1024sq", 0), ("anim16_1024sq", 1),
         # (256,3): four sine layers; (256,1): two; width 128; hidden arguments near
         # 300 revolutions (the range-reduced sine of every kernel family)
         ("table3_256x3", 0), ("table3_64x1_256x1", 1), ("stack2_64x1_128x2_512sq", 0),
         ("stack2_64x1_128x2_512sq", 1), ("stack3_bigarg_512sq", 2)]

# float32 keeps 24 bits, so a sine argument near K = 300 revolutions carries up to
# 2^-24 * 300 = 1.8e-5 revolutions (1.1e-4 rad) of rounding per operation; a few
# roundings per argument give activation errors near 3e-4 rad against activations
# of rms 0.7, i.e. a relative L2 error of N up to about 1e-3 on top of each form's
# own error.
BIGARG_EXTRA = 2e-3


def _torch():
    import torch
    return torch


def _net_eval_gpu(scene, level, x, t, precision, raw=True):
    torch = _torch()
    import paper_2201_09147_amd as nnm
    dev = torch.device("cuda", 0)
    stack = nnm.load_siren_stack(scene, precision, 0)
    n = x.shape[0]
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(t).to(dev) if t is not None else None
    val = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty((n, 3), dtype=torch.float32, device=dev)
    if raw:
        nnm.nnm_net_eval(stack, level, xd, td, val, grad)
    else:
        nnm.analytic_normal(stack, level, xd, td, val, grad)
    torch.cuda.synchronize()
    stack.close()
    return val.cpu().numpy(), grad.cpu().numpy()


def _net_input(scene, level, x, t):
    lvl = scene.levels[level]
    x64 = x.astype(np.float64)
    if lvl.net.d_in == 4:
        return np.concatenate([x64, t.astype(np.float64)[:, None]], 1)
    if lvl.follow_center:
        c = scene.rho * np.stack([np.cos(2 * np.pi * t.astype(np.float64)),
                                  np.sin(2 * np.pi * t.astype(np.float64)), 0 * t], 1)
        return x64 - c
    return x64


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name,level", CASES)
def test_net_value_and_gradient(name, level, precision):
    scene = ni.make_scene(name)
    n = 4096 if scene.levels[level].net.width >= 256 else 16384
    xs, ts = [], []
    for shell in (False, True):
        x, t = sample_points(n + 13, 31 + level + (7 if shell else 0), shell=shell)
        xs.append(x)
        ts.append(t)
    x = np.concatenate(xs)
    t = np.concatenate(ts)
    val, grad = _net_eval_gpu(scene, level, x, t, precision)
    # the oracle sees the same net input the GPU builds (for follow_center the
    # GPU subtracts a float32 c(t); compare against that input in float64)
    inp = _net_input(scene, level, x, t)
    rv, rg = orc.net_eval(scene.levels[level].net, inp)
    tol = NET_REL_L2[precision] + (BIGARG_EXTRA if name == "stack3_bigarg_512sq" else 0.0)
    ev, eg = rel_l2(val, rv), rel_l2(grad, rg)
    print(f"{name} level {level} {precision}: rel L2 N {ev:.2e} grad {eg:.2e} |N|max {np.abs(rv).max():.3e}")
    assert ev <= tol and eg <= tol


def _first_layer_bound(net):
    """Input inf-norm below which every first-layer sine argument stays within
    63 revolutions (the bound the packer derives; 1e-3 margin)."""
    W0, b0 = (np.asarray(a, np.float64) for a in net.layers[0])
    a = np.abs(W0).sum(axis=1) / (2 * np.pi)
    b = np.abs(b0) / (2 * np.pi)
    return float(np.min((63.0 - b) / a)) * (1.0 - 1e-3)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_first_layer_reduction_on_both_sides_of_the_bound(level, precision):
    """The streaming tiles skip the first layer's reduction to [0, 1)
    revolutions when every column of a wave lies within the level's bound.
    Points well inside it, far outside it (arguments up to about 190
    revolutions), and waves that mix the two, against the oracle."""
    scene = ni.make_scene("stack3_512sq")
    net = scene.levels[level].net
    bound = _first_layer_bound(net)
    rng = np.random.default_rng(90 + level)
    n = 2048
    inside = rng.uniform(-0.9 * bound, 0.9 * bound, size=(n, 3))
    outside = rng.uniform(-3.0 * bound, 3.0 * bound, size=(n, 3))
    outside[:, 0] = np.where(np.abs(outside[:, 0]) < 1.2 * bound, 1.2 * bound, outside[:, 0])
    mixed = np.where((np.arange(n) % 7 == 3)[:, None], outside, inside)  # a few large points per wave
    for name, x, extra in (("inside", inside, 0.0), ("outside", outside, BIGARG_EXTRA),
                           ("mixed", mixed, BIGARG_EXTRA)):
        x = np.ascontiguousarray(x.astype(np.float32))
        val, grad = _net_eval_gpu(scene, level, x, None, precision)
        rv, rg = orc.net_eval(net, x.astype(np.float64))
        ev, eg = rel_l2(val, rv), rel_l2(grad, rg)
        print(f"level {level} {precision} {name} (bound {bound:.2f}): rel L2 N {ev:.2e} grad {eg:.2e}")
        assert ev <= NET_REL_L2[precision] + extra and eg <= NET_REL_L2[precision] + extra


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_scene_function_and_raw_gradient(precision):
    scene = ni.make_scene("stack3_512sq")
    x, t = sample_points(3001, 5, shell=True)
    for level in range(3):
        val, grad = _net_eval_gpu(scene, level, x, None, precision, raw=False)
        rv, rg = orc.scene_eval(scene, level, x.astype(np.float64))
        tolv = 1e-6 if precision == "fp32" else 2e-4
        assert np.abs(val - rv).max() <= tolv
        assert np.abs(grad - rg).max() <= (1e-5 if precision == "fp32" else 5e-3)


def test_empty_and_single_point():
    torch = _torch()
    import paper_2201_09147_amd as nnm
    scene = ni.make_scene("single_64x1_128sq")
    stack = nnm.load_siren_stack(scene, "fp32", 0)
    dev = torch.device("cuda", 0)
    x0 = torch.empty((0, 3), dtype=torch.float32, device=dev)
    nnm.nnm_net_eval(stack, 0, x0, None, torch.empty(0, device=dev), torch.empty((0, 3), device=dev))
    x1 = np.array([[0.1, -0.2, 0.3]], np.float32)
    v = torch.empty(1, device=dev)
    g = torch.empty((1, 3), device=dev)
    nnm.nnm_net_eval(stack, 0, torch.from_numpy(x1).to(dev), None, v, g)
    torch.cuda.synchronize()
    rv, rg = orc.net_eval(scene.levels[0].net, x1.astype(np.float64))
    assert abs(v.item() - rv[0]) <= 1e-5 * max(1, abs(rv[0]))
    np.testing.assert_allclose(g.cpu().numpy()[0], rg[0], atol=1e-5 * np.abs(rg).max())
    stack.close()


@pytest.mark.parametrize("name,precision,pairs", [
    ("stack3_512sq", "fp32", [(1, 0), (2, 1)]),
    ("stack3_512sq", "bf16", [(2, 1)]),
    ("anim16_1024sq", "fp32", [(1, 0)]),
])
def test_sup_abs_diff_matches_oracle_on_the_same_points(name, precision, pairs):
    """nnm_sup_abs_diff (sampled |f_a - f_b|_inf, Sec. 3.3) against the oracle's
    float64 maximum over exactly the points the device drew (splitmix64)."""
    import torch
    import paper_2201_09147_amd as nnm
    from nnm_inputs.sampling import box_points
    s = ni.make_scene(name)
    stack = nnm.load_siren_stack(s, precision, 0)
    n, seed, lo, hi = (1 << 16) + 77, 1234, -1.5, 1.5
    x, t = box_points(seed, n, lo, hi)
    timed = s.frames > 1 or any(l.net.d_in == 4 for l in s.levels)
    for a, b in pairs:
        got = nnm.nnm_sup_abs_diff(stack, a, b, n, seed, lo, hi)
        fa = orc.scene_eval(s, a, x, t if timed else None, grad=False)
        fb = orc.scene_eval(s, b, x, t if timed else None, grad=False)
        ref = float(np.max(np.abs(fa - fb)))
        tol = 2e-6 + 1e-4 * ref if precision == "fp32" else 3e-2 * ref
        print(f"{name} {precision} sup|f{a} - f{b}| gpu {got:.6e} oracle {ref:.6e}")
        assert abs(got - ref) <= tol
    deltas, eps = nnm.nesting_thresholds(stack, n=n, seed=seed)
    assert all(d > 0 for d in deltas) and all(deltas[i] > deltas[i + 1] for i in range(len(deltas) - 1))
    stack.close()
    del torch


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_sup_abs_err_matches_oracle_on_the_same_points(precision):
    """nnm_sup_abs_err (sampled |f - f_level|_inf against a known SDF, the bound
    of Proposition 2, Sec. 3.3) against the oracle's float64 maximum over exactly
    the points the device drew.  Against the sphere |x| - 0.6 the difference is
    the small network term a N (about 1e-3); against the torus it is of order
    0.5, so both ends of the range are covered."""
    import paper_2201_09147_amd as nnm
    from nnm_inputs.sampling import box_points
    from nnm_inputs.torus import torus_sdf
    s = ni.make_scene("stack3_512sq")
    stack = nnm.load_siren_stack(s, precision, 0)
    n, seed, lo, hi = (1 << 16) + 77, 4321, -1.0, 1.0
    x, _ = box_points(seed, n, lo, hi)
    x64 = x.astype(np.float64)
    refs = {"sphere": (0.6, 0.0, np.sqrt(np.sum(x64 * x64, axis=1)) - 0.6),
            "torus": (0.5, 0.2, torus_sdf(x64))}
    for level in range(3):
        f = orc.scene_eval(s, level, x64, None, grad=False)
        for shape, (a, b, sdf) in refs.items():
            got = nnm.nnm_sup_abs_err(stack, level, shape, a, b, n, seed, lo, hi)
            ref = float(np.max(np.abs(f - sdf)))
            tol = 2e-6 + 1e-4 * ref if precision == "fp32" else 2e-6 + 3e-2 * ref
            print(f"{precision} level {level} sup|{shape} - f| gpu {got:.6e} oracle {ref:.6e}")
            assert abs(got - ref) <= tol
    deltas, sups = nnm.capacity_thresholds(stack, "sphere", 0.6, n=n, seed=seed, margin=0.0)
    assert all(deltas[i] > deltas[i + 1] for i in range(2))
    assert deltas == nnm.nnm_nesting_thresholds(2, sups)
    with pytest.raises(nnm.NnmError):
        nnm.nnm_sup_abs_err(stack, 0, "torus", 0.5, 0.0, n, seed, lo, hi)
    with pytest.raises(nnm.NnmError):
        nnm.nnm_sup_abs_err(stack, 3, "sphere", 0.6, 0.0, n, seed, lo, hi)
    stack.close()
