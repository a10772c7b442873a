"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle."""

import numpy as np

FP32_DEPTH_TOL = 1e-4      # max |depth - depth*| over common hits (FP32 form)
LOWP_DEPTH_TOL = 1e-3      # BF16 / FP16 forms
MASK_AGREEMENT = 0.999     # hit-mask agreement over all rays
FP32_MEAN_ANGLE_DEG = 0.01
LOWP_MEAN_ANGLE_DEG = 0.5
NET_REL_L2 = {"fp32": 1e-5, "bf16": 3e-2, "fp16": 5e-3}


def gpu_trace(scene, o, v, t=None, precision="fp32", final_level=-1, normal_level=-1, stack=None, kernels="auto",
              iterations=None):
    import torch
    import paper_2201_09147_amd as nnm
    dev = torch.device("cuda", 0)
    own = stack is None
    if own:
        stack = nnm.load_siren_stack(scene, precision, 0)
    p = nnm.TraceParams(scene.step_scale, scene.eps, scene.far, scene.max_steps, final_level, normal_level,
                        kernels=kernels, iterations=iterations)
    tt = None if t is None else torch.from_numpy(np.ascontiguousarray(t)).to(dev)
    out = nnm.render(stack, torch.from_numpy(o).to(dev), torch.from_numpy(v).to(dev), tt, p)
    torch.cuda.synchronize()
    res = {k: (val.cpu().numpy() if val is not None else None) for k, val in out.items()}
    if own:
        stack.close()
    return res


def compare(gpu, ref):
    """Error statistics of a GPU trace against the oracle."""
    hit = gpu["hit"] == 1
    rhit = ref["hit"] == 1
    both = hit & rhit
    stats = {"n": int(hit.size), "hits": int(rhit.sum()), "common": int(both.sum()),
             "mask_agreement": float(np.mean(hit == rhit))}
    if both.any():
        stats["depth_max_err"] = float(np.abs(gpu["depth"][both] - ref["depth"][both]).max())
        ang = angle_deg(gpu["normal"][both], ref["normal"][both])
        stats["angle_mean_deg"] = float(ang.mean())
        stats["angle_max_deg"] = float(ang.max())
        stats["angle_p999_deg"] = float(np.quantile(ang, 0.999))
    else:
        stats.update(depth_max_err=0.0, angle_mean_deg=0.0, angle_max_deg=0.0, angle_p999_deg=0.0)
    return stats


def angle_deg(a, b):
    """Angle between row vectors, atan2(|a x b|, a . b): well conditioned near 0."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.degrees(np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1)))


def check_fp32(stats):
    assert stats["mask_agreement"] >= MASK_AGREEMENT, stats
    assert stats["depth_max_err"] <= FP32_DEPTH_TOL, stats
    assert stats["angle_mean_deg"] <= FP32_MEAN_ANGLE_DEG, stats


def check_lowp(stats):
    assert stats["mask_agreement"] >= MASK_AGREEMENT, stats
    assert stats["depth_max_err"] <= LOWP_DEPTH_TOL, stats
    assert stats["angle_mean_deg"] <= LOWP_MEAN_ANGLE_DEG, stats


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def sample_points(n, seed, d_in=3, shell=False):
    rng = np.random.default_rng(seed)
    if shell:
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        x = d * rng.uniform(0.55, 0.65, size=(n, 1))
    else:
        x = rng.uniform(-1.5, 1.5, size=(n, 3))
    x = x.astype(np.float32)
    t = rng.uniform(0.0, 1.0, size=n).astype(np.float32)
    return x, t


def sphere_eps_counts(o, v, deltas, s, cap=4000):
    """Evaluations per level that eps-terminated tracing of the analytic sphere
    needs without a budget: at level j the recursion
    tau <- tau + s (|o + tau v| - 0.6 - delta_j) runs until its value d <= eps.
    Also returns the smallest margin |d - eps| met at a level exit (to skip rays
    whose count could depend on rounding)."""
    o64, v64 = o.astype(np.float64), v.astype(np.float64)
    n = o.shape[0]
    m = len(deltas)
    tau = np.zeros(n)
    counts = np.zeros((n, m), np.int64)
    margin = np.full(n, np.inf)
    reach = np.ones(n, bool)
    for j, delta in enumerate(deltas):
        active = reach.copy()
        k = np.zeros(n, np.int64)
        for _ in range(cap):
            if not active.any():
                break
            p = o64 + tau[:, None] * v64
            d = np.sqrt(np.sum(p * p, axis=1)) - 0.6 - delta
            k = np.where(active, k + 1, k)
            tau = np.where(active, tau + s.step_scale * d, tau)
            reach &= ~(active & (tau > s.far))
            done = active & (d <= s.eps)
            margin = np.where(active, np.minimum(margin, np.abs(d - s.eps)), margin)
            active &= ~done & (tau <= s.far)
        counts[:, j] = k
    return counts, reach, margin
