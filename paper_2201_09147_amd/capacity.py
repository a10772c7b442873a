"""Capacity sequences (Sec. 3.3, "MLPs for a single surface"): networks of
growing capacity fitted to one known SDF, then nested by Proposition 2.

A driver over the C ABI: every fitting step is fit_step, every sup is
nnm_sup_abs_err and the thresholds come from nnm_nesting_thresholds; this
module only loops and marshals.  The caller supplies the initial networks and
a batch function (step -> float32 arrays surf_x, surf_n, unif_x, unif_sdf).
"""

from typing import Callable, List, Sequence

import numpy as np

from ._binding import Fit, LevelSpec, capacity_thresholds, load_siren_stack


def fit_sequence(nets: Sequence, lrs: Sequence[float], steps: int, batch: Callable, device: int = 0,
                 max_points: int = 1 << 19, prefetch: int = 4, log: Callable = None):
    """Fit every network on the same batches with Adam (fit_step); returns the
    fitted parameter vectors and the last loss terms of each network.

    ``nets`` are objects with d_in, width, n_sine and flat() (the float32
    parameter vector); ``batch(step)`` returns host arrays."""
    import concurrent.futures as cf
    import torch
    dev = torch.device("cuda", device)
    fits = [Fit(n.d_in, n.width, n.n_sine, n.flat(), device, max_points) for n in nets]
    losses = [torch.empty(4, dtype=torch.float32, device=dev) for _ in nets]
    try:
        with cf.ThreadPoolExecutor(max(1, prefetch)) as pool:
            futs = {i: pool.submit(batch, i) for i in range(min(prefetch, steps))}
            for i in range(steps):
                b = futs.pop(i).result()
                if i + prefetch < steps:
                    futs[i + prefetch] = pool.submit(batch, i + prefetch)
                bt = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in b)
                for f, l, lr in zip(fits, losses, lrs):
                    f.step_adam(*bt, lr=lr, loss4=l)
                if log is not None and (i % 1000 == 0 or i == steps - 1):
                    log(i, [float(l.sum().item()) for l in losses])
        torch.cuda.synchronize()
        params = [f.params() for f in fits]
        last = [l.cpu().numpy().astype(np.float64) for l in losses]
    finally:
        for f in fits:
            f.close()
    return params, last


def nest_by_proposition2(levels: List[LevelSpec], shape: str, a: float, b: float = 0.0, n: int = 1 << 24,
                         seed: int = 0, lo: float = -1.0, hi: float = 1.0, margin: float = 1e-3, device: int = 0):
    """Sampled sup |f - f_j| of every level against the reference SDF over
    [lo, hi]^3, then Proposition 2's thresholds.  ``levels`` carry the fitted
    networks (amplitude 1, no base term); their deltas are replaced.
    Returns (deltas[m], sups[m])."""
    probe = [LevelSpec(l.d_in, l.width, l.n_sine, l.params, 1.0, float(len(levels) - j))
             for j, l in enumerate(levels)]
    stack = load_siren_stack(probe, "fp32", device, base_sphere=False, lipschitz_max=0.0)
    try:
        return capacity_thresholds(stack, shape, a, b, n, seed, lo, hi, margin)
    finally:
        stack.close()
