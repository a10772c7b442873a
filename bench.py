#!/usr/bin/env python3
"""Throughput of multiscale sphere tracing with analytic normals on one MI355X.

Workload (default): the three-level nested SIREN stack (32,1) |> (64,1) |>
(256,2) rendered at 1920x1080, every ray traced to a hit or a miss and every hit
given its analytic unit normal.  One step = one trace_rays call over the whole
frame with rays already resident in device memory.  Measured forms: FP32 and
BF16 hidden layers (the headline value is the --precision form).

Prints progress on stderr and ONE JSON line on stdout with the rays/s, the
roofline of the dominant kernel (HIP events around each launch, algorithmic
hidden-layer FLOPs from the per-level step counts), the error statistics
against the FP64 CPU oracle on a row sample, and the oracle's own rate on that
sample (cpu_baseline).  After its W warm-up calls each form keeps calling,
untimed, for 0.2 s (the GPU clock ramps up over tens of milliseconds after the
idle spell of packing a stack).  Each form runs its K timed calls three times: back to
back under the wall clock (the rays/s), with HIP events around each call (the
per-call spread), and with the library's profiler (the per-kernel durations;
its event pair around every launch adds about 10 us per kernel boundary, so
that pass is not the throughput).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/s to hit+normal at 1080p, 3-level SIREN; FP32 vs BF16-MFMA at stated err"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}  # dense MFMA, MI355X
SETTLE_S = 0.2  # untimed calls after the W warm-up steps, until the GPU clock has settled


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hidden_flops(net) -> int:
    """2 FLOP per multiply-accumulate of the width x width layers of one forward."""
    return 2 * (net.n_sine - 1) * net.width * net.width


def normal_hidden_flops(net) -> int:
    """Forward plus three tangent columns through the hidden layers."""
    return 4 * hidden_flops(net)


def run_form(scene, precision, o, v, t, steps, warmup, final_level=-1, normal_level=-1):
    import torch
    import paper_2201_09147_amd as nnm
    dev = torch.device("cuda", 0)
    n = o.shape[0]
    torch.cuda.synchronize()
    l0 = time.perf_counter()
    stack = nnm.load_siren_stack(scene, precision, 0)  # validation, packing, upload: outside the timed region
    torch.cuda.synchronize()
    load_ms = (time.perf_counter() - l0) * 1e3
    out = {
        "depth": torch.empty(n, dtype=torch.float32, device=dev),
        "hit": torch.empty(n, dtype=torch.uint8, device=dev),
        "normal": torch.empty((n, 3), dtype=torch.float32, device=dev),
        "steps": torch.empty((n, stack.m), dtype=torch.uint8, device=dev),
        "status": torch.empty(n, dtype=torch.uint8, device=dev),
    }
    prof = nnm.Profiler()
    params = nnm.TraceParams(scene.step_scale, scene.eps, scene.far, scene.max_steps, final_level, normal_level)

    def call(p):
        nnm.trace_rays(stack, p, o, v, t, out["depth"], out["hit"], out["normal"], out["steps"],
                       out["status"])

    for _ in range(warmup):
        call(params)
    torch.cuda.synchronize()
    # The GPU clock ramps up over tens of milliseconds of work after an idle
    # spell (stack packing, the previous form's host work): keep calling,
    # untimed, until the warm-up has run for SETTLE_S, so the K timed calls
    # measure the settled clock (on the 1080p frame the first ~15 calls after
    # idle take 2.0 -> 1.76 ms).
    settle = 0
    s0 = time.perf_counter()
    while time.perf_counter() - s0 < SETTLE_S and settle < 1000:
        call(params)
        settle += 1
        if settle % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    log(f"[{precision}] warmup done ({warmup} steps + {settle} settling calls, final level {final_level}, "
        f"normal level {normal_level})")
    timed = nnm.TraceParams(scene.step_scale, scene.eps, scene.far, scene.max_steps, final_level, normal_level,
                            profiler=prof)
    # 1. the throughput: K calls back to back, wall clock around all of them
    #    (no event between the kernels: an event pair around every launch, as
    #    the profiler records, costs about 10 us per kernel boundary)
    t0 = time.perf_counter()
    for i in range(steps):
        call(params)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    # 2. the spread: HIP events around each of K more calls on their (current) stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for i in range(steps):
        evs[i][0].record()
        call(params)
        evs[i][1].record()
    # 3. the per-kernel durations: K more calls with the library's profiler
    #    (HIP events around every launch, on the launch stream)
    tp0 = time.perf_counter()
    for i in range(steps):
        call(timed)
    torch.cuda.synchronize()
    ms_prof = (time.perf_counter() - tp0) * 1e3 / steps
    per_call = sorted(a.elapsed_time(b) for a, b in evs)
    timing = {"median_ms": round(per_call[len(per_call) // 2], 4), "min_ms": round(per_call[0], 4),
              "p90_ms": round(per_call[min(len(per_call) - 1, int(0.9 * len(per_call)))], 4),
              "profiled_ms_per_step": round(ms_prof, 4), "load_ms": round(load_ms, 3),
              "settling_calls": settle}
    report = prof.report()
    tag = precision if final_level < 0 else f"{precision} NNM {final_level}->{normal_level}"
    log(f"[{tag}] {steps} steps: {ms:.3f} ms/step, {n / ms * 1e3 / 1e9:.3f} Grays/s; per call median "
        f"{timing['median_ms']:.3f} min {timing['min_ms']:.3f} p90 {timing['p90_ms']:.3f} ms; "
        f"with per-kernel events {ms_prof:.3f} ms/step; stack load {load_ms:.1f} ms")
    evals = out["steps"].to(torch.int64).sum(dim=0).cpu().tolist()
    entering = (out["steps"] > 0).to(torch.int64).sum(dim=0).cpu().tolist()
    hits = int(out["hit"].to(torch.int64).sum().item())
    kernels = []
    for e in report:
        lvl = scene.levels[e["level"]]
        if e["kind"] == "trace":
            flops = evals[e["level"]] * hidden_flops(lvl.net)
            units = evals[e["level"]]
        elif e["kind"] == "order":  # queue entries sorted for the next level
            flops = 0
            units = entering[e["level"] + 1]
        else:
            flops = hits * normal_hidden_flops(lvl.net)
            units = hits
        avg_ms = e["total_ms"] / max(e["launches"], 1)
        kernels.append({"kind": e["kind"], "kernel": e["kernel"], "level": e["level"], "width": e["width"],
                        "avg_ms": avg_ms,
                        "evals": units,
                        "hidden_flops": flops,
                        "tflops": flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0})
    res = {"precision": precision, "workload": scene.name, "ms_per_step": ms, "rays_per_s": n / (ms * 1e-3), "hits": hits, "timing": timing,
           "evals_per_level": evals, "kernels": kernels,
           "outputs": {k: v_.cpu().numpy() for k, v_ in out.items()}}
    prof.close()
    stack.close()
    return res


def run_fit(steps, warmup):
    """Fitting workload: (256,2) SIREN, 2^16 surface + 2^18 uniform torus points
    per step, FP32 double backward + Adam (fit_step).  Batches are generated
    before the timed region and cycled."""
    import torch
    import nnm_inputs as ni
    import paper_2201_09147_amd as nnm
    scene = ni.make_scene("fit_torus_256x2")
    ns, nu = scene.extra["n_surf"], scene.extra["n_unif"]
    net = scene.levels[0].net
    dev = torch.device("cuda", 0)
    batches = [tuple(torch.from_numpy(a).to(dev) for a in ni.torus_batch(s, ns, nu)) for s in range(4)]
    fit = nnm.Fit(net.d_in, net.width, net.n_sine, net.flat(), 0, ns + nu)
    loss = torch.empty(4, dtype=torch.float32, device=dev)
    for i in range(warmup):
        fit.step_adam(*batches[i % 4], lr=scene.extra["lr"], loss4=loss)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fit.step_adam(*batches[i % 4], lr=scene.extra["lr"], loss4=loss)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    flop_point = 3 * 4 * 2 * (net.n_sine - 1) * net.width ** 2  # fwd+tangent, W^T products, weight grads
    tflops = (ns + nu) * flop_point / (ms * 1e-3) / 1e12
    fit.close()
    log(f"[fit] {steps} steps: {ms:.3f} ms/step, {tflops:.1f} TFLOP/s (hidden layers)")
    return {"workload": "fit_torus_256x2", "points_per_step": ns + nu, "ms_per_step": round(ms, 4),
            "steps_per_s": round(1e3 / ms, 3), "points_per_s": round((ns + nu) / (ms * 1e-3), 1),
            "hidden_tflops": round(tflops, 3), "frac_fp32_mfma_peak": round(tflops / PEAK_TFLOPS["fp32"], 5),
            "final_loss4": [round(float(v_), 6) for v_ in loss.cpu().numpy()]}


# HBM bytes per launch of the dominant kernel, from the FETCH_SIZE / WRITE_SIZE
# counter passes summarised in profiles/ (bf16 form).  Used only while the
# kernel's sources hash to the profiled build; otherwise the field is null.
HBM_PROFILE = os.path.join(ROOT, "profiles", "trace_ws_stack3_1080p_hbm.txt")


def measured_traffic(kernel, precision, workload="stack3_1080p"):
    """HBM bytes per launch of the dominant kernel from the committed counter
    profile: only for the profiled configuration (bf16 k_trace_ws on the 1080p
    stack) and only while the kernel sources hash to the profiled build."""
    import hashlib
    if (kernel != "k_trace_ws" or precision != "bf16" or workload != "stack3_1080p"
            or not os.path.exists(HBM_PROFILE)):
        return None
    fields = {}
    for line in open(HBM_PROFILE):
        key, sep, val = line.partition(":")
        if sep and key in ("traffic_bytes_per_launch", "kernel_sources_sha256_16", "kernel_sources"):
            fields[key] = val.strip()
    try:
        h = hashlib.sha256()
        for f in fields["kernel_sources"].split():
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != fields["kernel_sources_sha256_16"]:
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def _torus_trace_exact(o, v, step_scale, eps, far, budget=1024):
    """Sphere tracing of the exact torus SDF (a true distance, so every step is
    safe), float64, vectorised over rays: the reference surface of the fit."""
    import numpy as np
    import nnm_inputs as ni
    o64, v64 = o.astype(np.float64), v.astype(np.float64)
    tau = np.zeros(o.shape[0])
    live = np.ones(o.shape[0], bool)
    hit = np.zeros(o.shape[0], bool)
    for _ in range(budget):
        if not live.any():
            break
        d = ni.torus_sdf(o64[live] + tau[live, None] * v64[live])
        tl = tau[live] + step_scale * d
        tau[live] = tl
        idx = np.flatnonzero(live)
        done_hit = d <= eps
        done_far = tl > far
        hit[idx[done_hit & ~done_far]] = True
        live[idx[done_hit | done_far]] = False
    return hit, tau


def _torus_normal(p):
    import numpy as np
    q = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
    g = np.stack([(q - 0.5) * p[:, 0] / q, (q - 0.5) * p[:, 1] / q, p[:, 2]], axis=1)
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def run_fit_full():
    """The whole fitting workload: 2000 Adam steps of the (256,2) SIREN on fresh
    torus batches (host sampling prefetched on a thread pool), then fit quality
    on a held-out batch and a 1080p FP32 render of the fitted net against an
    exact sphere trace of the torus."""
    import concurrent.futures as cf
    import numpy as np
    import torch
    import nnm_inputs as ni
    import paper_2201_09147_amd as nnm
    scene = ni.make_scene("fit_torus_256x2")
    ns, nu, steps, lr = scene.extra["n_surf"], scene.extra["n_unif"], scene.extra["steps"], scene.extra["lr"]
    net = scene.levels[0].net
    dev = torch.device("cuda", 0)
    fit = nnm.Fit(net.d_in, net.width, net.n_sine, net.flat(), 0, ns + nu)
    loss = torch.empty(4, dtype=torch.float32, device=dev)
    ahead = 8
    hist = []
    with cf.ThreadPoolExecutor(4) as pool:
        futs = {i: pool.submit(ni.torus_batch, i, ns, nu) for i in range(min(ahead, steps))}
        t0 = time.perf_counter()
        for i in range(steps):
            b = futs.pop(i).result()
            if i + ahead < steps:
                futs[i + ahead] = pool.submit(ni.torus_batch, i + ahead, ns, nu)
            fit.step_adam(*(torch.from_numpy(a).to(dev, non_blocking=False) for a in b), lr=lr, loss4=loss)
            if i % 250 == 0 or i == steps - 1:
                hist.append([i] + [round(float(x), 6) for x in loss.cpu().numpy()])
                log(f"[fit-full] step {i}: loss terms {hist[-1][1:]}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    params = fit.params()
    fit.close()
    # held-out quality
    sx, sn, ux, us = ni.torus_batch(10 ** 6, ns, nu)
    pt = torch.from_numpy(params).to(dev)
    fs, gs = nnm.siren_forward_tangent(net.d_in, net.width, net.n_sine, pt, torch.from_numpy(sx).to(dev))
    fu, gu = nnm.siren_forward_tangent(net.d_in, net.width, net.n_sine, pt, torch.from_numpy(ux).to(dev))
    fs, gs, fu, gu = (a.cpu().numpy().astype(np.float64) for a in (fs, gs, fu, gu))
    cosang = np.sum(gs * sn, axis=1) / np.maximum(np.linalg.norm(gs, axis=1), 1e-30)
    quality = {"mean_abs_f_minus_sdf_uniform": float(np.mean(np.abs(fu - us))),
               "mean_abs_f_surface": float(np.mean(np.abs(fs))),
               "mean_normal_angle_deg_surface": float(np.degrees(np.mean(np.arccos(np.clip(cosang, -1, 1))))),
               "mean_abs_gradnorm_minus_1_uniform": float(np.mean(np.abs(np.linalg.norm(gu, axis=1) - 1)))}
    log(f"[fit-full] quality: {quality}")
    # 1080p FP32 render of the fitted net (no Lipschitz bound: lipschitz_max = 0)
    fitted = ni.Scene("fit_torus_256x2", [ni.SceneLevel(ni.SirenNet(net.d_in, net.width, net.n_sine,
                                                                      ni.unflatten_params(params, net.d_in, net.width,
                                                                                          net.n_sine)), 1.0)],
                      1920, 1080, r0=0.0, base_sphere=False)
    stack = nnm.load_siren_stack(fitted, "fp32", 0, lipschitz_max=0.0)
    o_np, v_np, _ = fitted.rays()
    # The net was fitted on [-1, 1]^3 only and is unconstrained outside, so the
    # ray setup starts every ray at its entry into that box (slab test) and
    # traces only the rays that enter it; depth adds the entry distance back,
    # and hits beyond the ray's exit from the box count as misses.
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / v_np.astype(np.float64)
        t1 = (-1.0 - o_np) * inv
        t2 = (1.0 - o_np) * inv
    t_in = np.maximum(np.max(np.minimum(t1, t2), axis=1), 0.0)
    t_out = np.min(np.maximum(t1, t2), axis=1)
    inbox = np.flatnonzero(t_out > t_in)
    o_box = (o_np[inbox] + t_in[inbox, None] * v_np[inbox]).astype(np.float32)
    o, v = torch.from_numpy(o_box).to(dev), torch.from_numpy(np.ascontiguousarray(v_np[inbox])).to(dev)
    prm = nnm.TraceParams(fitted.step_scale, fitted.eps, fitted.far, fitted.max_steps)
    out = nnm.render(stack, o, v, params=prm)
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = nnm.render(stack, o, v, params=prm)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    gb = {k: val.cpu().numpy() for k, val in out.items()}
    n_all = o_np.shape[0]
    g = {"hit": np.zeros(n_all, np.uint8), "depth": np.full(n_all, np.inf, np.float32),
         "normal": np.zeros((n_all, 3), np.float32)}
    # a hit past the ray's exit from the box is on the unconstrained part: a miss
    inside = (gb["hit"] == 1) & (t_in[inbox] + gb["depth"] <= t_out[inbox])
    g["hit"][inbox] = inside
    g["depth"][inbox] = np.where(inside, t_in[inbox] + gb["depth"], np.inf).astype(np.float32)
    g["normal"][inbox] = np.where(inside[:, None], gb["normal"], 0.0)
    rows = np.arange(0, 1080, 8)
    idx = (rows[:, None] * 1920 + np.arange(1920)[None, :]).reshape(-1)
    rhit, rtau = _torus_trace_exact(o_np[idx], v_np[idx], fitted.step_scale, fitted.eps, fitted.far)
    ghit = g["hit"][idx] == 1
    both = ghit & rhit
    p = o_np[idx][both].astype(np.float64) + g["depth"][idx][both, None] * v_np[idx][both].astype(np.float64)
    na = np.degrees(np.arccos(np.clip(np.sum(g["normal"][idx][both] * _torus_normal(p), axis=1), -1, 1)))
    render = {"ms_median": round(sorted(times)[2], 4), "rays_traced": int(inbox.size),
              "hits": int(g["hit"].astype(np.int64).sum()),
              "sample": f"every 8th row ({idx.size} rays) against an exact float64 sphere trace of the torus",
              "mask_agreement_vs_exact": float(np.mean(ghit == rhit)),
              "depth_abs_err_mean": float(np.mean(np.abs(g["depth"][idx][both] - rtau[both]))) if both.any() else None,
              "depth_abs_err_max": float(np.max(np.abs(g["depth"][idx][both] - rtau[both]))) if both.any() else None,
              "normal_angle_mean_deg_vs_exact": float(np.mean(na)) if both.any() else None}
    log(f"[fit-full] render 1080p: {render}")
    return {"steps": steps, "wall_s": round(wall, 2), "ms_per_step_incl_sampling": round(wall * 1e3 / steps, 3),
            "loss_history": hist, "quality_held_out": quality, "render_1080p_fp32": render}


# The paper's Table 3 (RTX 3090, trained models, 512x512, precision not
# stated): frames per second.  Context only, not a target.
PAPER_TABLE3_FPS = {"table3_256x3": 19.8, "table3_64x1": 128.8, "table3_64x1_256x1": 73.1,
                    "table3_64x1_256x2": 53.0, "table3_64x1_256x3": 41.6, "table3_64x1_256x1_256x3": 39.1}


def errors_vs_oracle(out, ref):
    """Mask agreement, max depth error and normal angles of GPU outputs against
    the oracle on the same rays."""
    import numpy as np
    hit, rhit = out["hit"] == 1, ref["hit"] == 1
    both = hit & rhit
    a64, b64 = out["normal"][both].astype(np.float64), ref["normal"][both]
    ang = np.degrees(np.arctan2(np.linalg.norm(np.cross(a64, b64), axis=1), np.sum(a64 * b64, axis=1)))
    return {"rays": int(hit.size), "mask_agreement": round(float(np.mean(hit == rhit)), 6),
            "depth_max_abs_err": float(np.abs(out["depth"][both] - ref["depth"][both]).max()) if both.any() else 0.0,
            "normal_angle_mean_deg": float(ang.mean()) if both.any() else 0.0,
            "normal_angle_max_deg": float(ang.max()) if both.any() else 0.0, "common_hits": int(both.sum())}


def run_extra_workload(name, forms, steps, warmup, rows_every, frames=None):
    """Another configuration in the default run, timed like the headline frame
    (one trace_rays call over all its rays), with its errors against the oracle
    on every rows_every-th row (of the listed frames)."""
    import numpy as np
    import torch
    import nnm_inputs as ni
    from oracle import tracing as orc
    scene = ni.make_scene(name)
    o_np, v_np, t_np = scene.rays()
    dev = torch.device("cuda", 0)
    o, v = torch.from_numpy(o_np).to(dev), torch.from_numpy(v_np).to(dev)
    t = torch.from_numpy(t_np).to(dev) if t_np is not None else None
    n = o_np.shape[0]
    log(f"[{name}] {n} rays")
    runs = {f: run_form(scene, f, o, v, t, steps, warmup) for f in forms}
    del o, v, t
    per_frame = scene.width * scene.height
    fr = np.asarray(frames if frames is not None else [0])
    rows = np.arange(rows_every // 2, scene.height, rows_every)
    idx = (fr[:, None, None] * per_frame + rows[None, :, None] * scene.width
           + np.arange(scene.width)[None, None, :]).reshape(-1)
    c0 = time.perf_counter()
    ref = orc.trace(scene, o_np[idx], v_np[idx], None if t_np is None else t_np[idx])
    oracle_s = time.perf_counter() - c0
    res = {"workload": name, "rays": n, "oracle_sample": f"every {rows_every}th row of frames {fr.tolist()} "
                                                      f"({idx.size} rays, {oracle_s:.1f} s on the host)",
           "forms": {}}
    for f, r in runs.items():
        err = errors_vs_oracle({k: val[idx] for k, val in r["outputs"].items()}, ref)
        res["forms"][f] = {"rays_per_s": round(r["rays_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                           "timing": r["timing"], "hits": r["hits"], "evals_per_level": r["evals_per_level"],
                           "roofline": roofline(r),
                           "kernels": [{k2: (round(v2, 5) if isinstance(v2, float) else v2) for k2, v2 in k.items()}
                                       for k in r["kernels"]],
                           "errors_vs_oracle": err}
        log(f"[{name} {f}] {r['rays_per_s'] / 1e6:.1f} Mrays/s; vs oracle {err}")
    return res


def run_table3(precisions, steps=20, warmup=3, oracle_rows_every=8):
    """The rows of Table 3 at 512x512 in fixed-iteration mode (20 steps on the
    first net, 5 on the second in the last row; the last net of a nested row
    gives the normals only), timed per call with HIP events."""
    import numpy as np
    import torch
    import nnm_inputs as ni
    import paper_2201_09147_amd as nnm
    from oracle import tracing as orc
    dev = torch.device("cuda", 0)
    rows = []
    for name, (nets, iters, normal) in ni.TABLE3_ROWS.items():
        scene = ni.make_scene(name)
        o_np, v_np, _ = scene.rays()
        o, v = torch.from_numpy(o_np).to(dev), torch.from_numpy(v_np).to(dev)
        final = len(iters) - 1
        row = {"scene": name, "nets": [f"({w},{k})" for w, k in nets], "iterations": iters,
               "normal_net": normal, "paper_fps_rtx3090": PAPER_TABLE3_FPS[name]}
        for prec in precisions:
            stack = nnm.load_siren_stack(scene, prec, 0)
            prm = nnm.TraceParams(scene.step_scale, scene.eps, scene.far, scene.max_steps, final, normal,
                                  iterations=iters)
            for _ in range(warmup):
                out = nnm.render(stack, o, v, params=prm)
            times = []
            for _ in range(steps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                out = nnm.render(stack, o, v, params=prm)
                b.record()
                times.append((a, b))
            torch.cuda.synchronize()
            ms = sorted(a.elapsed_time(b) for a, b in times)[steps // 2]
            row[prec] = {"ms_median": round(ms, 4), "fps": round(1e3 / ms, 1),
                         "mrays_per_s": round(o_np.shape[0] / (ms * 1e-3) / 1e6, 1),
                         "hits": int(out["hit"].to(torch.int64).sum().item())}
            if oracle_rows_every:
                if "_ref" not in row:
                    rws = np.arange(oracle_rows_every // 2, scene.height, oracle_rows_every)
                    idx = (rws[:, None] * scene.width + np.arange(scene.width)[None, :]).reshape(-1)
                    row["_idx"] = idx
                    row["_ref"] = orc.trace(scene, o_np[idx], v_np[idx], final_level=final, normal_level=normal,
                                            iterations=iters)
                idx = row["_idx"]
                g = {k: val.cpu().numpy()[idx] for k, val in out.items() if val is not None}
                row[prec]["errors_vs_oracle"] = errors_vs_oracle(g, row["_ref"])
            stack.close()
        row.pop("_ref", None)
        row.pop("_idx", None)
        log(f"[table3] {name}: " + ", ".join(f"{p_} {row[p_]['fps']} FPS" for p_ in precisions)
            + f" (paper, RTX 3090: {row['paper_fps_rtx3090']} FPS)")
        rows.append(row)
    return rows


def run_nesting(workload, precision, n=100_000_000):
    """Sampled sup |f_j - f_{j-1}| over [-1.5, 1.5]^3 for every adjacent pair of
    the stack (nnm_sup_abs_diff, 1e8 points each) and the thresholds of
    Proposition 1, beside the deltas the stack was built with."""
    import torch
    import nnm_inputs as ni
    import paper_2201_09147_amd as nnm
    scene = ni.make_scene(workload)
    stack = nnm.load_siren_stack(scene, precision, 0)
    pairs = []
    for j in range(1, stack.m):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sup = nnm.nnm_sup_abs_diff(stack, j, j - 1, n, 1000 + j, -1.5, 1.5)
        ms = (time.perf_counter() - t0) * 1e3
        pairs.append({"levels": [j - 1, j], "sup_abs_diff": sup, "points": n, "ms": round(ms, 2),
                      "points_per_s": round(n / (ms * 1e-3), 1)})
        log(f"[nesting] sup |f{j} - f{j - 1}| over 1e8 points = {sup:.6f} ({ms:.1f} ms)")
    deltas = nnm.nnm_nesting_thresholds(1, [0.0] + [p_["sup_abs_diff"] for p_ in pairs], 1e-4)
    stack.close()
    return {"workload": workload, "precision": precision, "pairs": pairs,
            "prop1_deltas": [round(d, 6) for d in deltas],
            "configured_deltas": [lv.delta for lv in scene.levels[:-1]]}


def run_mesh(workload, precision, res=512, steps=10, warmup=2):
    """Neural normal mapping onto a triangle mesh (Sec. 5, Fig. 5): the coarse
    (64,1) level on a res^3 grid (nnm_grid_values), its marching-tetrahedra
    mesh (nnm_mesh_extract), and the fine level's normals at the vertices
    (neural_normal_map).  Each stage is timed with HIP events on the stream the
    kernels run on.  Quality: normals of the coarse level (the mesh's own
    surface) and the mapped fine normals, both against the fine level's normal
    at the vertex projected onto the fine surface (two Newton steps along the
    gradient), as mean angle and mean squared difference of unit normals."""
    import numpy as np
    import torch
    import nnm_inputs as ni
    import paper_2201_09147_amd as nnm
    scene = ni.make_scene(workload)
    coarse, fine = len(scene.levels) - 2, len(scene.levels) - 1
    stack = nnm.load_siren_stack(scene, precision, 0)
    dev = torch.device("cuda", 0)
    lo, hi = -1.0, 1.0
    vals = torch.empty((res, res, res), dtype=torch.float32, device=dev)
    nnm.nnm_grid_values(stack, coarse, res, lo, hi, values=vals)
    V, T = nnm.extract_mesh(vals, lo, hi)
    nv, nt = int(V.shape[0]), int(T.shape[0])
    verts = torch.empty((nv, 3), dtype=torch.float32, device=dev)
    tris = torch.empty((nt, 3), dtype=torch.int32, device=dev)
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    normals = torch.empty((nv, 3), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        for _ in range(warmup):
            fn()
        ms = []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    ms_grid = timed(lambda: nnm.nnm_grid_values(stack, coarse, res, lo, hi, values=vals))
    ms_ext = timed(lambda: nnm.nnm_mesh_extract(vals, lo, hi, 0.0, verts, tris, counts))
    ms_nrm = timed(lambda: nnm.neural_normal_map(stack, fine, verts, normal=normals))
    ms_all = timed(lambda: (nnm.nnm_grid_values(stack, coarse, res, lo, hi, values=vals),
                            nnm.nnm_mesh_extract(vals, lo, hi, 0.0, verts, tris, counts),
                            nnm.neural_normal_map(stack, fine, verts, normal=normals)))
    torch.cuda.synchronize()
    assert counts.cpu().tolist() == [nv, nt]
    # quality against the fine surface
    coarse_n = nnm.neural_normal_map(stack, coarse, verts)
    x = verts.clone()
    val = torch.empty(nv, dtype=torch.float32, device=dev)
    grad = torch.empty((nv, 3), dtype=torch.float32, device=dev)
    for _ in range(2):
        nnm.analytic_normal(stack, fine, x, None, val, grad)
        x = x - (val / grad.square().sum(1).clamp_min(1e-12))[:, None] * grad
    ref_n = nnm.neural_normal_map(stack, fine, x)
    nnm.analytic_normal(stack, fine, x, None, val, grad)
    torch.cuda.synchronize()

    def stats(a):
        cosv = (a * ref_n).sum(1).clamp(-1, 1)
        ang = torch.rad2deg(torch.acos(cosv))
        return {"angle_mean_deg": round(float(ang.mean()), 4), "angle_p99_deg": round(float(ang.quantile(0.99)), 4)
                if nv <= 1 << 24 else None, "mse": float((a - ref_n).square().sum(1).mean())}

    q_coarse, q_nnm = stats(coarse_n), stats(normals)
    hflops = normal_hidden_flops(scene.levels[fine].net)
    tflops = hflops * nv / (ms_nrm * 1e-3) / 1e12
    peak = 2500.0 if precision in ("bf16", "fp16") else 157.3
    ext_bytes = 4 * res ** 3 + 12 * nv + 12 * nt
    out = {"workload": f"{workload} levels {coarse} -> {fine}", "precision": precision, "grid": res,
           "vertices": nv, "triangles": nt,
           "ms": {"grid_values": round(ms_grid, 4), "extract": round(ms_ext, 4), "neural_normal_map": round(ms_nrm, 4),
                  "all": round(ms_all, 4)},
           "grid_nodes_per_s": round(res ** 3 / (ms_grid * 1e-3), 1),
           "mapped_vertices_per_s": round(nv / (ms_nrm * 1e-3), 1),
           "normal_roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": peak, "unit": "TFLOP/s",
                               "frac": round(tflops / peak, 4)},
           "extract_roofline": {"bound": "hbm", "achieved": round(ext_bytes / (ms_ext * 1e-3) / 1e9, 1),
                                "peak": 8000.0, "unit": "GB/s",
                                "frac": round(ext_bytes / (ms_ext * 1e-3) / 8e12, 4)},
           "fine_surface_residual_max": float(val.abs().max()),
           "quality_vs_fine_surface": {"coarse_normals": q_coarse, "mapped_normals": q_nnm}}
    log(f"[mesh {precision}] {res}^3 grid {ms_grid:.3f} ms, extract {ms_ext:.3f} ms ({nv} verts, {nt} tris), "
        f"normals {ms_nrm:.3f} ms ({tflops:.1f} TFLOP/s), all {ms_all:.3f} ms; normals vs the fine surface: "
        f"coarse {q_coarse['angle_mean_deg']:.4f} deg (MSE {q_coarse['mse']:.3e}), mapped "
        f"{q_nnm['angle_mean_deg']:.4f} deg (MSE {q_nnm['mse']:.3e})")
    stack.close()
    return out


def _clip_to_box(o_np, v_np):
    """Entry and exit parameters of each ray with the box [-1, 1]^3 (slab test)."""
    import numpy as np
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / v_np.astype(np.float64)
        t1 = (-1.0 - o_np) * inv
        t2 = (1.0 - o_np) * inv
    t_in = np.maximum(np.max(np.minimum(t1, t2), axis=1), 0.0)
    t_out = np.min(np.maximum(t1, t2), axis=1)
    return t_in, t_out


def run_capacity(steps=4000, omega0=10.0):
    """Capacity-sequence training (Sec. 3.3): the three shapes of the nested
    stack, (32,1), (64,1) and (256,2), fitted to the torus on the same batches
    (first-layer frequency omega0 for all three: a smoother starting basis than
    30 keeps the fits' sup error off the corners of the training box); nesting
    thresholds from the sampled sup |torus - f_j| by Proposition 2; then
    multiscale sphere tracing of the trained stack at 1080p against single-
    level tracing of the finest net and against the exact torus."""
    import numpy as np
    import torch
    import nnm_inputs as ni
    import paper_2201_09147_amd as nnm
    from paper_2201_09147_amd import capacity as cap
    scene = ni.make_scene("fit_torus_256x2")
    ns, nu, lr = scene.extra["n_surf"], scene.extra["n_unif"], scene.extra["lr"]
    dev = torch.device("cuda", 0)
    # width, sine layers, init seed, Adam lr (the small nets learn slowly at 1e-4)
    shapes = [(32, 2, 11, 1e-3), (64, 2, 12, 1e-3), (256, 3, 13, lr)]
    nets = [ni.siren_init(seed, 3, w, k, 1.0, normalise=False, omega0=omega0) for w, k, seed, _ in shapes]
    t0 = time.perf_counter()
    params, last = cap.fit_sequence(nets, [sh[3] for sh in shapes], steps, lambda i: ni.torus_batch(i, ns, nu),
                                    max_points=ns + nu,
                                    log=lambda i, ls: log(f"[capacity] step {i}: " + " | ".join(
                                        f"({n_.width},{n_.n_sine - 1}) {l:.4f}" for n_, l in zip(nets, ls))))
    wall = time.perf_counter() - t0
    fitted = [ni.SirenNet(3, n_.width, n_.n_sine, ni.unflatten_params(p_, 3, n_.width, n_.n_sine))
              for n_, p_ in zip(nets, params)]
    final_loss = [[round(float(x), 6) for x in l] for l in last]

    def make(levels, deltas):
        lv = [ni.SceneLevel(n_, 1.0, d) for n_, d in zip(levels, deltas)]
        return ni.Scene("capacity_torus", lv, 1920, 1080, r0=0.0, base_sphere=False)

    # thresholds on the training domain [-1, 1]^3: Proposition 2 from the sampled
    # sup |torus - f_j| (the nets approximate one known SDF), and Proposition 1
    # from the sampled sup |f_j - f_(j-1)| beside it; the render uses Proposition 2
    d_p2, sups_p2 = cap.nest_by_proposition2([nnm.LevelSpec(3, n_.width, n_.n_sine, n_.flat(), 1.0, 0.0)
                                              for n_ in fitted], "torus", ni.torus.R_MAJOR, ni.torus.R_MINOR,
                                             1 << 26, 77, -1.0, 1.0, margin=1e-3)
    probe = nnm.load_siren_stack(make(fitted, [1.0, 0.5, 0.0]), "fp32", 0, lipschitz_max=0.0)
    d_p1, sups_p1 = nnm.nesting_thresholds(probe, 1 << 26, 77, -1.0, 1.0, margin=1e-3)
    probe.close()
    deltas = d_p2[:2]
    log(f"[capacity] sup |torus - f_j| = {[round(x, 5) for x in sups_p2]}: Prop. 2 deltas {deltas}; "
        f"sup |f_j - f_(j-1)| = {[round(x, 5) for x in sups_p1]}: Prop. 1 deltas {d_p1[:2]}")
    o_np, v_np, _ = make(fitted, deltas + [0.0]).rays()
    t_in, t_out = _clip_to_box(o_np, v_np)
    inbox = np.flatnonzero(t_out > t_in)
    o = torch.from_numpy((o_np[inbox] + t_in[inbox, None] * v_np[inbox]).astype(np.float32)).to(dev)
    v = torch.from_numpy(np.ascontiguousarray(v_np[inbox])).to(dev)
    # Algorithm 1 expects rays to start outside the coarse band |f_1| <= delta_1
    probe = nnm.load_siren_stack(make(fitted, deltas + [0.0]), "fp32", 0, lipschitz_max=0.0)
    f1 = torch.empty(o.shape[0], dtype=torch.float32, device=dev)
    nnm.nnm_net_eval(probe, 0, o, None, f1, None)
    start_outside = float((f1 > deltas[0]).float().mean().item())
    probe.close()
    log(f"[capacity] rays starting outside the coarse band: {start_outside:.4f}")
    rows = np.arange(0, 1080, 8)
    idx = (rows[:, None] * 1920 + np.arange(1920)[None, :]).reshape(-1)
    rhit, rtau = _torus_trace_exact(o_np[idx], v_np[idx], scene.step_scale, scene.eps, scene.far)
    out_rows = {}
    for label, sc in (("multiscale 3-level", make(fitted, deltas + [0.0])), ("single (256,2)", make(fitted[2:], [0.0]))):
        for prec in ("fp32", "bf16"):
            stack = nnm.load_siren_stack(sc, prec, 0, lipschitz_max=0.0)
            prm = nnm.TraceParams(sc.step_scale, sc.eps, sc.far, sc.max_steps)
            out = nnm.render(stack, o, v, params=prm)
            times = []
            for _ in range(7):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                out = nnm.render(stack, o, v, params=prm)
                b.record()
                times.append((a, b))
            torch.cuda.synchronize()
            ms = sorted(a.elapsed_time(b) for a, b in times)[3]
            gb = {k: val.cpu().numpy() for k, val in out.items()}
            stack.close()
            hit = np.zeros(o_np.shape[0], bool)
            depth = np.full(o_np.shape[0], np.inf)
            ins = (gb["hit"] == 1) & (t_in[inbox] + gb["depth"] <= t_out[inbox])
            hit[inbox] = ins
            depth[inbox] = np.where(ins, t_in[inbox] + gb["depth"], np.inf)
            both = hit[idx] & rhit
            out_rows[f"{label} {prec}"] = {
                "ms_median": round(ms, 4), "rays_traced": int(inbox.size), "hits": int(hit.sum()),
                "mask_agreement_vs_exact_torus": float(np.mean(hit[idx] == rhit)),
                "depth_abs_err_mean_vs_exact": float(np.mean(np.abs(depth[idx][both] - rtau[both]))),
                "evals_per_level": gb["steps"].astype(np.int64).sum(axis=0).tolist(), "_depth": depth, "_hit": hit}
            log(f"[capacity] {label} {prec}: {ms:.3f} ms, hits {int(hit.sum())}, mask agreement vs exact "
                f"{out_rows[f'{label} {prec}']['mask_agreement_vs_exact_torus']:.5f}")
    for prec in ("fp32", "bf16"):
        a, b = out_rows[f"multiscale 3-level {prec}"], out_rows[f"single (256,2) {prec}"]
        both = a["_hit"] & b["_hit"]
        a["vs_single_level"] = {"mask_agreement": float(np.mean(a["_hit"] == b["_hit"])),
                                "depth_max_abs_diff": float(np.max(np.abs(a["_depth"][both] - b["_depth"][both]))),
                                "speedup": round(b["ms_median"] / a["ms_median"], 3)}
    for r in out_rows.values():
        r.pop("_depth")
        r.pop("_hit")
    return {"steps": steps, "wall_s": round(wall, 2), "nets": ["(32,1)", "(64,1)", "(256,2)"], "omega0": omega0,
            "rays_starting_outside_coarse_band": start_outside,
            "adam_lr": [sh[3] for sh in shapes],
            "final_loss4": final_loss, "sup_abs_err_vs_torus": sups_p2, "deltas_prop2": d_p2,
            "sup_abs_diff": sups_p1, "deltas_prop1": d_p1, "renders_1080p": out_rows}


def roofline(form):
    dom = max(form["kernels"], key=lambda k: k["avg_ms"])
    peak = PEAK_TFLOPS[form["precision"]]
    return {"bound": "mfma", "achieved": round(dom["tflops"], 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(dom["tflops"] / peak, 5),
            "traffic": measured_traffic(dom["kernel"], form["precision"], form.get("workload", "")),
            "kernel": f"{dom['kernel']} (H={dom['width']}) level {dom['level']}",
            "avg_ms": round(dom["avg_ms"], 4), "flops_per_launch": dom["hidden_flops"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="stack3_1080p")
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--forms", default="fp32,bf16,fp16")
    ap.add_argument("--cpu-rows-every", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nnm-variant", action="store_true",
                    help="skip the neural-normal-mapping variant (trace to level m-2, normals of level m-1)")
    ap.add_argument("--fit-steps", type=int, default=10, help="fitting steps to time (0: skip)")
    ap.add_argument("--no-capacity", action="store_true",
                    help="skip fitting (32,1), (64,1), (256,2) to the torus, nesting them by Prop. 2, 1080p render")
    ap.add_argument("--no-nesting", action="store_true",
                    help="skip sup |f_j - f_(j-1)| of the stack over 1e8 points (Prop. 1 thresholds)")
    ap.add_argument("--no-table3", action="store_true",
                    help="skip the rows of the paper's Table 3 at 512^2 in fixed-iteration mode")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="skip the 4096^2 stress frame and the 16-frame animated call")
    ap.add_argument("--fit-full", action="store_true",
                    help="also run the whole 2000-step fit, its quality and a 1080p render of the fitted net")
    ap.add_argument("--no-mesh", action="store_true",
                    help="skip neural normal mapping onto the 512^3 marching-tetrahedra mesh of the (64,1) level")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): rays are independent, so a "
              f"frame shards across GPUs without communication; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import nnm_inputs as ni

    scene = ni.make_scene(args.workload)
    o_np, v_np, t_np = scene.rays()
    dev = torch.device("cuda", 0)
    o = torch.from_numpy(o_np).to(dev)
    v = torch.from_numpy(v_np).to(dev)
    t = torch.from_numpy(t_np).to(dev) if t_np is not None else None
    n = o_np.shape[0]
    log(f"workload {args.workload}: {n} rays, levels "
        + " |> ".join(f"({l.net.width},{l.net.n_sine - 1})" for l in scene.levels))

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 256 MiB read + 256 MiB written")
        del src, dst

    forms = [f for f in args.forms.split(",") if f]
    if args.precision not in forms:
        forms.append(args.precision)
    results = {f: run_form(scene, f, o, v, t, args.steps, args.warmup) for f in forms}
    # neural normal mapping variant (Sec. 5): trace to the second-finest level's
    # surface, normals of the finest level there
    m = len(scene.levels)
    nnm_res = {}
    if m >= 2 and not args.no_nnm_variant:
        nnm_res = {f: run_form(scene, f, o, v, t, args.steps, args.warmup, final_level=m - 2, normal_level=m - 1)
                   for f in forms}

    def optional(name, fn):
        """A workload beside the headline: its failure is recorded, not fatal."""
        try:
            return fn()
        except Exception as exc:  # noqa: BLE001 - reported in the JSON line
            log(f"[{name}] failed: {exc!r}")
            return {"error": repr(exc)}

    fit = optional("fit", lambda: run_fit(args.fit_steps, 2)) if args.fit_steps > 0 else None
    if isinstance(fit, dict) and "error" not in fit and args.fit_full:
        fit["full"] = optional("fit-full", run_fit_full)
    headline = args.workload == "stack3_1080p"
    nesting = optional("nesting", lambda: run_nesting(args.workload, args.precision)) \
        if not args.no_nesting else None
    capacity = optional("capacity", run_capacity) if not args.no_capacity and headline else None
    table3 = None if args.no_table3 else optional(
        "table3", lambda: run_table3([f for f in ("fp32", "bf16") if f in forms] or [args.precision]))
    extra = None
    if not args.no_extra_workloads and headline:
        xf = [f for f in ("fp32", "bf16") if f in forms] or [args.precision]
        extra = {"stack3_4096sq": optional("stack3_4096sq", lambda: run_extra_workload("stack3_4096sq", xf, 5, 2, 64)),
                 "anim16_1024sq": optional("anim16_1024sq", lambda: run_extra_workload(
                     "anim16_1024sq", xf, 5, 2, 64, frames=[0, 5, 10, 15]))}
    mesh = optional("mesh", lambda: [run_mesh(args.workload, f)
                                     for f in (("fp32", "bf16") if "fp32" in forms else (args.precision,))]) \
        if not args.no_mesh else None

    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        from oracle import tracing as orc
        rows = np.arange(0, scene.height, args.cpu_rows_every)
        idx = (rows[:, None] * scene.width + np.arange(scene.width)[None, :]).reshape(-1)
        threads = orc.max_threads()
        log(f"oracle on {idx.size} rays (every {args.cpu_rows_every}th row), {threads} threads")
        c0 = time.perf_counter()
        ref = orc.trace(scene, o_np[idx], v_np[idx], None if t_np is None else t_np[idx])
        c1 = time.perf_counter()
        # one core, on every 16th ray of the same sample
        idx1 = idx[::16]
        c2 = time.perf_counter()
        orc.trace(scene, o_np[idx1], v_np[idx1], None if t_np is None else t_np[idx1], threads=1)
        c3 = time.perf_counter()
        cpu = {"value": round(idx.size / (c1 - c0), 1), "unit": "rays/s", "cores": threads, "kind": "oracle",
               "sample": f"every {args.cpu_rows_every}th row of the {scene.width}x{scene.height} frame "
                         f"({idx.size} rays), FP64, {c1 - c0:.1f} s",
               "value_1core": round(idx1.size / (c3 - c2), 1),
               "sample_1core": f"every 16th ray of that sample ({idx1.size} rays), 1 thread, {c3 - c2:.1f} s"}
        log(f"oracle: {cpu['value']} rays/s on {threads} threads, {cpu['value_1core']} rays/s on 1")
        for f, r in results.items():
            g = {k: val[idx] for k, val in r["outputs"].items()}
            hit, rhit = g["hit"] == 1, ref["hit"] == 1
            both = hit & rhit
            a64, b64 = g["normal"][both].astype(np.float64), ref["normal"][both]
            ang = np.degrees(np.arctan2(np.linalg.norm(np.cross(a64, b64), axis=1), np.sum(a64 * b64, axis=1)))
            # the roofline's evaluation counts come from the kernels' own steps
            # output; on the sampled rows they are checked against the oracle's
            ge = g["steps"].astype(np.int64).sum(axis=0).tolist()
            oe = ref["steps"].astype(np.int64).sum(axis=0).tolist()
            errors[f] = {"mask_agreement": round(float(np.mean(hit == rhit)), 6),
                         "depth_max_abs_err": float(np.abs(g["depth"][both] - ref["depth"][both]).max()),
                         "normal_angle_mean_deg": float(ang.mean()),
                         "normal_angle_max_deg": float(ang.max()),
                         "common_hits": int(both.sum()),
                         "evals_per_level_on_sample": {"gpu": ge, "oracle": oe,
                                                       "rel_diff": [round((a - b) / max(b, 1), 6)
                                                                    for a, b in zip(ge, oe)]}}
            log(f"[{f}] vs oracle: {errors[f]}")

    nnm_block = None
    if nnm_res:
        nnm_block = {"final_level": m - 2, "normal_level": m - 1, "forms": {}}
        if cpu is not None:
            # oracle of the variant on every (4 x cpu-rows-every)th row of the frame
            every8 = 4 * args.cpu_rows_every
            rows8 = np.arange(0, scene.height, every8)
            idx8 = (rows8[:, None] * scene.width + np.arange(scene.width)[None, :]).reshape(-1)
            log(f"oracle of the NNM variant on {idx8.size} rays (every {every8}th row) ...")
            c0 = time.perf_counter()
            ref8 = orc.trace(scene, o_np[idx8], v_np[idx8], None if t_np is None else t_np[idx8],
                             final_level=m - 2, normal_level=m - 1)
            log(f"oracle of the NNM variant on {idx8.size} rays: {time.perf_counter() - c0:.1f} s")
        for f, r in nnm_res.items():
            full = results[f]["outputs"]
            g = r["outputs"]
            both = (g["hit"] == 1) & (full["hit"] == 1)
            a64, b64 = g["normal"][both].astype(np.float64), full["normal"][both].astype(np.float64)
            ang = np.degrees(np.arctan2(np.linalg.norm(np.cross(a64, b64), axis=1), np.sum(a64 * b64, axis=1)))
            entry = {"rays_per_s": round(r["rays_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                     "timing": r["timing"], "hits": r["hits"], "evals_per_level": r["evals_per_level"],
                     "kernels": r["kernels"],
                     "speedup_vs_full": round(results[f]["ms_per_step"] / r["ms_per_step"], 3),
                     "vs_full_trace": {"mask_agreement": round(float(np.mean(g["hit"] == full["hit"])), 6),
                                       "depth_max_abs_diff": float(np.abs(g["depth"][both] - full["depth"][both]).max()),
                                       "normal_angle_mean_deg": float(ang.mean()),
                                       "normal_angle_p99_deg": float(np.quantile(ang, 0.99))}}
            if cpu is not None:
                gg = {k: val[idx8] for k, val in g.items()}
                hit, rhit = gg["hit"] == 1, ref8["hit"] == 1
                bb = hit & rhit
                a64, b64 = gg["normal"][bb].astype(np.float64), ref8["normal"][bb]
                ang = np.degrees(np.arctan2(np.linalg.norm(np.cross(a64, b64), axis=1), np.sum(a64 * b64, axis=1)))
                entry["errors_vs_oracle"] = {"rays": int(idx8.size), "mask_agreement": round(float(np.mean(hit == rhit)), 6),
                                             "depth_max_abs_err": float(np.abs(gg["depth"][bb] - ref8["depth"][bb]).max()),
                                             "normal_angle_mean_deg": float(ang.mean()),
                                             "normal_angle_max_deg": float(ang.max())}
            nnm_block["forms"][f] = entry
            log(f"[{f} NNM] {entry['rays_per_s'] / 1e6:.1f} Mrays/s, {entry['speedup_vs_full']}x the full trace; "
                f"vs full: {entry['vs_full_trace']}")

    head = results[args.precision]
    line = {
        "metric": METRIC,
        "value": round(head["rays_per_s"], 1),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": args.workload, "rays": n, "width": scene.width, "height": scene.height,
                   "levels": [f"({l.net.width},{l.net.n_sine - 1})" for l in scene.levels],
                   "deltas": [l.delta for l in scene.levels[:-1]], "eps": scene.eps,
                   "step_scale": scene.step_scale, "max_steps_per_level": scene.max_steps},
        "roofline": roofline(head),
        "cpu_baseline": cpu,
        "errors_vs_oracle": errors,
        "fit": fit,
        "nnm_variant": nnm_block,
        "table3_fixed_iterations": table3,
        "extra_workloads": extra,
        "mesh_normal_mapping": mesh,
        "nesting": nesting,
        "capacity_sequence": capacity,
        "timing": head["timing"],
        "rays_per_s_median_call": round(n / (head["timing"]["median_ms"] * 1e-3), 1),
        "forms": {f: {"rays_per_s": round(r["rays_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                      "timing": r["timing"],
                      "roofline": roofline(r), "hits": r["hits"], "evals_per_level": r["evals_per_level"],
                      "frame_mfma_frac": round(sum(k["hidden_flops"] for k in r["kernels"])
                                               / (r["ms_per_step"] * 1e-3) / 1e12
                                               / PEAK_TFLOPS[r["precision"]], 5),
                      "kernels": [{k2: (round(v2, 5) if isinstance(v2, float) else v2) for k2, v2 in k.items()}
                                  for k in r["kernels"]]}
                  for f, r in results.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
