"""GPU parity of multiscale sphere tracing with analytic normals (trace_rays)
against the FP64 oracle, plus structural checks.

Gates (per precision form): hit-mask agreement >= 99.9% over all rays; max
depth error over common hits <= 1e-4 (fp32) / 1e-3 (bf16, fp16); mean normal
angle <= 0.01 deg (fp32) / 0.5 deg (bf16, fp16).
Sizes: the 128^2 single-net scene and the 512^2 three-level scene in full
(both span many wave tiles and end in a ragged tail), the 1080p scene on a
subset of rows, the 16-frame animated scene on a subset of frames and rows.
"""

import numpy as np
import pytest

import nnm_inputs as ni
import paper_2201_09147_amd as nnm
from oracle import tracing as orc
from tests.parity import angle_deg, check_fp32, check_lowp, compare, gpu_trace

pytestmark = pytest.mark.gpu


def _report(tag, st):
    print(f"{tag}: " + ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}" for k, v in st.items()))


def test_single_net_128sq_fp32():
    s = ni.make_scene("single_64x1_128sq")
    o, v, _ = s.rays()
    g = gpu_trace(s, o, v)
    r = orc.trace(s, o, v)
    st = compare(g, r)
    _report("single 128^2 fp32", st)
    check_fp32(st)
    # steps and status agree on rays where both sides agree on the mask
    same = (g["hit"] == r["hit"])
    assert np.mean(g["steps"][same] == r["steps"][same]) >= 0.99
    assert np.mean(g["status"] == r["status"]) >= 0.99


@pytest.mark.parametrize("mode", ["full", "nnm"])
def test_stack3_512sq_fp32(mode):
    s = ni.make_scene("stack3_512sq")
    o, v, _ = s.rays()
    if mode == "full":
        g = gpu_trace(s, o, v)
        r = orc.trace(s, o, v)
    else:
        g = gpu_trace(s, o, v, final_level=1, normal_level=2)
        r = orc.trace(s, o, v, final_level=1, normal_level=2)
    st = compare(g, r)
    _report(f"stack3 512^2 fp32 {mode}", st)
    check_fp32(st)
    assert st["common"] > 50000


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_stack3_1080p_rows(precision):
    s = ni.make_scene("stack3_1080p")
    rows = np.arange(3, 1080, 24)
    o, v, _ = s.rays(rows=rows)
    g = gpu_trace(s, o, v, precision=precision)
    r = orc.trace(s, o, v)
    st = compare(g, r)
    _report(f"stack3 1080p rows/24 {precision}", st)
    (check_fp32 if precision == "fp32" else check_lowp)(st)


def test_stack3_1080p_full_image_sampled_rows():
    """The full 1080p frame in the bench's launch configuration; sampled rows
    checked against the oracle ray by ray."""
    import torch
    s = ni.make_scene("stack3_1080p")
    o, v, _ = s.rays()
    g = gpu_trace(s, o, v, precision="bf16")
    rows = np.arange(5, 1080, 40)
    idx = (rows[:, None] * 1920 + np.arange(1920)[None, :]).reshape(-1)
    r = orc.trace(s, o[idx], v[idx])
    sub = {k: (val[idx] if val is not None else None) for k, val in g.items()}
    st = compare(sub, r)
    _report("stack3 1080p full, sampled rows, bf16", st)
    check_lowp(st)
    # whole-frame invariants: every ray ends in exactly one terminal state
    hit = g["hit"] == 1
    term = g["status"] & (nnm.ST_HIT | nnm.ST_FAR | nnm.ST_BUDGET | nnm.ST_NONFINITE)
    assert np.all(term != 0)
    assert np.all(((g["status"] & nnm.ST_HIT) != 0) == hit)
    assert np.all(np.isinf(g["depth"][~hit])) and np.all(np.isfinite(g["depth"][hit]))
    assert np.all(g["normal"][~hit] == 0)
    np.testing.assert_allclose(np.linalg.norm(g["normal"][hit], axis=1), 1.0, atol=1e-5)
    del torch


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("mode", ["full", "nnm"])
def test_fixed_iterations_match_oracle(precision, mode):
    """Fixed-iteration mode (the paper's experiments): exact step counts per
    level, hits decided by the last |d|, against the oracle's fixed mode."""
    import torch
    s = ni.make_scene("stack3_512sq").with_size(256, 200)
    o, v, _ = s.rays()
    final, normal = (2, 2) if mode == "full" else (1, 2)
    its = [20, 10, 8][:final + 1]
    stack = nnm.load_siren_stack(s, precision, 0)
    dev = torch.device("cuda", 0)
    p = nnm.TraceParams(s.step_scale, s.eps, s.far, s.max_steps, final, normal, iterations=its)
    out = nnm.render(stack, torch.from_numpy(o).to(dev), torch.from_numpy(v).to(dev), None, p)
    g = {k: val.cpu().numpy() for k, val in out.items()}
    r = orc.trace(s, o, v, final_level=final, normal_level=normal, iterations=its)
    st = compare(g, r)
    _report(f"fixed iterations {its} {mode} {precision}", st)
    (check_fp32 if precision == "fp32" else check_lowp)(st)
    hit = g["hit"] == 1
    assert np.all(g["steps"][hit][:, :final + 1] == np.array(its))
    with pytest.raises(nnm.NnmError):
        nnm.render(stack, torch.from_numpy(o[:4]).to(dev), torch.from_numpy(v[:4]).to(dev),
                   params=nnm.TraceParams(iterations=[20, 0, 5]))
    stack.close()


def test_stack3_4096sq_stress_sampled_rows():
    """The 4096x4096 stress run (16.8 M rays) in one call, bf16; every 256th
    row checked against the oracle ray by ray, whole-frame invariants on all."""
    s = ni.make_scene("stack3_4096sq")
    o, v, _ = s.rays()
    g = gpu_trace(s, o, v, precision="bf16")
    rows = np.arange(17, 4096, 256)
    idx = (rows[:, None] * 4096 + np.arange(4096)[None, :]).reshape(-1)
    r = orc.trace(s, o[idx], v[idx])
    sub = {k: (val[idx] if val is not None else None) for k, val in g.items()}
    st = compare(sub, r)
    _report("stack3 4096^2 full, sampled rows, bf16", st)
    check_lowp(st)
    hit = g["hit"] == 1
    assert np.all((g["status"] & (nnm.ST_HIT | nnm.ST_FAR | nnm.ST_BUDGET | nnm.ST_NONFINITE)) != 0)
    assert np.all(np.isinf(g["depth"][~hit])) and np.all(np.isfinite(g["depth"][hit]))
    np.testing.assert_allclose(np.linalg.norm(g["normal"][hit], axis=1), 1.0, atol=1e-5)


def test_anim16_all_frames_one_launch():
    """All 16 frames of the animated scene (16 x 1024^2 rays) in one call, bf16;
    sampled rows of every frame checked against the oracle."""
    s = ni.make_scene("anim16_1024sq")
    o, v, t = s.rays()
    g = gpu_trace(s, o, v, t, precision="bf16")
    n_frame = 1024 * 1024
    rows = np.arange(11, 1024, 128)
    idx = np.concatenate([f * n_frame + (rows[:, None] * 1024 + np.arange(1024)[None, :]).reshape(-1)
                          for f in range(16)])
    r = orc.trace(s, o[idx], v[idx], t[idx])
    sub = {k: (val[idx] if val is not None else None) for k, val in g.items()}
    st = compare(sub, r)
    _report("anim16 all frames, sampled rows, bf16", st)
    check_lowp(st)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_anim16_frames(precision):
    s = ni.make_scene("anim16_1024sq")
    rows = np.arange(7, 1024, 32)
    frames = [0, 5, 11]
    o, v, t = s.rays(rows=rows, frames=frames)
    g = gpu_trace(s, o, v, t, precision=precision)
    r = orc.trace(s, o, v, t)
    st = compare(g, r)
    _report(f"anim16 frames {frames} {precision}", st)
    (check_fp32 if precision == "fp32" else check_lowp)(st)


def test_analytic_sphere_closed_form():
    s = ni.make_scene("stack3_512sq").with_size(256, 256).with_amplitudes([0.0, 0.0, 0.0])
    o, v, _ = s.rays()
    g = gpu_trace(s, o, v)
    oo, vv = o.astype(np.float64), v.astype(np.float64)
    b = np.sum(oo * vv, 1)
    disc = b * b - np.sum(oo * oo, 1) + 0.36
    tstar = -b - np.sqrt(np.maximum(disc, 0))
    hit = g["hit"] == 1
    both = hit & (disc > 0)
    assert np.mean(hit == (disc > 0)) >= 0.999
    p = oo[both] + tstar[both, None] * vv[both]
    cosi = np.abs(np.sum(p / 0.6 * vv[both], 1))
    gap = tstar[both] - g["depth"][both]
    assert np.all(gap >= -2e-6)
    assert np.all(gap <= 1.05 * s.eps / cosi + 2e-6)
    pe = oo[hit] + g["depth"][hit, None] * vv[hit]
    n_ref = pe / np.linalg.norm(pe, axis=1, keepdims=True)
    assert angle_deg(g["normal"][hit], n_ref).max() < 1e-3


def test_deterministic_repeat():
    s = ni.make_scene("stack3_512sq").with_size(320, 200)
    o, v, _ = s.rays()
    import torch
    stack = nnm.load_siren_stack(s, "bf16", 0)
    a = gpu_trace(s, o, v, stack=stack)
    b = gpu_trace(s, o, v, stack=stack)
    stack.close()
    for k in ("depth", "hit", "normal", "steps", "status"):
        assert np.array_equal(a[k], b[k]), k
    del torch


def test_edge_cases():
    import torch
    dev = torch.device("cuda", 0)
    s = ni.make_scene("stack3_512sq")
    stack = nnm.load_siren_stack(s, "fp32", 0)
    # n = 0
    z3 = torch.empty((0, 3), device=dev)
    out = nnm.render(stack, z3, z3)
    assert out["depth"].numel() == 0
    # rays pointing away, a camera inside the first band, a grazing ray
    o = np.array([[0, 0, 2.5], [0, 0, 0.62], [0, 0.6, 2.5], [0.0, 0.0, 2.5]], np.float32)
    v = np.array([[0, 0, 1], [0, 0, -1], [0, 0, -1], [0, 0, -1]], np.float32)
    g = gpu_trace(s, o, v, stack=stack)
    r = orc.trace(s, o, v)
    assert g["hit"][0] == 0 and g["status"][0] & nnm.ST_FAR
    assert g["status"][1] & nnm.ST_NEG_STEP
    assert np.array_equal(g["hit"], r["hit"])
    # a one-step budget: everything misses on the first level
    s1 = ni.make_scene("stack3_512sq").with_size(40, 30)
    s1.max_steps = 1
    o, v, _ = s1.rays()
    g = gpu_trace(s1, o, v, stack=stack)
    assert np.all(g["hit"] == 0)
    assert np.all(g["steps"][:, 1:] == 0)
    # invalid arguments are rejected before any launch
    with pytest.raises(nnm.NnmError):
        nnm.render(stack, torch.zeros((4, 3), device=dev), torch.zeros((4, 3), device=dev),
                   params=nnm.TraceParams(final_level=3))
    with pytest.raises(nnm.NnmError):
        nnm.render(stack, torch.zeros((4, 3), device=dev), torch.zeros((4, 3), device=dev),
                   params=nnm.TraceParams(max_steps=0))
    stack.close()


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_paired_tiles_small_and_ragged_counts(precision):
    """In bf16/fp16 the (32,1) and (64,1) levels trace one ray per lane, as two
    32-column tiles per wave, and evaluate only one tile while a lane half has
    no live ray.  Ray counts below, at and around one and two tiles, and a
    few hundred, take the two-tile and the one-tile paths with either half
    live; every count is compared with the oracle ray by ray (with fewer than
    1,000 rays the mask gate means no ray may disagree)."""
    s = ni.make_scene("stack3_512sq")
    o, v, _ = s.rays()
    rng = np.random.default_rng(2201)
    stack = nnm.load_siren_stack(s, precision, 0)
    hits = 0
    for n in (1, 2, 31, 32, 33, 63, 64, 65, 97, 300):
        idx = rng.choice(o.shape[0], n, replace=False)
        oo, vv = np.ascontiguousarray(o[idx]), np.ascontiguousarray(v[idx])
        g = gpu_trace(s, oo, vv, stack=stack)
        r = orc.trace(s, oo, vv)
        st = compare(g, r)
        check_lowp(st)
        hits += st["hits"]
    stack.close()
    assert hits > 100


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_weight_stationary_matches_streaming(precision):
    """The (256,2) level runs the weight-stationary kernels in bf16/fp16; the
    streaming kernels (kernels="streaming") compute the same sums in another K order."""
    s = ni.make_scene("stack3_512sq").with_size(384, 256)
    o, v, _ = s.rays()
    ws = gpu_trace(s, o, v, precision=precision)
    st = gpu_trace(s, o, v, precision=precision, kernels="streaming")
    both = (ws["hit"] == 1) & (st["hit"] == 1)
    assert np.mean(ws["hit"] == st["hit"]) >= 0.9995
    assert np.abs(ws["depth"][both] - st["depth"][both]).max() <= 2e-4
    assert angle_deg(ws["normal"][both], st["normal"][both]).mean() <= 0.01
    r = orc.trace(s, o, v)
    check_lowp(compare(ws, r))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_concurrent_streams_share_a_stack(precision):
    """trace_rays calls on two streams with one stack, running at the same time,
    give bit-identical outputs to the same calls made one after another (the
    stack is read-only; every call has its own stream-ordered scratch)."""
    import torch
    import paper_2201_09147_amd as nnm
    scene = ni.make_scene("stack3_512sq").with_size(320, 200)
    o, v, _ = scene.rays()
    dev = torch.device("cuda", 0)
    stack = nnm.load_siren_stack(scene, precision, 0)
    cut = 27_001
    parts = [(torch.from_numpy(o[:cut]).to(dev), torch.from_numpy(v[:cut]).to(dev)),
             (torch.from_numpy(o[cut:]).to(dev), torch.from_numpy(v[cut:]).to(dev))]
    ref = [nnm.render(stack, oi, vi) for oi, vi in parts]
    params = nnm.TraceParams(scene.step_scale, scene.eps, scene.far, scene.max_steps)

    def alloc(n):
        return {"depth": torch.empty(n, device=dev), "hit": torch.empty(n, dtype=torch.uint8, device=dev),
                "normal": torch.empty((n, 3), device=dev), "steps": torch.empty((n, 3), dtype=torch.uint8, device=dev),
                "status": torch.empty(n, dtype=torch.uint8, device=dev)}

    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    for _ in range(3):
        outs = [alloc(oi.shape[0]) for oi, _ in parts]
        torch.cuda.synchronize()
        for (oi, vi), out, st in zip(parts, outs, streams):
            with torch.cuda.stream(st):
                nnm.trace_rays(stack, params, oi, vi, None, out["depth"], out["hit"], out["normal"], out["steps"],
                               out["status"], stream=st)
        torch.cuda.synchronize()
        for out, r in zip(outs, ref):
            for key in ("depth", "hit", "normal", "steps", "status"):
                assert torch.equal(out[key], r[key]), key
    stack.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_budget_per_level_matches_oracle(precision):
    """Algorithm 1's per-level budget on the GPU: on the analytic sphere (all
    amplitudes 0) each ray's per-level counts k_j are known; with budgets from
    min k - 1 to max k + 1 (so k_j - 1, k_j and k_j + 1 all occur) hit/miss,
    status and every level's count equal the oracle's on the rays whose exits
    are not within float32 rounding of eps.  fp32 runs the streaming tile on
    every level, bf16 the weight-stationary kernel on the (256,2) level."""
    from tests.parity import sphere_eps_counts
    s = ni.make_scene("stack3_512sq").with_size(64, 52).with_amplitudes([0.0, 0.0, 0.0])
    o, v, _ = s.rays()
    deltas = [s.levels[0].delta, s.levels[1].delta, 0.0]
    need, reach, margin = sphere_eps_counts(o, v, deltas, s)
    keep = reach & (margin > 5e-6) & (need.max(axis=1) <= 40)
    o, v, need = np.ascontiguousarray(o[keep]), np.ascontiguousarray(v[keep]), need[keep]
    kmax = need.max(axis=1)
    assert keep.sum() > 400
    for budget in range(int(kmax.min()) - 1, int(kmax.max()) + 2):
        s.max_steps = budget
        g = gpu_trace(s, o, v, precision=precision)
        r = orc.trace(s, o, v)
        assert np.array_equal(r["hit"] == 1, kmax <= budget)
        assert np.array_equal(g["hit"], r["hit"]), budget
        assert np.array_equal(g["status"], r["status"]), budget
        assert np.array_equal(g["steps"], r["steps"]), budget


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_nonfinite_values_match_oracle(precision):
    """The NONFINITE path: a stack (32,1) |> (64,1) |> 4-D (256,2) with a static
    centre, and rays whose time is NaN on every 7th ray and NaN origins on every
    11th.  A NaN origin fails at level 0's first evaluation; a NaN time only
    reaches the 4-D last level, so those rays trace levels 0-1 normally and fail
    at their first level-2 evaluation (the weight-stationary kernel in bf16).
    Status of those rays equals the oracle's exactly, as do the counts of the
    rays that fail at level 0 and the last-level count (1) of the late ones;
    their level 0-1 counts follow the usual step agreement, and the other rays
    pass the usual gates."""
    base = ni.make_scene("stack3_512sq").with_size(96, 80)
    fine4 = ni.make_scene("anim16_1024sq").levels[1]
    levels = [base.levels[0], base.levels[1], ni.SceneLevel(fine4.net, fine4.amplitude, 0.0)]
    s = ni.Scene("mixed_4d", levels, 96, 80)
    o, v, _ = base.rays()
    o = o.copy()
    n = o.shape[0]
    t = np.full(n, 0.25, np.float32)
    t[::7] = np.nan
    o[3::11, 0] = np.nan
    g = gpu_trace(s, o, v, t, precision=precision)
    r = orc.trace(s, o, v, t)
    bad_o = np.zeros(n, bool)
    bad_o[3::11] = True
    assert np.all(r["status"][bad_o] == orc.ST_NONFINITE) and np.all(r["steps"][bad_o] == [1, 0, 0])
    late = np.zeros(n, bool)
    late[::7] = True
    late &= ~bad_o & ((r["status"] & orc.ST_NONFINITE) != 0)
    assert late.sum() > 20 and np.all(r["steps"][late][:, 2] == 1)
    nf = bad_o | late
    assert np.array_equal(g["status"][nf], r["status"][nf])
    # the failing evaluation is counted on its level and nothing after it
    assert np.array_equal(g["steps"][bad_o], r["steps"][bad_o])
    assert np.all(g["steps"][late][:, 2] == 1)
    # levels 0-1 of the late rays are ordinary float32 tracing: a one-step eps
    # flip against the float64 oracle is allowed on a few rays, as elsewhere
    d01 = np.abs(g["steps"][late][:, :2].astype(int) - r["steps"][late][:, :2].astype(int))
    assert d01.max() <= 1 and np.mean(d01 == 0) >= 0.99, d01.sum()
    assert np.all(g["hit"][nf] == 0) and np.all(np.isinf(g["depth"][nf])) and np.all(g["normal"][nf] == 0)
    keep = ~np.isnan(t) & ~bad_o
    st = compare({k: val[keep] for k, val in g.items()}, {k: val[keep] for k, val in r.items()})
    _report(f"non-finite mix {precision}", st)
    (check_fp32 if precision == "fp32" else check_lowp)(st)


def test_time_dependent_levels_require_times():
    """A stack whose levels read the time (4-D net, moving centre) refuses
    t = NULL with E_INVAL before any launch; a static 3-D stack accepts it."""
    import torch
    dev = torch.device("cuda", 0)
    s = ni.make_scene("anim16_1024sq")
    stack = nnm.load_siren_stack(s, "fp32", 0)
    z = torch.zeros((4, 3), device=dev)
    for call in (lambda: nnm.render(stack, z, z),
                 lambda: nnm.analytic_normal(stack, 1, z, None, torch.empty(4, device=dev), torch.empty((4, 3), device=dev)),
                 lambda: nnm.analytic_normal(stack, 0, z, None, torch.empty(4, device=dev), torch.empty((4, 3), device=dev)),
                 lambda: nnm.neural_normal_map(stack, 1, z, None)):
        with pytest.raises(nnm.NnmError) as e:
            call()
        assert e.value.code == -1 and "time" in str(e.value)
    stack.close()
    s3 = ni.make_scene("stack3_512sq")
    stack = nnm.load_siren_stack(s3, "fp32", 0)
    out = nnm.render(stack, z, torch.tensor([[0.0, 0.0, -1.0]] * 4, device=dev))
    torch.cuda.synchronize()
    assert out["hit"].shape == (4,)
    stack.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("row", sorted(ni.TABLE3_ROWS))
def test_table3_rows_fixed_iterations(row, precision):
    """Every row of the Table-3 replica (fixed iteration counts; the last net of a
    nested row gives the normals only) against the oracle's fixed-iteration mode,
    at 128x128: (256,3) alone, (64,1) alone, (64,1) |> (256,k) for k = 1, 2, 3, and
    the three-net row (20 steps on (64,1), 5 on (256,1), normals of (256,3))."""
    nets, its, normal = ni.TABLE3_ROWS[row]
    s = ni.make_scene(row).with_size(128, 128)
    o, v, _ = s.rays()
    final = len(its) - 1
    g = gpu_trace(s, o, v, precision=precision, final_level=final, normal_level=normal, iterations=its)
    r = orc.trace(s, o, v, final_level=final, normal_level=normal, iterations=its)
    st = compare(g, r)
    _report(f"table3 {row} {precision}", st)
    (check_fp32 if precision == "fp32" else check_lowp)(st)
    hit = g["hit"] == 1
    # the three-net row gives its (256,1) level 5 steps only: about a quarter of
    # the object's rays end within eps then (the oracle's count), so the floor
    # that keeps the comparison meaningful is 500 common hits
    assert st["common"] > 500
    assert np.all(g["steps"][hit][:, :final + 1] == np.array(its))


@pytest.mark.parametrize("name,precision", [("stack2_64x1_128x2_512sq", "fp32"), ("stack2_64x1_128x2_512sq", "bf16"),
                                            ("stack2_64x1_128x2_512sq", "fp16"),
                                            ("table3_64x1_256x1", "fp32"), ("table3_64x1_256x1", "bf16"),
                                            ("table3_64x1_256x3", "fp32"), ("table3_64x1_256x3", "bf16"),
                                            ("stack3_bigarg_512sq", "fp32"), ("stack3_bigarg_512sq", "bf16"),
                                            ("stack3_bigarg_512sq", "fp16"),
                                            ("stack3_wsmid_512sq", "fp32"), ("stack3_wsmid_512sq", "bf16")])
def test_other_widths_and_depths_eps_mode(name, precision):
    """Eps-terminated multiscale tracing with normals for the configurations the
    validator accepts beyond the headline stack: width 128, (256,1) and (256,3)
    fine levels (streaming tile in every form), a (256,2) level whose hidden
    sine arguments reach 300 revolutions (the range-reduced streaming tile in
    fp32, the range-reduced weight-stationary kernels in bf16 / fp16), and a
    (256,2) level in the middle of the stack (in bf16 the weight-stationary
    tracer pushes its rays, with their order keys, to a (256,3) level)."""
    s = ni.make_scene(name).with_size(192, 160)
    o, v, _ = s.rays()
    for final, normal in ((len(s.levels) - 1, len(s.levels) - 1), (len(s.levels) - 2, len(s.levels) - 1)):
        g = gpu_trace(s, o, v, precision=precision, final_level=final, normal_level=normal)
        r = orc.trace(s, o, v, final_level=final, normal_level=normal)
        st = compare(g, r)
        _report(f"{name} final {final} normal {normal} {precision}", st)
        (check_fp32 if precision == "fp32" else check_lowp)(st)
        assert st["common"] > 3000
