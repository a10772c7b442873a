"""CPU pins of the oracle's multiscale sphere tracing (Algorithm 1), normals and
neural normal mapping.

  P1  analytic sphere (all amplitudes 0): closed-form first hit, incidence-bounded
      depth error, hit mask, radial normals, level-switch radii 0.6 + delta_j.
  P4  brute-force first root on tiny images (the first-hit claim after Algorithm 1).
  P5  Lipschitz safety: product bound, sampled |grad f|, certified sampling of
      every step segment.
  P6  nesting (Eq.(1), Proposition 1 with the sampled sup norm).
  P7  multiscale tracing reaches the same surface as plain tracing of f_m.
  P8  neural normal mapping is exact on exact SDFs (|grad f| = 1).
  P12 moving sphere (time input) closed form.
  Status bits: far exit, budget exhaustion, start inside the band.
"""

import numpy as np
import pytest

import nnm_inputs as ni
from oracle import tracing as T
from tests.parity import sphere_eps_counts


def _sphere_hit(o, v, c=None, r=0.6):
    o = np.asarray(o, np.float64)
    v = np.asarray(v, np.float64)
    if c is not None:
        o = o - c
    b = np.sum(o * v, axis=1)
    disc = b * b - np.sum(o * o, axis=1) + r * r
    tstar = -b - np.sqrt(np.maximum(disc, 0.0))
    return disc, tstar, o


def _check_sphere(res, o, v, eps, c=None, r=0.6):
    disc, tstar, orel = _sphere_hit(o, v, c, r)
    hit = res["hit"] == 1
    budget = (res["status"] & T.ST_BUDGET) != 0
    vv = np.asarray(v, np.float64)
    # closest approach of the ray line to the centre
    dmin = np.sqrt(np.maximum(np.sum(orel * orel, 1) - np.sum(orel * vv, 1) ** 2, 0.0))
    mism = hit != (disc > 0)
    # allowed: grazing rays that ran out of budget, or near misses within eps
    ok = budget | (hit & (dmin - r <= eps * 1.0001))
    assert np.all(ok[mism]), np.nonzero(mism & ~ok)
    both = hit & (disc > 0)
    p_star = orel[both] + tstar[both, None] * vv[both]
    cos_inc = np.abs(np.sum(p_star / r * vv[both], axis=1))
    gap = tstar[both] - res["depth"][both]
    assert np.all(gap >= -1e-12)
    assert np.all(gap <= 1.02 * eps / cos_inc + 1e-12), np.max(gap * cos_inc / eps)
    # radial normals at the end point
    p = orel[hit] + res["depth"][hit, None] * vv[hit]
    np.testing.assert_allclose(res["normal"][hit], p / np.linalg.norm(p, axis=1, keepdims=True), atol=1e-12)
    assert np.all(res["normal"][~hit] == 0.0)
    assert np.all(np.isinf(res["depth"][~hit]))
    return mism.mean()


@pytest.mark.parametrize("nlevels", [1, 3])
def test_p1_analytic_sphere(nlevels):
    s = ni.make_scene("stack3_512sq").with_size(96, 96).with_amplitudes([0.0, 0.0, 0.0])
    if nlevels == 1:
        s.levels = s.levels[2:]
    o, v, _ = s.rays()
    res = T.trace(s, o, v)
    frac = _check_sphere(res, o, v, s.eps)
    assert frac <= 1e-3
    # level-switch radii: the point after the last step of level j sits in
    # [0.6 + delta_j, 0.6 + delta_j + eps]
    if nlevels == 3:
        idx = np.nonzero(res["hit"])[0][::97][:24]
        for i in idx:
            lt, ld, ll, tau_end, st = T.trace_log(s, o[i], v[i])
            for j in (0, 1):
                k = np.nonzero(ll == j)[0][-1]
                tau_after = lt[k] + s.step_scale * ld[k]
                rad = np.linalg.norm(o[i].astype(np.float64) + tau_after * v[i].astype(np.float64))
                assert 0.0 <= rad - 0.6 - s.levels[j].delta <= s.eps * 1.0001


def test_p12_moving_sphere():
    s = ni.make_scene("anim16_1024sq").with_size(48, 48, frames=4).with_amplitudes([0.0, 0.0])
    o, v, t = s.rays()
    res = T.trace(s, o, v, t)
    hit_any = 0
    for fidx in range(4):
        sl = slice(fidx * 48 * 48, (fidx + 1) * 48 * 48)
        tt = fidx / 4
        c = 0.2 * np.array([np.cos(2 * np.pi * tt), np.sin(2 * np.pi * tt), 0.0])
        sub = {k: (val[sl] if val is not None else None) for k, val in res.items()}
        _check_sphere(sub, o[sl], v[sl], s.eps, c=c)
        hit_any += sub["hit"].sum()
    assert hit_any > 0


def _first_hit_check(s, o, v, res, level):
    root = T.first_root(s, level, o, v)
    hit = res["hit"] == 1
    budget = (res["status"] & T.ST_BUDGET) != 0
    finite = np.isfinite(root)
    # masks agree except grazing budget-edge rays and near misses within eps
    p_end = o.astype(np.float64) + np.where(hit, res["depth"], 0.0)[:, None] * v.astype(np.float64)
    f_end = T.scene_eval(s, level, p_end, grad=False)
    mism = hit != finite
    ok = (budget & ~hit) | (hit & ~finite & (f_end <= s.eps))
    assert np.all(ok[mism])
    both = hit & finite
    assert both.sum() > 0
    _, g = T.scene_eval(s, level, o[both].astype(np.float64) + root[both, None] * v[both].astype(np.float64))
    cos_inc = np.abs(np.sum(g * v[both].astype(np.float64), axis=1))
    gap = root[both] - res["depth"][both]
    assert np.all(gap >= -1e-9), gap.min()
    assert np.all(gap <= s.eps / cos_inc + 1e-9), np.max(gap * cos_inc)
    return mism.mean()


def test_p4_first_root_single_net():
    s = ni.make_scene("single_64x1_128sq").with_size(32, 32)
    o, v, _ = s.rays()
    res = T.trace(s, o, v)
    assert _first_hit_check(s, o, v, res, 0) <= 0.01


def test_p4_first_root_three_levels():
    s = ni.make_scene("stack3_512sq").with_size(16, 16)
    o, v, _ = s.rays()
    res = T.trace(s, o, v)
    assert _first_hit_check(s, o, v, res, 2) <= 0.02


def test_p5_lipschitz_product_bound_all_scene_levels():
    for name in ["single_64x1_128sq", "stack3_512sq", "anim16_1024sq"]:
        s = ni.make_scene(name)
        for lvl in s.levels:
            # independent recomputation with numpy's SVD on the float32 weights
            prod = 1.0
            for i, (W, _) in enumerate(lvl.net.layers):
                Wd = np.asarray(W, np.float64)
                if i == 0:
                    Wd = Wd[:, :3]
                prod *= np.linalg.norm(Wd, 2)
            assert 1.0 + lvl.amplitude * prod <= 1.03 + 1e-9


def test_p5_sampled_gradient_norm():
    s = ni.make_scene("stack3_512sq")
    rng = np.random.default_rng(21)
    for j, n in [(0, 1 << 16), (1, 1 << 15), (2, 1 << 12)]:
        x = rng.uniform(-1.5, 1.5, size=(n, 3))
        x = x[np.linalg.norm(x, axis=1) > 1e-3]
        _, g = T.scene_eval(s, j, x)
        assert np.linalg.norm(g, axis=1).max() <= 1.03


def test_p5_every_step_segment_is_safe():
    s = ni.make_scene("stack3_512sq").with_size(12, 12)
    o, v, _ = s.rays()
    pts_lv = []
    m = len(s.levels)
    for i in range(o.shape[0]):
        lt, ld, ll, _, _ = T.trace_log(s, o[i], v[i])
        for tau, d, j in zip(lt, ld, ll):
            if d <= 0:
                continue
            u = np.linspace(0.0, s.step_scale * d, 9)
            p = o[i].astype(np.float64)[None, :] + (tau + u)[:, None] * v[i].astype(np.float64)[None, :]
            pts_lv.append((j, p))
    for j in range(m):
        P = np.concatenate([p for (jj, p) in pts_lv if jj == j]) if any(jj == j for jj, _ in pts_lv) else None
        if P is None:
            continue
        delta = 0.0 if j == m - 1 else s.levels[j].delta
        fj = T.scene_eval(s, j, P, grad=False)
        assert np.all(fj - delta > 0.0)
        fm = T.scene_eval(s, m - 1, P, grad=False)
        assert np.all(fm > 0.0)


def test_p6_nesting_prop1():
    s = ni.make_scene("stack3_512sq")
    rng = np.random.default_rng(22)
    deltas = [s.levels[0].delta, s.levels[1].delta, 0.0]
    for j, n in [(0, 1 << 15), (1, 1 << 12)]:
        x = rng.uniform(-1.5, 1.5, size=(n, 3))
        fa = T.scene_eval(s, j, x, grad=False)
        fb = T.scene_eval(s, j + 1, x, grad=False)
        sup = np.abs(fa - fb).max()
        # Proposition 1: delta_j >= delta_{j+1} + sup |f_j - f_{j+1}|
        assert deltas[j] >= deltas[j + 1] + sup, (j, sup)
        # inclusion of the bands (Eq.(1)) on points near the surfaces
        dirs = rng.normal(size=(n, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        y = dirs * rng.uniform(0.6 - 0.06, 0.6 + 0.06, size=(n, 1))
        ga = T.scene_eval(s, j, y, grad=False)
        gb = T.scene_eval(s, j + 1, y, grad=False)
        inner = np.abs(gb) <= deltas[j + 1] if j + 1 < 2 else np.abs(gb) <= 1e-3
        assert np.all(np.abs(ga[inner]) <= deltas[j])


def test_p7_multiscale_equals_single_level():
    s = ni.make_scene("stack3_512sq").with_size(64, 64)
    o, v, _ = s.rays()
    multi = T.trace(s, o, v)
    single = ni.make_scene("stack3_512sq").with_size(64, 64)
    single.levels = single.levels[2:]
    one = T.trace(single, o, v)
    both = (multi["hit"] == 1) & (one["hit"] == 1)
    assert both.sum() > 500
    assert np.abs(multi["depth"][both] - one["depth"][both]).max() <= 1e-4
    assert np.mean(multi["hit"] != one["hit"]) <= 1e-3
    # normals of the same net at nearby end points
    cosang = np.clip(np.sum(multi["normal"][both] * one["normal"][both], axis=1), -1, 1)
    assert np.degrees(np.arccos(cosang)).max() < 0.05


def test_p8_neural_normal_mapping_exact_on_exact_sdf():
    s = ni.make_scene("anim16_1024sq").with_size(40, 40, frames=1).with_amplitudes([0.0, 0.0])
    o, v, _ = s.rays()
    t = np.full(o.shape[0], 0.3, np.float32)
    # trace the coarse level to its zero set, take the fine level's normal there
    res = T.trace(s, o, v, t, final_level=0, normal_level=1)
    hit = res["hit"] == 1
    assert hit.sum() > 100
    t64 = float(np.float32(0.3))  # the time the rays carry
    c = 0.2 * np.array([np.cos(2 * np.pi * t64), np.sin(2 * np.pi * t64), 0.0])
    q = o[hit].astype(np.float64) + res["depth"][hit, None] * v[hit].astype(np.float64)
    # closest point on the fine surface and its normal: straight-line transport
    f_q = T.scene_eval(s, 1, q, t[hit].astype(np.float64), grad=False)
    q_closest = q - f_q[:, None] * res["normal"][hit]
    f_c, g_c = T.scene_eval(s, 1, q_closest, t[hit].astype(np.float64))
    assert np.abs(f_c).max() <= 1e-12
    n_c = g_c / np.linalg.norm(g_c, axis=1, keepdims=True)
    np.testing.assert_allclose(res["normal"][hit], n_c, atol=1e-12)
    np.testing.assert_allclose(res["normal"][hit], (q - c) / np.linalg.norm(q - c, axis=1, keepdims=True),
                               atol=1e-12)


def test_status_far_budget_and_start_inside():
    s = ni.make_scene("stack3_512sq")
    # rays pointing away from the scene leave through far
    o = np.tile(np.array([[0.0, 0.0, 2.5]], np.float32), (4, 1))
    v = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (4, 1))
    r = T.trace(s, o, v)
    assert np.all(r["hit"] == 0) and np.all(r["status"] & T.ST_FAR)
    assert np.all(r["steps"][:, 1:] == 0)
    # a one-step budget: every ray misses by budget on the first level
    s1 = ni.make_scene("stack3_512sq").with_size(8, 8)
    s1.max_steps = 1
    o, v, _ = s1.rays()
    r = T.trace(s1, o, v)
    assert np.all(r["hit"] == 0)
    assert np.all((r["status"] & (T.ST_BUDGET | T.ST_FAR)) != 0)
    # a camera inside the first band sees d < 0 on its first step
    o = np.array([[0.0, 0.0, 0.62]], np.float32)
    v = np.array([[0.0, 0.0, -1.0]], np.float32)
    r = T.trace(s, o, v)
    assert r["status"][0] & T.ST_NEG_STEP


def test_fixed_iterations_sphere_recursion():
    """Fixed-iteration mode on the analytic sphere (all amplitudes 0): every
    level is the recursion tau <- tau + s (|o + tau v| - 0.6 - delta_j) taken
    exactly iters[j] times (delta = 0 on the last traced level), a miss once
    tau > far, and after the last level a hit iff the last |d| <= eps."""
    s = ni.make_scene("stack3_512sq").with_size(48, 40).with_amplitudes([0.0, 0.0, 0.0])
    o, v, _ = s.rays()
    iters = [7, 4, 3]
    for final in (2, 1):
        r = T.trace(s, o, v, final_level=final, normal_level=final, iterations=iters)
        o64, v64 = o.astype(np.float64), v.astype(np.float64)
        tau = np.zeros(o.shape[0])
        alive = np.ones(o.shape[0], bool)
        last_d = np.zeros(o.shape[0])
        for j in range(final + 1):
            delta = 0.0 if j == final else s.levels[j].delta
            for _ in range(iters[j]):
                d = np.linalg.norm(o64 + tau[:, None] * v64, axis=1) - 0.6 - delta
                tau = np.where(alive, tau + s.step_scale * d, tau)
                last_d = np.where(alive, d, last_d)
                alive &= tau <= s.far
        hit = alive & (np.abs(last_d) <= s.eps)
        assert np.array_equal(r["hit"] == 1, hit)
        np.testing.assert_allclose(r["depth"][hit], tau[hit], rtol=0, atol=1e-12)
        assert np.all(np.isinf(r["depth"][~hit]))
        assert np.all(r["steps"][hit][:, :final + 1] == np.array(iters[:final + 1]))
        # hits carry the sphere's radial normal
        p = o64[hit] + tau[hit, None] * v64[hit]
        np.testing.assert_allclose(r["normal"][hit], p / np.linalg.norm(p, axis=1, keepdims=True), atol=1e-12)


def test_budget_pins_on_axis_closed_form():
    """Algorithm 1's per-level budget on the analytic sphere, from a closed form.
    A ray from (0,0,2.5) straight at the centre meets the level-j band at
    distance 1.9 - (0.6 + delta_j) along the ray; each step removes the fraction
    s = 0.9 of what is left, so the k-th evaluation sees d_1 (1 - s)^(k-1).
    With deltas (0.05, 0.01, 0) and eps = 1e-4 the counts are 6, 4, 4:
    1.85e-5 <= eps < 1.85e-4; then d_1 = 0.04 + 1.85e-6 gives 4.0e-5 at k = 4;
    then d_1 = 0.01 + 4.0e-6 gives 1.0004e-4 > eps at k = 3 and 1.0e-5 at k = 4.
    A budget of k - 1 must miss with that level's count equal to the budget;
    a budget of exactly k must hit (the budget counts evaluations)."""
    s = ni.make_scene("stack3_512sq").with_amplitudes([0.0, 0.0, 0.0])
    o = np.array([[0.0, 0.0, 2.5]], np.float32)
    v = np.array([[0.0, 0.0, -1.0]], np.float32)
    need = [6, 4, 4]
    for budget in range(1, 9):
        s.max_steps = budget
        r = T.trace(s, o, v)
        first_short = next((j for j, kj in enumerate(need) if kj > budget), None)
        if first_short is None:
            assert r["hit"][0] == 1 and r["status"][0] == T.ST_HIT, budget
            assert list(r["steps"][0]) == need
            assert abs(r["depth"][0] - 1.9) <= s.eps
        else:
            assert r["hit"][0] == 0 and r["status"][0] == T.ST_BUDGET, budget
            want = [need[j] if j < first_short else (budget if j == first_short else 0) for j in range(3)]
            assert list(r["steps"][0]) == want, (budget, list(r["steps"][0]))
            assert np.isinf(r["depth"][0]) and np.all(r["normal"][0] == 0.0)


def test_budget_pins_recursion_many_rays():
    """The per-level budget on many rays of the analytic sphere: for every
    budget B, a ray hits iff each level's count k_j <= B, a miss at the first
    level with k_j > B is flagged BUDGET with steps = (k_0, ..., k_{j-1}, B, 0...),
    and a hit reports every k_j (so B = k_j - 1, k_j, k_j + 1 all occur)."""
    s = ni.make_scene("stack3_512sq").with_size(40, 40).with_amplitudes([0.0, 0.0, 0.0])
    o, v, _ = s.rays()
    deltas = [s.levels[0].delta, s.levels[1].delta, 0.0]
    need, reach, margin = sphere_eps_counts(o, v, deltas, s)
    keep = reach & (margin > 1e-9) & (need.max(axis=1) <= 40)
    o, v, need = o[keep], v[keep], need[keep]
    kmax = need.max(axis=1)
    assert keep.sum() > 300 and len(np.unique(kmax)) >= 3
    for budget in range(int(kmax.min()) - 1, int(kmax.max()) + 2):
        s.max_steps = budget
        r = T.trace(s, o, v)
        hit = kmax <= budget
        assert np.array_equal(r["hit"] == 1, hit), budget
        assert np.all(r["status"][hit] == T.ST_HIT)
        assert np.array_equal(r["steps"][hit], need[hit].astype(np.uint8))
        assert np.all(r["status"][~hit] == T.ST_BUDGET)
        for i in np.nonzero(~hit)[0]:
            j = int(np.argmax(need[i] > budget))
            want = np.concatenate([need[i, :j], [budget], np.zeros(2 - j, np.int64)])
            assert np.array_equal(r["steps"][i], want.astype(np.uint8)), (budget, i)


def test_nonfinite_ray_status_and_steps():
    """A ray whose scene value is not finite is a miss flagged NONFINITE, and the
    evaluation that produced it counts on its level (a NaN origin fails at the
    first evaluation of level 0; the finite rays beside it are untouched)."""
    s = ni.make_scene("stack3_512sq")
    o = np.array([[np.nan, 0.0, 2.5], [0.0, 0.0, 2.5], [0.0, np.inf, 2.5]], np.float32)
    v = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0], [0.0, 0.0, -1.0]], np.float32)
    r = T.trace(s, o, v)
    for i in (0, 2):
        assert r["hit"][i] == 0 and r["status"][i] == T.ST_NONFINITE
        assert list(r["steps"][i]) == [1, 0, 0]
        assert np.isinf(r["depth"][i]) and np.all(r["normal"][i] == 0.0)
    assert r["hit"][1] == 1
