"""Capacity sequence (Sec. 3.3, "MLPs for a single surface", Proposition 2) on
the GPU: (32,1), (64,1) and (256,2) SIRENs fitted to the analytic torus with
fit_step on the same batches, nested by Proposition 2 from their sampled sup
|torus - f_j|, then traced multiscale.

Gates:
* the thresholds are Proposition 2's recursion of the sampled sups;
* nesting holds on fresh points (not the ones the sups were taken on): every
  point of the delta_(j+1) band of f_(j+1) lies in the delta_j band of f_j,
  with the networks evaluated by the float64 oracle;
* the GPU multiscale trace (fp32, rays started where they enter the training
  box) against the oracle's multiscale trace of the same fitted stack on a
  row sample: hit-mask agreement >= 99.5% over all rays and, on the rays whose
  per-level step counts agree, depth within 1e-4;
* the multiscale trace against single-level tracing of the finest network:
  hit-mask agreement >= 99%.
* at least half of the rays start outside the coarse band (Algorithm 1's
  precondition; the full-size fit in bench.py --capacity has all of them
  outside).
Reduced size (2^14 + 2^16 points per step, 3000 steps, 480x270 rays) so the
test runs in well under a minute; bench.py --capacity runs the full workload.
"""

import numpy as np
import pytest

import nnm_inputs as ni
import paper_2201_09147_amd as nnm
from paper_2201_09147_amd import capacity
from tests.parity import compare, gpu_trace

pytestmark = pytest.mark.gpu

SHAPES = [(32, 2, 11, 1e-3), (64, 2, 12, 1e-3), (256, 3, 13, 2e-4)]  # width, sine layers, seed, Adam lr
OMEGA0 = 10.0


@pytest.fixture(scope="module")
def fitted_sequence():
    nets = [ni.siren_init(seed, 3, w, k, 1.0, normalise=False, omega0=OMEGA0) for w, k, seed, _ in SHAPES]
    ns, nu = 1 << 14, 1 << 16
    params, loss = capacity.fit_sequence(nets, [lr for *_, lr in SHAPES], 3000,
                                         lambda i: ni.torus_batch(i, ns, nu, seed=21), max_points=ns + nu)
    fitted = [ni.SirenNet(3, n.width, n.n_sine, ni.unflatten_params(p, 3, n.width, n.n_sine))
              for n, p in zip(nets, params)]
    print("capacity sequence: final loss sums", [round(float(l.sum()), 5) for l in loss])
    levels = [nnm.LevelSpec(3, n.width, n.n_sine, n.flat(), 1.0, 0.0) for n in fitted]
    deltas, sups = capacity.nest_by_proposition2(levels, "torus", ni.torus.R_MAJOR, ni.torus.R_MINOR,
                                                 n=1 << 24, seed=5, margin=1e-3)
    print("sup |torus - f_j|:", [round(x, 5) for x in sups], "Prop. 2 deltas:", [round(x, 5) for x in deltas])
    return fitted, deltas, sups


def _scene(fitted, deltas, width, height):
    lv = [ni.SceneLevel(n, 1.0, float(d)) for n, d in zip(fitted, deltas[:-1])] + [ni.SceneLevel(fitted[-1], 1.0)]
    return ni.Scene("capacity_torus", lv, width, height, r0=0.0, base_sphere=False)


def test_thresholds_follow_proposition_2(fitted_sequence):
    _, deltas, sups = fitted_sequence
    e = [s + 1e-3 for s in sups]
    m = len(e)
    ref = [0.0] * m
    ref[m - 1] = e[m - 1] + e[m - 2]
    for i in range(m - 1, 0, -1):
        ref[i - 1] = ref[i] + e[i] + e[i - 1]
    assert np.allclose(deltas, ref, rtol=1e-12, atol=1e-12)
    # the fits are real: every sup is below the SDF's own range
    assert max(sups) < 0.5


def test_nesting_holds_on_fresh_points(fitted_sequence):
    from oracle import tracing as orc
    fitted, deltas, _ = fitted_sequence
    rng = np.random.default_rng(404)
    pts = np.concatenate([rng.uniform(-1.0, 1.0, size=(1 << 15, 3)),
                          ni.torus_surface_samples(rng, 1 << 14)[0] + rng.normal(0.0, 0.05, size=((1 << 14), 3))])
    pts = np.clip(pts, -1.0, 1.0)
    f = [orc.net_eval(n, pts, grad=False) for n in fitted]
    for j in range(len(fitted) - 1):
        inner = np.abs(f[j + 1]) <= deltas[j + 1]
        assert inner.sum() > 1000
        assert np.all(np.abs(f[j][inner]) <= deltas[j]), j


def _box_rays(width, height):
    o, v = ni.pinhole_rays(width, height)
    o64, v64 = o.astype(np.float64), v.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = (-1.0 - o64) / v64, (1.0 - o64) / v64
    t_in = np.maximum(np.max(np.minimum(t1, t2), axis=1), 0.0)
    t_out = np.min(np.maximum(t1, t2), axis=1)
    keep = t_out > t_in
    o_in = (o64[keep] + t_in[keep, None] * v64[keep]).astype(np.float32)
    return np.ascontiguousarray(o_in), np.ascontiguousarray(v[keep]), (t_out - t_in)[keep], np.flatnonzero(keep)


def test_multiscale_trace_matches_oracle_and_single_level(fitted_sequence):
    from oracle import tracing as orc
    fitted, deltas, _ = fitted_sequence
    W, H = 480, 270
    sc = _scene(fitted, deltas, W, H)
    o, v, tl, keep = _box_rays(W, H)
    # how many rays start outside the coarse band (Algorithm 1's precondition)
    f0 = orc.net_eval(fitted[0], o.astype(np.float64), grad=False)
    outside = float(np.mean(f0 > deltas[0]))
    print(f"rays starting outside the coarse band: {outside:.4f} (delta_1 = {deltas[0]:.4f})")
    assert outside >= 0.5
    stack = nnm.load_siren_stack(sc, "fp32", 0, lipschitz_max=0.0)
    g = gpu_trace(sc, o, v, stack=stack)
    stack.close()
    single = _scene(fitted[-1:], [0.0], W, H)
    stack = nnm.load_siren_stack(single, "fp32", 0, lipschitz_max=0.0)
    gs = gpu_trace(single, o, v, stack=stack)
    stack.close()
    for d_ in (g, gs):
        d_["hit"] = np.where(d_["depth"] <= tl, d_["hit"], 0).astype(np.uint8)
    rows = np.flatnonzero((keep // W) % 6 == 3)
    r = orc.trace(sc, o[rows], v[rows])
    r["hit"] = np.where(r["depth"] <= tl[rows], r["hit"], 0).astype(np.uint8)
    gr = {k: (val[rows] if val is not None else None) for k, val in g.items()}
    st = compare(gr, r)
    print("multiscale fp32 vs oracle (row sample):", st)
    assert st["hits"] > 1000
    assert st["mask_agreement"] >= 0.995
    same = np.all(gr["steps"] == r["steps"], axis=1) & (gr["hit"] == 1) & (r["hit"] == 1)
    assert same.sum() >= 0.95 * st["common"]
    assert np.abs(gr["depth"][same] - r["depth"][same]).max() <= 1e-4
    both = (g["hit"] == 1) & (gs["hit"] == 1)
    agree = float(np.mean(g["hit"] == gs["hit"]))
    print(f"multiscale vs single-level: mask agreement {agree:.5f}, depth diff max "
          f"{np.abs(g['depth'][both] - gs['depth'][both]).max():.2e}; evaluations per level "
          f"{g['steps'].astype(np.int64).sum(axis=0).tolist()} vs {gs['steps'].astype(np.int64).sum(axis=0).tolist()}")
    assert agree >= 0.99
