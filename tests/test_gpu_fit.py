"""GPU parity of the fitting path (forward with tangent, double backward,
Adam) against the float64 oracle, plus structural checks.

Gates: value and gradient relative L2 <= 1e-5; parameter gradient relative
L2 <= 1e-4 (float32 accumulation over thousands of points); Adam update within
1e-3 lr of the oracle's update from the oracle gradient, except where the
gradient is below 1e-6 of its largest entry.
"""

import numpy as np
import pytest

import nnm_inputs as ni
import paper_2201_09147_amd as nnm
from oracle import fitting as F
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda", 0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_dev())


def _batch(ns, nu, step=0):
    return ni.torus_batch(step, ns, nu)


@pytest.mark.parametrize("seed,d_in,H,K", [(6, 3, 256, 3), (2, 3, 64, 2), (4, 4, 256, 3)])
def test_forward_tangent(seed, d_in, H, K):
    net = ni.siren_init(seed, d_in, H, K, 1.0, normalise=False)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, size=(3000 + 5, d_in)).astype(np.float32)
    v, g = nnm.siren_forward_tangent(d_in, H, K, _t(net.flat()), _t(x))
    rv, rg = F.net_value_grad(net.layers, x.astype(np.float64))
    assert rel_l2(v.cpu().numpy(), rv) <= 1e-5
    assert rel_l2(g.cpu().numpy(), rg) <= 1e-5


@pytest.mark.parametrize("seed,d_in,H,K", [(6, 3, 256, 3), (2, 3, 64, 2), (4, 4, 256, 3)])
def test_backward_upstream_adjoints(seed, d_in, H, K):
    import torch
    net = ni.siren_init(seed, d_in, H, K, 1.0, normalise=False)
    rng = np.random.default_rng(4)
    n = 2000 + 3
    x = rng.uniform(-1, 1, size=(n, d_in)).astype(np.float32)
    dv = rng.normal(size=n).astype(np.float32)
    dg = rng.normal(size=(n, 3)).astype(np.float32)
    dx = torch.empty((n, d_in), dtype=torch.float32, device=_dev())
    dp, dx = nnm.siren_backward(d_in, H, K, _t(net.flat()), _t(x), _t(dv), _t(dg), dx=dx)
    grads, rdx = F.backward(net.layers, x.astype(np.float64), dv.astype(np.float64), dg.astype(np.float64))
    ref = F.flatten_grads(grads)
    e = rel_l2(dp.cpu().numpy(), ref)
    print(f"backward H={H} K={K} d_in={d_in}: rel L2 dparams {e:.2e}")
    assert e <= 1e-4
    assert rel_l2(dx.cpu().numpy(), rdx) <= 1e-4


@pytest.mark.parametrize("seed,d_in,H,K,n", [(3, 3, 32, 2, 1), (5, 3, 32, 2, 37), (7, 3, 64, 2, 5),
                                              (8, 3, 128, 3, 999), (9, 4, 256, 2, 300)])
def test_backward_per_parameter_block(seed, d_in, H, K, n):
    """Every weight and bias block on its own (the whole-vector norm is dominated
    by the output weights), at every width, down to a single point (one column
    tile), with ragged batch sizes."""
    import torch
    net = ni.siren_init(seed, d_in, H, K, 1.0, normalise=False)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(n, d_in)).astype(np.float32)
    dv = rng.normal(size=n).astype(np.float32)
    dg = rng.normal(size=(n, 3)).astype(np.float32)
    dx = torch.empty((n, d_in), dtype=torch.float32, device=_dev())
    dp, dx = nnm.siren_backward(d_in, H, K, _t(net.flat()), _t(x), _t(dv), _t(dg), dx=dx)
    grads, rdx = F.backward(net.layers, x.astype(np.float64), dv.astype(np.float64), dg.astype(np.float64))
    got = ni.unflatten_params(dp.cpu().numpy().astype(np.float64), d_in, H, K)
    ref = ni.unflatten_params(F.flatten_grads(grads), d_in, H, K)
    for i, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        ew, eb = rel_l2(gw, rw), rel_l2(gb, rb)
        print(f"H={H} K={K} n={n} layer {i}: rel L2 W {ew:.2e}, b {eb:.2e}")
        assert ew <= 1e-4 and eb <= 1e-4, (i, ew, eb)
    assert rel_l2(dx.cpu().numpy(), rdx) <= 1e-4


def _fit(net, max_points):
    return nnm.Fit(net.d_in, net.width, net.n_sine, net.flat(), 0, max_points)


@pytest.mark.parametrize("ns,nu", [(256, 1024), (4096 + 3, 16384 + 5)])
def test_loss_and_gradient(ns, nu):
    import torch
    net = ni.siren_init(6, 3, 256, 3, 1.0, normalise=False)
    sx, sn, ux, us = _batch(ns, nu)
    fit = _fit(net, ns + nu)
    loss = torch.empty(4, dtype=torch.float32, device=_dev())
    dp = torch.empty(net.n_params, dtype=torch.float32, device=_dev())
    fit.loss_grad(_t(sx), _t(sn), _t(ux), _t(us), loss, dp)
    terms, grads = F.loss_and_grad(net.layers, sx, sn, ux, us)
    np.testing.assert_allclose(loss.cpu().numpy(), terms, rtol=1e-5, atol=1e-7)
    e = rel_l2(dp.cpu().numpy(), F.flatten_grads(grads))
    print(f"loss+grad ns={ns} nu={nu}: rel L2 {e:.2e}")
    assert e <= 1e-4
    got = ni.unflatten_params(dp.cpu().numpy().astype(np.float64), 3, 256, 3)
    ref = ni.unflatten_params(F.flatten_grads(grads), 3, 256, 3)
    for i, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        assert rel_l2(gw, rw) <= 1e-4 and rel_l2(gb, rb) <= 1e-4, i
    fit.close()


def test_adam_step_and_determinism():
    import torch
    net = ni.siren_init(6, 3, 256, 3, 1.0, normalise=False)
    sx, sn, ux, us = _batch(512, 2048, 1)
    fit = _fit(net, 4096)
    dp1 = torch.empty(net.n_params, dtype=torch.float32, device=_dev())
    dp2 = torch.empty_like(dp1)
    loss = torch.empty(4, dtype=torch.float32, device=_dev())
    args = (_t(sx), _t(sn), _t(ux), _t(us))
    fit.loss_grad(*args, loss, dp1)
    fit.loss_grad(*args, loss, dp2)
    assert torch.equal(dp1, dp2), "gradient is not bitwise reproducible"
    # the reduction partitions follow the batch, not the workspace size
    other = _fit(net, 1 << 16)
    dp3 = torch.empty_like(dp1)
    other.loss_grad(*args, loss, dp3)
    other.close()
    assert torch.equal(dp1, dp3), "gradient depends on the fit's max_points"
    lr = 1e-4
    fit.step_adam(*args, lr=lr)
    p_gpu = fit.params()
    _, grads = F.loss_and_grad(net.layers, sx, sn, ux, us)
    g = F.flatten_grads(grads)
    p_ref, _, _ = F.adam_update(net.flat(), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    diff = np.abs(p_gpu.astype(np.float64) - p_ref)
    big = np.abs(g) > 1e-6 * np.abs(g).max()
    assert diff[big].max() <= 1e-3 * lr + 1e-7 * np.abs(p_ref[big]).max()
    assert diff.max() <= 2.0 * lr + 1e-6
    assert fit.step == 1
    fit.close()


def test_checkpoint_resume_is_bitwise():
    import torch
    net = ni.siren_init(6, 3, 64, 2, 1.0, normalise=False)
    batches = [tuple(_t(a) for a in _batch(256, 1024, s)) for s in range(4)]
    a = _fit(net, 2048)
    for b in batches:
        a.step_adam(*b, lr=1e-3)
    pa = a.params()
    b_ = _fit(net, 2048)
    for b in batches[:2]:
        b_.step_adam(*b, lr=1e-3)
    ckpt = b_.state()
    c = _fit(ni.siren_init(9, 3, 64, 2, 1.0, normalise=False), 2048)
    c.load_state(*ckpt)
    for b in batches[2:]:
        c.step_adam(*b, lr=1e-3)
    assert c.step == 4
    assert np.array_equal(pa, c.params())
    for f in (a, b_, c):
        f.close()
    del torch


def test_fit_export_writes_a_loadable_network(tmp_path):
    """fit_export after a few steps: the file holds exactly the fit's parameters,
    and a stack loaded from it evaluates the fitted network (against the oracle)."""
    import torch
    net = ni.siren_init(6, 3, 64, 2, 1.0, normalise=False)
    fit = _fit(net, 2048)
    for s in range(3):
        fit.step_adam(*(_t(a) for a in _batch(256, 1024, s)), lr=1e-3)
    path = tmp_path / "fitted.nnmw"
    fit.export(str(path))
    d_in, width, n_sine, params = nnm.nnm_read_net_file(str(path))
    assert (d_in, width, n_sine) == (3, 64, 2)
    assert np.array_equal(params, fit.params())
    fitted = ni.read_net_file(str(path))
    spec = nnm.LevelSpec(d_in, width, n_sine, params, 1.0, 0.0)
    stack = nnm.load_siren_stack([spec], "fp32", 0, base_sphere=False, lipschitz_max=0.0)
    x = np.random.default_rng(1).uniform(-1, 1, size=(1000, 3)).astype(np.float32)
    val = torch.empty(1000, device=_dev())
    nnm.nnm_net_eval(stack, 0, _t(x), None, val, None)
    torch.cuda.synchronize()
    from oracle import tracing as orc
    ref = orc.net_eval(fitted, x.astype(np.float64), grad=False)
    assert np.abs(val.cpu().numpy() - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    stack.close()
    fit.close()


def test_autograd_function_matches_torch_double_backward():
    import torch
    from paper_2201_09147_amd.autograd import siren
    net = ni.siren_init(6, 3, 256, 3, 1.0, normalise=False)
    sx, sn, ux, us = _batch(128, 512, 2)
    x = np.concatenate([sx, ux])
    ns = sx.shape[0]
    params = _t(net.flat()).requires_grad_(True)
    xt = _t(x).requires_grad_(True)
    N, g = siren(xt, params, 3, 256, 3)
    loss = (N[:ns].abs().mean() + (1 - (_t(sn) * g[:ns]).sum(1)).mean() + (N[ns:] - _t(us)).abs().mean()
            + ((g[ns:].norm(dim=1) - 1) ** 2).mean())
    dparams, dx = torch.autograd.grad(loss, [params, xt])
    # float64 CPU reference with torch's own double backward
    ps = []
    for W, b in net.layers:
        ps += [torch.tensor(np.asarray(W, np.float64), requires_grad=True),
               torch.tensor(np.asarray(b, np.float64), requires_grad=True)]
    xr = torch.tensor(x.astype(np.float64), requires_grad=True)
    h = xr
    for i in range(4):
        h = torch.nn.functional.linear(h, ps[2 * i], ps[2 * i + 1])
        if i < 3:
            h = torch.sin(h)
    Nr = h[:, 0]
    (gr,) = torch.autograd.grad(Nr.sum(), xr, create_graph=True)
    lr_ = (Nr[:ns].abs().mean() + (1 - (torch.tensor(sn, dtype=torch.float64) * gr[:ns]).sum(1)).mean()
           + (Nr[ns:] - torch.tensor(us, dtype=torch.float64)).abs().mean() + ((gr[ns:].norm(dim=1) - 1) ** 2).mean())
    refs = torch.autograd.grad(lr_, ps + [xr])
    ref_p = np.concatenate([r.detach().numpy().reshape(-1) for r in refs[:-1]])
    assert rel_l2(dparams.cpu().numpy(), ref_p) <= 1e-4
    assert rel_l2(dx.cpu().numpy(), refs[-1].detach().numpy()) <= 1e-4


def test_full_size_fit_steps_decrease_loss():
    """The fitting workload's batch (2^16 surface + 2^18 uniform points): finite,
    reproducible, and the loss goes down over a few steps."""
    import torch
    scene = ni.make_scene("fit_torus_256x2")
    ns, nu = scene.extra["n_surf"], scene.extra["n_unif"]
    net = scene.levels[0].net
    fit = _fit(net, ns + nu)
    loss = torch.empty(4, dtype=torch.float32, device=_dev())
    hist = []
    for step in range(12):
        b = tuple(_t(a) for a in ni.torus_batch(step, ns, nu))
        fit.step_adam(*b, lr=1e-4, loss4=loss)
        hist.append(loss.cpu().numpy().copy())
    hist = np.array(hist)
    print("loss terms per step:", hist.sum(1))
    assert np.all(np.isfinite(hist))
    assert hist[-1].sum() < hist[0].sum()
    fit.close()


@pytest.fixture(scope="module")
def fitted_torus_net():
    """A reduced C4 fit: the (256,2) SIREN of the torus workload, 1000 Adam steps
    (lr 1e-3) on fresh batches of 2^14 surface + 2^16 uniform points."""
    scene = ni.make_scene("fit_torus_256x2")
    net = scene.levels[0].net
    ns, nu = 1 << 14, 1 << 16
    fit = _fit(net, ns + nu)
    loss = _t(np.zeros(4))
    for step in range(1000):
        fit.step_adam(*(_t(a) for a in ni.torus_batch(step, ns, nu)), lr=1e-3, loss4=loss)
    params = fit.params()
    fit.close()
    print("fitted torus net: final loss terms", loss.cpu().numpy())
    layers = ni.unflatten_params(params, net.d_in, net.width, net.n_sine)
    return ni.SirenNet(net.d_in, net.width, net.n_sine, layers)


def _box_rays(width, height):
    """Camera rays of the torus workload started where they enter the training
    box [-1, 1]^3 (the net is unconstrained outside), and their exit parameter."""
    o, v = ni.pinhole_rays(width, height)
    o64, v64 = o.astype(np.float64), v.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = (-1.0 - o64) / v64, (1.0 - o64) / v64
    t_in = np.maximum(np.max(np.minimum(t1, t2), axis=1), 0.0)
    t_out = np.min(np.maximum(t1, t2), axis=1)
    keep = t_out > t_in
    o_in = (o64[keep] + t_in[keep, None] * v64[keep]).astype(np.float32)
    return np.ascontiguousarray(o_in), np.ascontiguousarray(v[keep]), (t_out - t_in)[keep], np.flatnonzero(keep)


def _exact_torus_trace(o, v, s, eps, far, max_steps):
    """Sphere tracing of the exact torus SDF in float64 (a true distance, so every
    step is safe): the first hit within eps."""
    o64, v64 = o.astype(np.float64), v.astype(np.float64)
    tau = np.zeros(o.shape[0])
    live = np.ones(o.shape[0], bool)
    hit = np.zeros(o.shape[0], bool)
    for _ in range(max_steps):
        d = ni.torus_sdf(o64 + tau[:, None] * v64)
        tau = np.where(live, tau + s * d, tau)
        hit |= live & (d <= eps) & (tau <= far)
        live &= (d > eps) & (tau <= far)
    return hit, np.where(hit, tau, np.inf)


def test_fitted_net_gradients(fitted_torus_net):
    """The analytic gradient of the fitted net (Sec. 5.1) against the oracle's
    (pinned by complex step and finite differences) and against torch autograd
    in float64."""
    import torch
    from oracle import tracing as orc
    fnet = fitted_torus_net
    fs = ni.Scene("fitted_torus", [ni.SceneLevel(fnet, 1.0)], 192, 108, r0=0.0, base_sphere=False)
    stack = nnm.load_siren_stack(fs, "fp32", 0, lipschitz_max=0.0)
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-1, 1, size=(4096, 3)), ni.torus_batch(99, 4096, 0)[0]]).astype(np.float32)
    val = torch.empty(x.shape[0], dtype=torch.float32, device=_dev())
    grad = torch.empty((x.shape[0], 3), dtype=torch.float32, device=_dev())
    nnm.analytic_normal(stack, 0, _t(x), None, val, grad)
    gv, gg = val.cpu().numpy(), grad.cpu().numpy()
    rv, rg = orc.net_eval(fnet, x.astype(np.float64))
    assert rel_l2(gv, rv) <= 1e-5 and rel_l2(gg, rg) <= 1e-5
    xt = torch.tensor(x.astype(np.float64), requires_grad=True)
    h = xt
    for i, (W, b) in enumerate(fnet.layers):
        h = torch.nn.functional.linear(h, torch.tensor(np.asarray(W, np.float64)), torch.tensor(np.asarray(b, np.float64)))
        if i < len(fnet.layers) - 1:
            h = torch.sin(h)
    (tg,) = torch.autograd.grad(h[:, 0].sum(), xt)
    assert rel_l2(gg, tg.numpy()) <= 1e-5
    assert rel_l2(rg, tg.numpy()) <= 1e-10
    stack.close()


def test_fitted_net_render_1080p_gated(fitted_torus_net):
    """The C4 render: the fitted net traced at 1920x1080 in fp32 (rays started at
    the training box, hits past the box exit counted as misses).

    A fitted net has no Lipschitz bound, so a step may jump over a thin part of
    its zero set, and whether it does can depend on rounding.  The gates
    therefore hold on the rays the oracle certifies: every step segment
    [tau, tau + s d] of the oracle's trace has f > 0 at 32 samples (f_m - delta
    > 0 of Algorithm 1's safety condition), and no exit is within float32
    rounding of eps or of the budget.  On those rays the GPU must agree with the
    oracle on hit or miss and within 1e-4 in depth, and its render must match
    the exact torus.  Gated too: the fraction of certified steps over all
    sampled steps (the fit keeps |grad f| near 1), and mask agreement with the
    oracle over all sampled rows."""
    from oracle import tracing as orc
    from tests.parity import compare, gpu_trace
    fnet = fitted_torus_net
    W, H = 1920, 1080
    fs = ni.Scene("fitted_torus", [ni.SceneLevel(fnet, 1.0)], W, H, r0=0.0, base_sphere=False)
    o_all, v_all, t_len, in_box = _box_rays(W, H)
    stack = nnm.load_siren_stack(fs, "fp32", 0, lipschitz_max=0.0)
    g = gpu_trace(fs, o_all, v_all, precision="fp32", stack=stack)
    stack.close()
    # rays of every 30th image row
    sel = np.flatnonzero((in_box // W) % 30 == 7)
    o, v, tl = o_all[sel], v_all[sel], t_len[sel]
    r = orc.trace(fs, o, v)
    gs = {k: (val[sel] if val is not None else None) for k, val in g.items()}
    for d_ in (gs, r):
        d_["hit"] = np.where(d_["depth"] <= tl, d_["hit"], 0).astype(np.uint8)
    st = compare(gs, r)
    print("fitted net 1080p render vs oracle (sampled rows):", st)
    assert st["hits"] > 2000
    assert st["mask_agreement"] >= 0.995
    # certify a subsample of the rays with the oracle's own step log
    cert = np.zeros(sel.size, bool)
    safe = total = 0
    for i in range(0, sel.size, max(1, sel.size // 1500)):
        tau, d, _, tau_end, status = orc.trace_log(fs, o[i], v[i], cap=256)
        u = np.linspace(0.0, 1.0, 33)[None, 1:]
        seg = tau[:, None] + fs.step_scale * np.maximum(d, 0.0)[:, None] * u
        pts = o[i].astype(np.float64)[None, None, :] + seg[:, :, None] * v[i].astype(np.float64)[None, None, :]
        fv = orc.net_eval(fnet, pts.reshape(-1, 3), grad=False).reshape(seg.shape)
        ok = (fv > 0.0).all(axis=1) & (d > 0)
        safe += int(ok.sum())
        total += ok.size
        well = np.all(np.abs(d - fs.eps) > 1e-6) and tau.size < fs.max_steps - 1
        cert[i] = bool(ok.all() and well)
    print(f"fitted net step safety: {safe}/{total} = {safe / total:.4f}; certified rays {cert.sum()}")
    assert safe / total >= 0.97
    assert cert.sum() >= 1000
    assert np.array_equal(gs["hit"][cert], r["hit"][cert])
    both = cert & (gs["hit"] == 1) & (r["hit"] == 1)
    assert both.sum() > 200
    assert np.abs(gs["depth"][both] - r["depth"][both]).max() <= 1e-4
    # against the exact torus on the certified rays
    ehit, etau = _exact_torus_trace(o[cert], v[cert], fs.step_scale, fs.eps, fs.far, 256)
    ehit &= etau <= tl[cert]
    agree = np.mean(gs["hit"][cert] == ehit)
    bt = (gs["hit"][cert] == 1) & ehit
    derr = np.abs(gs["depth"][cert][bt] - etau[bt])
    print(f"fitted net vs exact torus on certified rays: mask agreement {agree:.4f}, depth err mean "
          f"{derr.mean():.2e} max {derr.max():.2e}")
    assert agree >= 0.98 and derr.mean() <= 0.01

