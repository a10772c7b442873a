"""CPU pins of the fitting oracle.

  P10 the hand-written reverse mode through primal and tangent against central
      differences of the loss (float64) and against torch float64 autograd with
      create_graph (double backward);
  Adam closed-form first two steps (Kingma & Ba, bias-corrected);
  P11 torus data: closed-form sdf values, unit normals equal to grad sdf,
      area-uniform surface sampling (E[cos v] = r / (2R)).
"""

import numpy as np
import pytest

import nnm_inputs as ni
from oracle import fitting as F


def _batch(ns=48, nu=96, seed=3):
    sx, sn, ux, us = ni.torus_batch(seed, ns, nu)
    return (sx.astype(np.float64), sn.astype(np.float64), ux.astype(np.float64), us.astype(np.float64))


def _net(seed=6):
    return ni.siren_init(seed, 3, 256, 3, 1.0, normalise=False)


def _loss(layers, b):
    x = np.concatenate([b[0], b[2]])
    N, g = F.net_value_grad(layers, x)
    ns = b[0].shape[0]
    return F.loss_terms(N[:ns], g[:ns], b[1], N[ns:], g[ns:], b[3]).sum()


def test_p10_gradient_central_differences():
    net = _net()
    b = _batch()
    layers = [(np.asarray(W, np.float64), np.asarray(bb, np.float64)) for W, bb in net.layers]
    terms, grads = F.loss_and_grad(layers, *b)
    flat_g = F.flatten_grads(grads)
    flat_p = np.concatenate([np.concatenate([W.reshape(-1), bb.reshape(-1)]) for W, bb in layers])
    rng = np.random.default_rng(5)
    idx = rng.choice(flat_p.size, size=64, replace=False)
    shapes = [(W.shape, bb.shape) for W, bb in layers]

    def unflat(p):
        out, off = [], 0
        for ws, bs in shapes:
            nW, nb = int(np.prod(ws)), int(np.prod(bs))
            out.append((p[off:off + nW].reshape(ws), p[off + nW:off + nW + nb].reshape(bs)))
            off += nW + nb
        return out

    for k in idx:
        h = 1e-6 * max(1.0, abs(flat_p[k]))
        pp, pm = flat_p.copy(), flat_p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (_loss(unflat(pp), b) - _loss(unflat(pm), b)) / (2 * h)
        scale = max(abs(flat_g[k]), 1e-3 * np.abs(flat_g).max())
        assert abs(fd - flat_g[k]) <= 1e-6 * scale + 1e-9, (k, fd, flat_g[k])


def test_p10_gradient_matches_torch_double_backward():
    torch = pytest.importorskip("torch")
    net = _net()
    b = _batch(32, 64, 4)
    terms, grads = F.loss_and_grad(net.layers, *b)
    params = []
    for W, bb in net.layers:
        params.append(torch.tensor(np.asarray(W, np.float64), requires_grad=True))
        params.append(torch.tensor(np.asarray(bb, np.float64), requires_grad=True))
    ns = b[0].shape[0]
    x = torch.tensor(np.concatenate([b[0], b[2]]), requires_grad=True)
    h = x
    K = len(net.layers) - 1
    for i in range(K + 1):
        h = torch.nn.functional.linear(h, params[2 * i], params[2 * i + 1])
        if i < K:
            h = torch.sin(h)
    N = h[:, 0]
    (g,) = torch.autograd.grad(N.sum(), x, create_graph=True)
    n_s = torch.tensor(b[1])
    sdf = torch.tensor(b[3])
    loss = (N[:ns].abs().mean() + (1 - (n_s * g[:ns]).sum(1) / g[:ns].norm(dim=1)).mean()
            + (N[ns:] - sdf).abs().mean()
            + ((g[ns:].norm(dim=1) - 1) ** 2).mean())
    tg = torch.autograd.grad(loss, params)
    np.testing.assert_allclose(terms.sum(), loss.item(), rtol=1e-12)
    for i, (dW, db) in enumerate(grads):
        for mine, ref in ((dW, tg[2 * i]), (db, tg[2 * i + 1])):
            ref = ref.numpy()
            scale = np.abs(ref).max()
            assert np.abs(mine - ref).max() <= 1e-10 * scale + 1e-300


def test_adam_closed_form_first_steps():
    p0 = np.array([1.0, -2.0, 0.5, 0.0])
    g1 = np.array([0.3, -1e-3, 2.0, 0.0])
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    p1, m, v = F.adam_update(p0, g1, np.zeros(4), np.zeros(4), 1, lr, b1, b2, eps)
    # step 1: mhat = g, vhat = g^2
    np.testing.assert_allclose(p1, p0 - lr * g1 / (np.abs(g1) + eps), rtol=1e-15)
    g2 = np.array([-0.1, 4e-3, 2.0, 1.0])
    p2, m2, v2 = F.adam_update(p1, g2, m, v, 2, lr, b1, b2, eps)
    mhat = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vhat = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    np.testing.assert_allclose(p2, p1 - lr * mhat / (np.sqrt(vhat) + eps), rtol=1e-14)


def test_p11_torus_closed_forms():
    pts = np.array([[0.5, 0.0, 0.0], [0.7, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, -0.3, 0.0]])
    ref = np.array([-0.2, 0.0, 0.3, np.sqrt(0.25 + 1.0) - 0.2, 0.0])
    np.testing.assert_allclose(ni.torus_sdf(pts), ref, atol=1e-15)
    rng = np.random.default_rng(1)
    sp, sn = ni.torus_surface_samples(rng, 20000)
    assert np.abs(ni.torus_sdf(sp)).max() < 1e-12
    np.testing.assert_allclose(np.linalg.norm(sn, axis=1), 1.0, atol=1e-12)
    h = 1e-6
    fd = np.stack([(ni.torus_sdf(sp[:200] + h * e) - ni.torus_sdf(sp[:200] - h * e)) / (2 * h)
                   for e in np.eye(3)], 1)
    np.testing.assert_allclose(fd, sn[:200], atol=1e-8)
    # area-uniform: E[cos v] = r / (2R) = 0.2; cos v = (rho - R) / r
    cosv = (np.sqrt(sp[:, 0] ** 2 + sp[:, 1] ** 2) - 0.5) / 0.2
    assert abs(cosv.mean() - 0.2) < 4 * np.sqrt(0.5 / 20000)
    up, us = ni.torus_uniform_samples(rng, 1000)
    assert up.min() >= -1 and up.max() <= 1
    np.testing.assert_allclose(us, ni.torus_sdf(up))
