"""CPU pins of the oracle's network value and analytic gradient.

What pins what:
  * parameter counts <-> the paper's "Mem" column (Tables 1 and 3): the (H, k)
    architecture notation;
  * tiny nets with closed forms: weight layout ([out][in] row major), biases,
    layer count, sine activation, 4-D input;
  * torch float64 forward: the Eq.(2) value on the real scene nets;
  * complex-step derivative (Squire & Trapp 1998) and central differences: the
    Eq.(3)-(4) Jacobian chain, independently of its formula.
"""

import os

import numpy as np
import pytest

import nnm_inputs as ni
from oracle import fitting as F
from oracle import tracing as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _net(d_in, layers):
    H = np.asarray(layers[0][0]).shape[0]
    K = len(layers) - 1
    return ni.SirenNet(d_in, H, K, [(np.asarray(W, np.float32), np.asarray(b, np.float32))
                                    for W, b in layers])


def _parse_notation(tok):
    """'(64,1)|>(256,3)' -> [(64, 1), (256, 3)]"""
    out = []
    for part in tok.split("|>"):
        h, k = part.strip("()").split(",")
        out.append((int(h), int(k)))
    return out


def test_param_count_matches_paper_mem_column():
    rows = []
    with open(os.path.join(GOLDEN, "paper_mem_column.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows.append((parts[0], float(parts[1])))
    assert len(rows) == 6
    for model, mem_kb in rows:
        nets = _parse_notation(model)
        # (H, k): k square H x H matrices -> k + 1 sine layers.
        kib = sum(ni.param_count(3, H, k + 1) * 4 / 1024.0 for H, k in nets)
        # The paper's files carry 0.5-1 KiB of overhead per net.
        assert 0.0 <= mem_kb - kib <= 1.0 * len(nets) + 1e-9, (model, mem_kb, kib)
    assert ni.param_count(3, 64, 2) == 4481
    assert ni.param_count(3, 256, 3) == 132865


def test_closed_form_one_sine_layer():
    W0 = [[1.0, 0.0, 0.0], [0.0, 2.0, 0.0]]
    b0 = [0.5, -0.25]
    W1 = [[3.0, -1.0]]
    b1 = [0.125]
    net = _net(3, [(W0, b0), (W1, b1)])
    rng = np.random.default_rng(11)
    x = rng.uniform(-2, 2, size=(64, 3))
    N, g = T.net_eval(net, x)
    ref = 3.0 * np.sin(x[:, 0] + 0.5) - np.sin(2.0 * x[:, 1] - 0.25) + 0.125
    gref = np.stack([3.0 * np.cos(x[:, 0] + 0.5), -2.0 * np.cos(2.0 * x[:, 1] - 0.25), 0 * x[:, 0]], 1)
    np.testing.assert_allclose(N, ref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(g, gref, rtol=0, atol=1e-13)


def test_closed_form_hidden_layer_asymmetric():
    # dyadic values: exact in float32
    W0 = [[0.375, -0.25, 0.125], [0.0625, 0.5, -0.3125]]
    b0 = [0.125, -0.25]
    W1 = [[0.75, -0.5], [0.25, 0.875]]
    b1 = [0.0625, 0.0]
    W2 = [[1.5, -2.0]]
    b2 = [0.3125]
    net = _net(3, [(W0, b0), (W1, b1), (W2, b2)])
    rng = np.random.default_rng(12)
    x = rng.uniform(-3, 3, size=(64, 3))
    s1 = np.sin(0.375 * x[:, 0] - 0.25 * x[:, 1] + 0.125 * x[:, 2] + 0.125)
    s2 = np.sin(0.0625 * x[:, 0] + 0.5 * x[:, 1] - 0.3125 * x[:, 2] - 0.25)
    ref = 1.5 * np.sin(0.75 * s1 - 0.5 * s2 + 0.0625) - 2.0 * np.sin(0.25 * s1 + 0.875 * s2) + 0.3125
    N, _ = T.net_eval(net, x)
    np.testing.assert_allclose(N, ref, rtol=0, atol=1e-13)


def test_closed_form_time_input_and_spatial_gradient():
    # N(x, t) = 2 sin(x + 3 t) + 0.5 sin(y - t); grad is spatial only.
    W0 = [[1.0, 0.0, 0.0, 3.0], [0.0, 1.0, 0.0, -1.0]]
    b0 = [0.0, 0.0]
    W1 = [[2.0, 0.5]]
    b1 = [0.0]
    net = _net(4, [(W0, b0), (W1, b1)])
    rng = np.random.default_rng(13)
    x = rng.uniform(-1, 1, size=(32, 4))
    N, g = T.net_eval(net, x)
    np.testing.assert_allclose(N, 2 * np.sin(x[:, 0] + 3 * x[:, 3]) + 0.5 * np.sin(x[:, 1] - x[:, 3]),
                               atol=1e-13)
    np.testing.assert_allclose(g[:, 0], 2 * np.cos(x[:, 0] + 3 * x[:, 3]), atol=1e-13)
    np.testing.assert_allclose(g[:, 1], 0.5 * np.cos(x[:, 1] - x[:, 3]), atol=1e-13)
    np.testing.assert_allclose(g[:, 2], 0.0, atol=1e-15)


@pytest.mark.parametrize("seed,d_in,H,K", [(0, 3, 64, 2), (3, 3, 256, 3), (4, 4, 256, 3), (1, 3, 32, 2)])
def test_forward_matches_torch_float64(seed, d_in, H, K):
    torch = pytest.importorskip("torch")
    net = ni.siren_init(seed, d_in, H, K, 0.02)
    rng = np.random.default_rng(100 + seed)
    x = rng.uniform(-1.5, 1.5, size=(96, d_in))
    h = torch.from_numpy(x)
    for i, (W, b) in enumerate(net.layers):
        Wt = torch.from_numpy(np.asarray(W, np.float64))
        bt = torch.from_numpy(np.asarray(b, np.float64))
        h = torch.nn.functional.linear(h, Wt, bt)
        if i < K:
            h = torch.sin(h)
    N = T.net_eval(net, x, grad=False)
    np.testing.assert_allclose(N, h[:, 0].numpy(), rtol=0, atol=1e-12 * max(1.0, np.abs(N).max()))


def _complex_step_grad(net, x, hstep=1e-30):
    """d N / d x_k = Im N(x + i h e_k) / h with complex sine (no subtraction error)."""
    out = np.zeros((x.shape[0], 3))
    for k in range(3):
        z = x.astype(np.complex128).copy()
        z[:, k] += 1j * hstep
        h = z
        for i, (W, b) in enumerate(net.layers):
            h = h @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
            if i < net.n_sine:
                h = np.sin(h)
        out[:, k] = h[:, 0].imag / hstep
    return out


@pytest.mark.parametrize("seed,d_in,H,K", [(0, 3, 64, 2), (3, 3, 256, 3), (4, 4, 256, 3), (1, 3, 32, 2)])
def test_gradient_complex_step(seed, d_in, H, K):
    net = ni.siren_init(seed, d_in, H, K, 0.02)
    rng = np.random.default_rng(200 + seed)
    x = rng.uniform(-1.5, 1.5, size=(64, d_in))
    _, g = T.net_eval(net, x)
    gcs = _complex_step_grad(net, x)
    scale = np.abs(gcs).max()
    np.testing.assert_allclose(g, gcs, rtol=0, atol=1e-12 * scale)


def test_gradient_central_differences():
    net = ni.siren_init(2, 3, 64, 2, 0.015)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1.0, 1.0, size=(48, 3))
    _, g = T.net_eval(net, x)
    h = 1e-5
    fd = np.zeros_like(g)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd[:, k] = (T.net_eval(net, x + e, grad=False) - T.net_eval(net, x - e, grad=False)) / (2 * h)
    scale = np.abs(g).max()
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-8 * scale)


def test_two_oracle_gradient_forms_agree():
    """Explicit-Jacobian product (C) and the G_i recursion (numpy) agree."""
    net = ni.siren_init(3, 3, 256, 3, 0.02)
    rng = np.random.default_rng(8)
    x = rng.uniform(-1.2, 1.2, size=(40, 3))
    N, g = T.net_eval(net, x)
    N2, g2 = F.net_value_grad(net.layers, x)
    np.testing.assert_allclose(N, N2, atol=1e-13)
    np.testing.assert_allclose(g, g2, atol=1e-12 * np.abs(g).max())


def test_scene_function_and_gradient():
    s = ni.make_scene("stack3_512sq")
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, size=(50, 3))
    for j, lvl in enumerate(s.levels):
        f, gf = T.scene_eval(s, j, x)
        N, gN = T.net_eval(lvl.net, x)
        r = np.linalg.norm(x, axis=1)
        np.testing.assert_allclose(f, r - 0.6 + lvl.amplitude * N, atol=1e-14)
        np.testing.assert_allclose(gf, x / r[:, None] + lvl.amplitude * gN, atol=1e-14)


def test_scene_moving_centre_inputs():
    s = ni.make_scene("anim16_1024sq")
    rng = np.random.default_rng(10)
    x = rng.uniform(-1, 1, size=(30, 3))
    t = rng.uniform(0, 1, size=30)
    c = 0.2 * np.stack([np.cos(2 * np.pi * t), np.sin(2 * np.pi * t), 0 * t], 1)
    # coarse level: input x - c(t)
    f0, g0 = T.scene_eval(s, 0, x, t)
    N0, gN0 = T.net_eval(s.levels[0].net, x - c)
    r = np.linalg.norm(x - c, axis=1)
    np.testing.assert_allclose(f0, r - 0.6 + 0.005 * N0, atol=1e-14)
    np.testing.assert_allclose(g0, (x - c) / r[:, None] + 0.005 * gN0, atol=1e-14)
    # fine level: 4-D input (x, t)
    f1, g1 = T.scene_eval(s, 1, x, t)
    N1, gN1 = T.net_eval(s.levels[1].net, np.concatenate([x, t[:, None]], 1))
    np.testing.assert_allclose(f1, r - 0.6 + 0.02 * N1, atol=1e-14)
    np.testing.assert_allclose(g1, (x - c) / r[:, None] + 0.02 * gN1, atol=1e-14)
