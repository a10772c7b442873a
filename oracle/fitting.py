"""Float64 fitting oracle (test infrastructure; see oracle/__init__.py).

The network is the SIREN of the paper's Eq.(2) (phi = sin).  Its spatial
gradient is carried forward as three tangent columns, following Eq.(3)-(4) in
the G_i form of Sec. 5.1 (G_i = phi'(a_i) * (W_i G_{i-1})):

    h_0 = x,  T_0 = d h_0 / d x_spatial        (identity on the 3 spatial inputs)
    a_i = W_i h_i + b_i,    dA_i = W_i T_i
    h_{i+1} = sin(a_i),     T_{i+1} = cos(a_i) * dA_i          (i = 0..K-1)
    N = W_K h_K + b_K,      g = grad N = W_K T_K

Fitting loss of one batch (unit weights, the four terms of the eikonal
fitting setup the paper trains its SDFs with):

    L = mean_surf |N| + mean_surf (1 - n . g) + mean_unif |N - sdf| + mean_unif (|g| - 1)^2

Its parameter gradient is the hand-written reverse mode through both the
primal and the tangent (a double backward, since g is itself a derivative):

    Nbar, gbar from the loss; W_K-bar = Nbar h_K^T + gbar T_K^T; b_K-bar = Nbar
    hbar_K = W_K^T Nbar;  Tbar_K = W_K^T gbar
    for i = K-1 .. 0:
        abar_i  = cos(a_i) * hbar_{i+1} - sin(a_i) * sum_j Tbar_{i+1}[:, j] * dA_i[:, j]
        dAbar_i = cos(a_i) * Tbar_{i+1}
        W_i-bar = abar_i h_i^T + dAbar_i T_i^T;  b_i-bar = abar_i
        hbar_i  = W_i^T abar_i;  Tbar_i = W_i^T dAbar_i

The subgradient of |.| at 0 is 0 and the gradient of |g| at g = 0 is 0.
Adam follows Kingma & Ba (bias-corrected, no weight decay).
"""

import numpy as np


def _as64(layers):
    return [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in layers]


def forward_tangent(layers, x):
    """Per-layer forward state for points x[P, d_in] (float64).

    Returns dict with h (list K+1 of [P, n_in]), T (list K+1 of [P, n_in, 3]),
    a, dA (lists K), N [P], g [P, 3]."""
    L = _as64(layers)
    x = np.asarray(x, np.float64)
    P, d_in = x.shape
    K = len(L) - 1
    T0 = np.zeros((P, d_in, 3))
    for j in range(3):
        T0[:, j, j] = 1.0
    h, T, a, dA = [x], [T0], [], []
    for i in range(K):
        W, b = L[i]
        ai = h[i] @ W.T + b
        dAi = np.einsum("oc,pcj->poj", W, T[i])
        a.append(ai)
        dA.append(dAi)
        h.append(np.sin(ai))
        T.append(np.cos(ai)[:, :, None] * dAi)
    WK, bK = L[K]
    N = h[K] @ WK[0] + bK[0]
    g = np.einsum("c,pcj->pj", WK[0], T[K])
    return {"h": h, "T": T, "a": a, "dA": dA, "N": N, "g": g}


def net_value_grad(layers, x):
    st = forward_tangent(layers, x)
    return st["N"], st["g"]


def loss_terms(N_s, g_s, n_s, N_u, g_u, sdf_u):
    """The four loss terms (surface |N|, surface normal, uniform |N - sdf|, eikonal)."""
    t0 = np.mean(np.abs(N_s)) if N_s.size else 0.0
    # normal term on the unit gradient: 1 - n . grad N / |grad N| (cosine; 0 for a zero gradient)
    gn = np.linalg.norm(g_s, axis=1)
    cos = np.where(gn > 0.0, np.sum(n_s * g_s, axis=1) / np.where(gn > 0.0, gn, 1.0), 0.0)
    t1 = np.mean(1.0 - cos) if N_s.size else 0.0
    t2 = np.mean(np.abs(N_u - sdf_u)) if N_u.size else 0.0
    t3 = np.mean((np.linalg.norm(g_u, axis=1) - 1.0) ** 2) if N_u.size else 0.0
    return np.array([t0, t1, t2, t3])


def loss_adjoints(N_s, g_s, n_s, N_u, g_u, sdf_u):
    """dL/dN and dL/dg per point, surface points first then uniform points."""
    ns, nu = N_s.shape[0], N_u.shape[0]
    Nb_s = np.sign(N_s) / max(ns, 1)
    # d/dg (1 - n . g / |g|) = -(n - (n . u) u) / |g| with u = g / |g|
    n_s = np.asarray(n_s, np.float64)
    gs_norm = np.linalg.norm(g_s, axis=1)
    gs_safe = np.where(gs_norm > 0.0, gs_norm, 1.0)
    u = g_s / gs_safe[:, None]
    proj = n_s - np.sum(n_s * u, axis=1)[:, None] * u
    gb_s = np.where(gs_norm[:, None] > 0.0, -proj / gs_safe[:, None], 0.0) / max(ns, 1)
    Nb_u = np.sign(N_u - sdf_u) / max(nu, 1)
    norm = np.linalg.norm(g_u, axis=1)
    safe = np.where(norm > 0.0, norm, 1.0)
    gb_u = np.where(norm[:, None] > 0.0, 2.0 * (norm - 1.0)[:, None] * g_u / safe[:, None], 0.0) / max(nu, 1)
    return np.concatenate([Nb_s, Nb_u]), np.concatenate([gb_s, gb_u], axis=0)


def backward(layers, x, Nbar, gbar):
    """Parameter gradient given upstream dL/dN [P] and dL/dg [P, 3] (reverse mode
    through primal and tangent).  Returns (list of (dW, db), dx [P, d_in])."""
    L = _as64(layers)
    st = forward_tangent(layers, x)
    K = len(L) - 1
    h, T, a, dA = st["h"], st["T"], st["a"], st["dA"]
    Nbar = np.asarray(Nbar, np.float64)
    gbar = np.asarray(gbar, np.float64)
    grads = [None] * (K + 1)
    WK = L[K][0]
    dWK = (Nbar @ h[K] + np.einsum("pj,pcj->c", gbar, T[K]))[None, :]
    dbK = np.array([Nbar.sum()])
    grads[K] = (dWK, dbK)
    hbar = Nbar[:, None] * WK[0][None, :]
    Tbar = WK[0][None, :, None] * gbar[:, None, :]
    for i in range(K - 1, -1, -1):
        W = L[i][0]
        c, s = np.cos(a[i]), np.sin(a[i])
        abar = c * hbar - s * np.sum(Tbar * dA[i], axis=2)
        dAbar = c[:, :, None] * Tbar
        dW = abar.T @ h[i] + np.einsum("poj,pcj->oc", dAbar, T[i])
        db = abar.sum(axis=0)
        grads[i] = (dW, db)
        hbar = abar @ W
        Tbar = np.einsum("oc,poj->pcj", W, dAbar)
    return grads, hbar


def loss_and_grad(layers, surf_x, surf_n, unif_x, unif_sdf):
    """Loss terms [4] and parameter gradient of the fitting loss (float64)."""
    surf_x = np.asarray(surf_x, np.float64)
    unif_x = np.asarray(unif_x, np.float64)
    x = np.concatenate([surf_x, unif_x], axis=0)
    st = forward_tangent(layers, x)
    ns = surf_x.shape[0]
    N, g = st["N"], st["g"]
    n_s = np.asarray(surf_n, np.float64)
    sdf_u = np.asarray(unif_sdf, np.float64)
    terms = loss_terms(N[:ns], g[:ns], n_s, N[ns:], g[ns:], sdf_u)
    Nbar, gbar = loss_adjoints(N[:ns], g[:ns], n_s, N[ns:], g[ns:], sdf_u)
    grads, _ = backward(layers, x, Nbar, gbar)
    return terms, grads


def adam_update(flat_params, flat_grad, m, v, step, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1).  Returns (params, m, v) as float64."""
    p = np.asarray(flat_params, np.float64)
    g = np.asarray(flat_grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def flatten_grads(grads):
    return np.concatenate([np.concatenate([dW.reshape(-1), db.reshape(-1)]) for dW, db in grads])
