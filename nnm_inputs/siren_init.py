"""SIREN weight generation (input data, not part of the rendering method).

Layout convention (used by every consumer): a network with input size
``d_in``, width ``H`` and ``n_sine`` sine layers has ``n_sine + 1`` affine
layers.  Layer ``i`` holds ``W_i`` with shape ``[out][in]`` (row major) and
``b_i`` with shape ``[out]``:

* layer 0:            ``[H][d_in]``  (omega0 = 30 already folded in)
* layers 1..n_sine-1: ``[H][H]``
* layer n_sine:       ``[1][H]``     (linear output layer)

so that N(x) = W_K h_K + b_K with h_0 = x and h_{i+1} = sin(W_i h_i + b_i),
the MLP form of the paper's Eq.(2) with the sine activation.

The paper's architecture notation (H, k) (Experiments section) means k
square H x H matrices, i.e. ``n_sine = k + 1``.

Initialisation (SIREN scheme, drawn layer by layer, W row major then b, from
one ``default_rng(seed)`` stream, computed in float64 and rounded once to
float32):

* layer 0:  W ~ 30 * U(-1/d_in, 1/d_in),   b ~ 30 * U(-1/sqrt(d_in), 1/sqrt(d_in))
* hidden:   W ~ U(-sqrt(6/H), sqrt(6/H)), b ~ U(-1/sqrt(H), 1/sqrt(H))
* output:   W ~ U(-sqrt(6/H)/30, sqrt(6/H)/30), b ~ U(-1/sqrt(H), 1/sqrt(H))

Optional ``bias_turns = k`` adds 2 pi k to every hidden-layer bias (layers
1..n_sine-1).  sin is 2 pi periodic, so the network stays the same function up
to the float32 rounding of the shifted biases, while its hidden pre-activations
grow to about k revolutions: a stand-in for trained networks whose hidden
arguments are large, exercising a kernel's sine argument reduction.

Lipschitz safety: the scene function is f = |x - c| - r0 + a * N(x), so
|grad f| <= 1 + a * Lip(N) and Lip(N) <= sigma(W_K) * prod_{i<K} sigma(W_i)
(|sin'| <= 1; for layer 0 only the spatial columns count).  The output layer
(W_K and b_K) is scaled by c = min(1, (L_max - 1) / (a * prod sigma)) so that
|grad f| <= L_max = 1.03 holds as a theorem; with a step scale s = 0.9 every
sphere-tracing step is then safe (s * L_max < 1).
"""

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

OMEGA0 = 30.0
LIP_MAX = 1.03
# The bound is enforced on the float32-rounded weights with a tiny margin.
_LIP_MARGIN = 1.0 - 1e-6


@dataclass
class SirenNet:
    d_in: int
    width: int
    n_sine: int
    layers: List[Tuple[np.ndarray, np.ndarray]]  # float32 (W [out][in], b [out])

    @property
    def n_params(self) -> int:
        return param_count(self.d_in, self.width, self.n_sine)

    def flat(self) -> np.ndarray:
        return flatten_params(self.layers)


def layer_shapes(d_in: int, width: int, n_sine: int):
    shapes = []
    for i in range(n_sine + 1):
        fan_in = d_in if i == 0 else width
        fan_out = 1 if i == n_sine else width
        shapes.append((fan_out, fan_in))
    return shapes


def param_count(d_in: int, width: int, n_sine: int) -> int:
    return sum(o * i + o for (o, i) in layer_shapes(d_in, width, n_sine))


def flatten_params(layers) -> np.ndarray:
    parts = []
    for W, b in layers:
        parts.append(np.asarray(W, dtype=np.float32).reshape(-1))
        parts.append(np.asarray(b, dtype=np.float32).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def unflatten_params(flat: np.ndarray, d_in: int, width: int, n_sine: int):
    flat = np.asarray(flat)
    layers = []
    off = 0
    for (o, i) in layer_shapes(d_in, width, n_sine):
        W = flat[off:off + o * i].reshape(o, i)
        off += o * i
        b = flat[off:off + o]
        off += o
        layers.append((W, b))
    if off != flat.size:
        raise ValueError(f"parameter vector has {flat.size} entries, expected {off}")
    return layers


def _spectral_norm(M: np.ndarray) -> float:
    return float(np.linalg.svd(np.asarray(M, dtype=np.float64), compute_uv=False)[0])


def lipschitz_product_bound(layers, spatial_cols: int = 3) -> float:
    """Upper bound of Lip(N) w.r.t. the spatial input: product of spectral norms."""
    prod = 1.0
    for i, (W, _) in enumerate(layers):
        Wd = np.asarray(W, dtype=np.float64)
        if i == 0:
            Wd = Wd[:, :spatial_cols]
        prod *= _spectral_norm(Wd)
    return prod


def siren_init(seed: int, d_in: int, width: int, n_sine: int, amplitude: float,
               lip_max: float = LIP_MAX, normalise: bool = True, bias_turns: int = 0,
               omega0: float = OMEGA0) -> SirenNet:
    """Draw a SIREN with the scheme in the module docstring; float32 result.

    ``omega0`` is the first layer's frequency scale (30 unless a caller asks
    for a smoother starting basis, as the coarse nets of a capacity sequence
    do); the output layer's 1/omega0 factor follows it."""
    if n_sine < 1:
        raise ValueError("a SIREN needs at least one sine layer")
    rng = np.random.default_rng(seed)
    layers64 = []
    for i, (fan_out, fan_in) in enumerate(layer_shapes(d_in, width, n_sine)):
        if i == 0:
            w_lim, b_lim, scale = 1.0 / fan_in, 1.0 / np.sqrt(fan_in), omega0
        elif i < n_sine:
            w_lim, b_lim, scale = np.sqrt(6.0 / fan_in), 1.0 / np.sqrt(fan_in), 1.0
        else:
            w_lim, b_lim, scale = np.sqrt(6.0 / fan_in) / omega0, 1.0 / np.sqrt(fan_in), 1.0
        W = rng.uniform(-w_lim, w_lim, size=(fan_out, fan_in)) * scale
        b = rng.uniform(-b_lim, b_lim, size=(fan_out,)) * scale
        if 0 < i < n_sine:
            b = b + 2.0 * np.pi * bias_turns
        layers64.append((W, b))
    layers = [(W.astype(np.float32), b.astype(np.float32)) for (W, b) in layers64]
    if normalise and amplitude > 0.0:
        bound = lipschitz_product_bound(layers)
        c = min(1.0, (lip_max - 1.0) * _LIP_MARGIN / (amplitude * bound))
        if c < 1.0:
            WK, bK = layers64[-1]
            layers[-1] = ((WK * c).astype(np.float32), (bK * c).astype(np.float32))
    return SirenNet(d_in, width, n_sine, layers)
