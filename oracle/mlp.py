"""Warm-start network, FP64 reference (TEST INFRASTRUCTURE ONLY, see oracle/__init__.py).

The learned warm start maps (log10 Kn, x, y) to the steady macroscopic fields
(rho, u_x, u_y) of the cavity, which then seed the solver at equilibrium
(Eqs. 3, 5).  The network is a multilayer perceptron:

    h_0 = tanh(W_0 a + b_0),  h_l = tanh(W_l h_{l-1} + b_l)  (l = 1..L-1),
    y   = W_L h_{L-1} + b_L,

with a the encoded input (3 values), hidden width 128 and four hidden layers
(L = 4).  Training minimises the mean squared error over samples and outputs,
E = (1 / (3 n)) sum_s sum_o (y_so - t_so)^2, with Adam (Kingma & Ba 2015:
first and second moment estimates with bias correction).

Everything here is plain numpy in float64: forward, backward by the chain rule
written out layer by layer, and the Adam update.  ``bf16=True`` rounds the
operands of the hidden-to-hidden products to bfloat16 (round to nearest even)
at exactly the points where the GPU kernels feed its matrix cores; all other
arithmetic stays float64.

Parameters are one flat vector, layer by layer: W_0 (128 x 3, row-major by
output), b_0, W_1 (128 x 128), b_1, ..., W_L (3 x 128), b_L.

Pinned by tests/test_oracle_mlp.py: the gradient against central finite
differences, closed forms of the forward pass for special weights, the
output-bias gradient, Adam's first step and zero-gradient invariance, and the
bfloat16 rounding on values whose rounding is known.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

N_IN, N_OUT = 3, 3


def layer_shapes(width: int = 128, hidden: int = 4) -> List[Tuple[int, int]]:
    """(out, in) of every weight matrix."""
    return [(width, N_IN)] + [(width, width)] * (hidden - 1) + [(N_OUT, width)]


def param_count(width: int = 128, hidden: int = 4) -> int:
    return sum(o * i + o for o, i in layer_shapes(width, hidden))


def unpack(theta: np.ndarray, width: int = 128, hidden: int = 4):
    """Flat vector -> [(W, b), ...] as views."""
    out, k = [], 0
    for o, i in layer_shapes(width, hidden):
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    assert k == theta.size
    return out


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (8 significant bits), nearest even, via float32; returned as float64.

    The value is first rounded to float32 (nearest even), then the low 16 bits of the
    float32 pattern are rounded away: add 0x7fff plus the lowest kept bit, truncate."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    keep = (u >> 16) & 1
    r = ((u + 0x7FFF + keep) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta: np.ndarray, a: np.ndarray, width: int = 128, hidden: int = 4, bf16: bool = False):
    """a: (n, 3).  Returns (y (n, 3), [h_0, ..., h_{L-1}])."""
    layers = unpack(theta, width, hidden)
    hs = []
    W, b = layers[0]
    h = np.tanh(a @ W.T + b)
    hs.append(h)
    for W, b in layers[1:-1]:
        if bf16:
            z = round_bf16(h) @ round_bf16(W).T + b
        else:
            z = h @ W.T + b
        h = np.tanh(z)
        hs.append(h)
    W, b = layers[-1]
    y = h @ W.T + b
    return y, hs


def loss(theta, a, t, width=128, hidden=4, bf16=False) -> float:
    y, _ = forward(theta, a, width, hidden, bf16)
    return float(np.mean((y - t) ** 2))


def gradient(theta: np.ndarray, a: np.ndarray, t: np.ndarray, width: int = 128, hidden: int = 4,
             bf16: bool = False) -> Tuple[float, np.ndarray]:
    """Loss and its gradient with respect to the flat parameter vector (chain rule)."""
    layers = unpack(theta, width, hidden)
    y, hs = forward(theta, a, width, hidden, bf16)
    n = a.shape[0]
    E = float(np.mean((y - t) ** 2))
    grads = [None] * len(layers)
    dy = 2.0 * (y - t) / (N_OUT * n)                 # dE/dy
    W, _ = layers[-1]
    grads[-1] = (dy.T @ hs[-1], dy.sum(axis=0))
    dh = dy @ W                                      # dE/dh_{L-1}
    for l in range(len(layers) - 2, 0, -1):          # hidden-to-hidden layers, last to first
        dz = dh * (1.0 - hs[l] ** 2)                 # tanh' = 1 - tanh^2
        W, _ = layers[l]
        if bf16:
            gW = round_bf16(dz).T @ round_bf16(hs[l - 1])
            dh = round_bf16(dz) @ round_bf16(W)
        else:
            gW = dz.T @ hs[l - 1]
            dh = dz @ W
        grads[l] = (gW, dz.sum(axis=0))
    dz = dh * (1.0 - hs[0] ** 2)
    grads[0] = (dz.T @ a, dz.sum(axis=0))
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return E, g


def _gradient_perturbed(theta, a, t, width, hidden, rng, u):
    """``gradient`` with every operand that the bf16 path rounds multiplied instead by (1 + d),
    d uniform on [-u, u] and drawn independently per element: weights once per call (the
    kernels round one copy of each weight matrix for the forward and the backward product),
    activations and back-propagated values once per element (each is rounded once and the
    rounded value feeds both products that use it)."""
    layers = unpack(theta, width, hidden)

    def pert(x):
        return x * (1.0 + rng.uniform(-u, u, size=x.shape))

    Wp = [None] + [pert(W) for W, _ in layers[1:-1]] + [None]
    W, b = layers[0]
    h = np.tanh(a @ W.T + b)
    hs, hps = [h], []
    for l in range(1, len(layers) - 1):
        hp = pert(h)
        hps.append(hp)
        h = np.tanh(hp @ Wp[l].T + layers[l][1])
        hs.append(h)
    W, b = layers[-1]
    y = h @ W.T + b
    n = a.shape[0]
    E = float(np.mean((y - t) ** 2))
    grads = [None] * len(layers)
    dy = 2.0 * (y - t) / (N_OUT * n)
    grads[-1] = (dy.T @ hs[-1], dy.sum(axis=0))
    dh = dy @ W
    for l in range(len(layers) - 2, 0, -1):
        dz = dh * (1.0 - hs[l] ** 2)
        dzp = pert(dz)
        grads[l] = (dzp.T @ hps[l - 1], dz.sum(axis=0))
        dh = dzp @ Wp[l]
    dz = dh * (1.0 - hs[0] ** 2)
    grads[0] = (dz.T @ a, dz.sum(axis=0))
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return E, g


def rounding_spread(theta: np.ndarray, a: np.ndarray, t: np.ndarray, width: int = 128, hidden: int = 4,
                    runs: int = 8, seed: int = 0, u: float = 2.0 ** -8) -> Tuple[float, np.ndarray]:
    """How far bfloat16 operands in the hidden-to-hidden products can move the loss and every
    gradient element from the exact values: a standard deviation per element, estimated by
    Monte Carlo arithmetic (Parker 1997) — the evaluation repeated with each rounded operand
    perturbed by a random relative error of the rounding's size (uniform on [-u, u], u = 2^-8
    for 8 significant bits, which overstates round-to-nearest by ~1.4x in standard deviation).
    Unlike a variance propagated through the layers, this keeps the correlation of the errors
    that one rounded weight matrix puts on every sample; unlike a worst-case bound (|W| for W),
    it is not three to four orders of magnitude above the actual error.
    Returns (sigma of E, sigma of g per element)."""
    E0, g0 = gradient(theta, a, t, width, hidden)
    rng = np.random.default_rng(seed)
    dE, dg = [], []
    for _ in range(runs):
        E, g = _gradient_perturbed(theta, a, t, width, hidden, rng, u)
        dE.append(E - E0)
        dg.append(g - g0)
    return float(np.sqrt(np.mean(np.square(dE)))), np.sqrt(np.mean(np.square(dg), axis=0))


def adam_step(theta, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
