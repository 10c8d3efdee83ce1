"""Pins of the FP64 warm-start network oracle (oracle/mlp.py) against facts fixed by the
mathematics: finite differences, closed-form forward passes, the output-bias gradient,
Adam's first step, bfloat16 rounding of values whose rounding is known, and the spread of the
rounding error against the error of exact bfloat16 rounding."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp


def test_param_count_matches_architecture():
    # 3*128+128 + 3*(128*128+128) + 128*3+3
    assert mlp.param_count() == 50435
    assert mlp.param_count(8, 2) == (8 * 3 + 8) + (8 * 8 + 8) + (3 * 8 + 3)


@pytest.mark.parametrize("width,hidden", [(6, 4), (5, 2)])
def test_gradient_matches_central_differences(width, hidden):
    theta = W.mlp_params(3, width, hidden)
    a, t = W.mlp_samples(7, 4)
    E, g = mlp.gradient(theta, a, t, width, hidden)
    assert E == pytest.approx(mlp.loss(theta, a, t, width, hidden), rel=1e-15)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (mlp.loss(tp, a, t, width, hidden) - mlp.loss(tm, a, t, width, hidden)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-8 * max(1.0, np.abs(fd).max())


def test_full_width_directional_derivatives():
    """Width 128, four hidden layers: the gradient's projection on random directions equals
    the central difference of the loss along them."""
    theta = W.mlp_params(11)
    a, t = W.mlp_samples(16, 12)
    _, g = mlp.gradient(theta, a, t)
    rng = np.random.default_rng(5)
    for _ in range(4):
        d = rng.standard_normal(theta.size)
        d /= np.linalg.norm(d)
        h = 1e-5
        fd = (mlp.loss(theta + h * d, a, t) - mlp.loss(theta - h * d, a, t)) / (2 * h)
        assert abs(g @ d - fd) <= 1e-7 * max(1e-3, abs(fd))


def test_forward_closed_forms():
    width, hidden = 128, 4
    theta = W.mlp_params(2)
    layers = mlp.unpack(theta, width, hidden)
    a, _ = W.mlp_samples(5, 1)
    # zero weights everywhere: hidden activations are tanh of the biases, output is W_L tanh(b) + b_L
    z = theta.copy()
    for Wm, _ in mlp.unpack(z, width, hidden):
        Wm[...] = 0.0
    Wl, bl = mlp.unpack(z, width, hidden)[-1]
    y, hs = mlp.forward(z, a, width, hidden)
    assert np.array_equal(y, np.broadcast_to(bl, y.shape))
    z2 = theta.copy()
    for Wm, _ in mlp.unpack(z2, width, hidden)[:-1]:
        Wm[...] = 0.0
    Wl2, bl2 = mlp.unpack(z2, width, hidden)[-1]
    b3 = mlp.unpack(z2, width, hidden)[-2][1]
    y2, _ = mlp.forward(z2, a, width, hidden)
    assert np.allclose(y2, np.tanh(b3) @ Wl2.T + bl2, rtol=0, atol=1e-15)
    # one path: x_0 -> unit 0 of every layer (weight 1), biases zero, output 0 reads unit 0
    z3 = np.zeros_like(theta)
    L = mlp.unpack(z3, width, hidden)
    L[0][0][0, 0] = 1.0
    for l in range(1, hidden):
        L[l][0][0, 0] = 1.0
    L[-1][0][0, 0] = 1.0
    y3, _ = mlp.forward(z3, a, width, hidden)
    expect = a[:, 0].copy()
    for _ in range(hidden):
        expect = np.tanh(expect)
    assert np.allclose(y3[:, 0], expect, rtol=0, atol=1e-15)
    assert np.array_equal(y3[:, 1:], np.zeros((a.shape[0], 2)))


def test_output_bias_gradient_is_mean_residual():
    theta = W.mlp_params(7)
    a, t = W.mlp_samples(33, 8)
    y, _ = mlp.forward(theta, a)
    _, g = mlp.gradient(theta, a, t)
    gb = g[-3:]
    assert np.allclose(gb, 2.0 * (y - t).sum(axis=0) / (3 * a.shape[0]), rtol=1e-13, atol=0)


def test_adam_first_step_and_zero_gradient():
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    t1, m1, v1 = mlp.adam_step(theta, g, m, v, 1, lr, eps=eps)
    # bias correction makes the first moments g and g^2: the step is lr g / (|g| + eps)
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-17)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    t2, m2, v2 = mlp.adam_step(theta, np.zeros(50), m, v, 1, lr)
    assert np.array_equal(t2, theta)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -2.5, 0.0, 3.0e38,
                     1.0 + 2.0 ** -8 + 2.0 ** -20])
    r = mlp.round_bf16(vals)
    # bf16 keeps 7 fraction bits: ulp(1) = 2^-7
    assert r[0] == 1.0
    assert r[1] == 1.0                          # tie -> even (1.0)
    assert r[2] == 1.0 + 2 * 2.0 ** -7          # tie -> even (1 + 2 ulp)
    assert r[3] == 1.0
    assert r[4] == -2.5
    assert r[5] == 0.0
    assert r[7] == 1.0 + 2.0 ** -7              # above the tie: rounds up
    assert np.isfinite(r[6])
    x = np.random.default_rng(1).standard_normal(1000)
    rx = mlp.round_bf16(x)
    # half an ulp: at most 2^-8 relative (ulp = 2^-7 relative at the bottom of a binade)
    assert np.all(np.abs(rx - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))
    assert np.abs(rx - x).max() > 2.0 ** -10 * np.abs(x).max()   # and not finer than bf16


def test_bf16_products_stay_close_to_fp64():
    """The bfloat16 operand rounding changes outputs and gradients by a small relative amount
    (the bound the GPU comparison against the plain FP64 oracle uses)."""
    theta = W.mlp_params(21)
    a, t = W.mlp_samples(256, 22)
    y, _ = mlp.forward(theta, a)
    yb, _ = mlp.forward(theta, a, bf16=True)
    assert np.abs(yb - y).max() <= 2e-2 * np.abs(y).max()
    _, g = mlp.gradient(theta, a, t)
    _, gb = mlp.gradient(theta, a, t, bf16=True)
    assert np.linalg.norm(gb - g) <= 3e-2 * np.linalg.norm(g)


@pytest.mark.parametrize("n,hidden", [(777, 4), (130, 2), (65, 4), (1, 3), (3000, 4)])
def test_rounding_spread_predicts_the_bf16_error(n, hidden):
    """The Monte Carlo spread of the gradient under random operand errors of the bf16 rounding's
    size predicts the actual error of exact bfloat16 rounding at those points, element by
    element: every element within 6 sigma of plain FP64, and the normalised errors neither far
    below 1 (a spread that would hide real faults) nor above it (one that would be too tight)."""
    f32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)  # noqa: E731
    theta = f32(W.mlp_params(3 + n, 128, hidden))
    a, t = W.mlp_samples(n, 13 + n)
    a, t = f32(a), f32(t)
    Eb, gb = mlp.gradient(theta, a, t, 128, hidden, bf16=True)
    E64, g64 = mlp.gradient(theta, a, t, 128, hidden)
    sE, sg = mlp.rounding_spread(theta, a, t, 128, hidden, runs=32)
    assert np.all(np.abs(gb - g64) <= 6 * sg)
    assert abs(Eb - E64) <= 6 * sE
    z = (gb - g64)[sg > 0] / sg[sg > 0]
    assert 0.4 <= np.sqrt(np.mean(z * z)) <= 1.2
    # the spread is linear in the rounding size and vanishes without rounding
    _, sg2 = mlp.rounding_spread(theta, a, t, 128, hidden, runs=32, u=2.0 ** -9)
    assert 0.4 <= np.median(sg2[sg > 0] / sg[sg > 0]) <= 0.6
    assert np.all(mlp.rounding_spread(theta, a, t, 128, hidden, runs=2, u=0.0)[1] == 0)


def test_rounding_spread_is_zero_without_hidden_products():
    """One hidden layer has no 128 x 128 product, so nothing is rounded to bf16."""
    theta = W.mlp_params(5, 128, 1)
    a, t = W.mlp_samples(50, 6)
    sE, sg = mlp.rounding_spread(theta, a, t, 128, 1, runs=4)
    assert sE == 0 and np.all(sg == 0)


def test_training_lowers_the_loss():
    width, hidden = 16, 2
    theta = W.mlp_params(31, width, hidden)
    a, t = W.mlp_samples(64, 32)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    E0 = mlp.loss(theta, a, t, width, hidden)
    for s in range(1, 301):
        _, g = mlp.gradient(theta, a, t, width, hidden)
        theta, m, v = mlp.adam_step(theta, g, m, v, s, 1e-2)
    assert mlp.loss(theta, a, t, width, hidden) < 0.2 * E0
