"""Warm-start network kernels (through the C ABI) against the FP64 oracle of oracle/mlp.py.

Bars, from the arithmetic (bf16 operands with 8 significant bits in the 128 x 128 products,
fp32 elsewhere; a float32 emulation of these kernels lands within 1.5e-3 (max) / 1.3e-4
(rms) of the bf16-emulating oracle on outputs and 1.3e-5 on gradients, and the bf16
rounding itself moves outputs by <= 7e-3 and gradients by <= 2.4e-3 from plain FP64):
  outputs   vs bf16-emulating oracle: rms <= 1e-3 rms(y), max <= 1e-2 max|y|
            vs plain FP64 oracle:     max <= 3e-2 max|y|
  gradient  vs bf16-emulating oracle: ||g - g_ref|| <= 2e-4 ||g_ref||; loss within 1e-4
            vs plain FP64 oracle:     ||g - g_ref|| <= 1e-2 ||g_ref||, and per element
                                      |g - g_ref| <= 6 sigma + 1e-5 (|g_ref| + max|g_ref|),
                                      sigma the oracle's Monte Carlo spread of the bf16
                                      rounding error on that element (loss: 6 sigma_E)
  Adam      fp32 update vs FP64 oracle: <= 1e-6 relative (three steps)
Sizes are ragged (not multiples of the 64-sample tile)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_0692_amd as F
    return F


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype or np.float32)).cuda()


@pytest.mark.parametrize("n,seed", [(1000, 21), (64, 5), (1, 9)])
def test_forward_matches_oracle(F, n, seed):
    import torch
    theta = f32(W.mlp_params(seed))
    a, _ = W.mlp_samples(n, seed + 1)
    a = f32(a)
    net = F.Mlp(params=theta, max_batch=64)
    y = net.forward(dev(torch, a)).cpu().numpy().astype(np.float64)
    yb, _ = mlp.forward(theta, a, bf16=True)
    y64, _ = mlp.forward(theta, a)
    scale = np.abs(yb).max()
    assert np.sqrt(np.mean((y - yb) ** 2)) <= 1e-3 * np.sqrt(np.mean(yb ** 2))
    assert np.abs(y - yb).max() <= 1e-2 * scale
    assert np.abs(y - y64).max() <= 3e-2 * np.abs(y64).max()


@pytest.mark.parametrize("n,hidden", [(777, 4), (130, 2), (64, 1), (65, 4), (1, 3), (97, 5), (300, 8)])
def test_gradient_matches_oracle(F, n, hidden):
    import torch
    theta = f32(W.mlp_params(3 + n, 128, hidden))
    a, t = W.mlp_samples(n, 13 + n)
    a, t = f32(a), f32(t)
    net = F.Mlp(hidden=hidden, params=theta, max_batch=1024)
    net.backward(dev(torch, a), dev(torch, t))
    g = net.grad.cpu().numpy().astype(np.float64)
    E = net.last_loss()
    Eb, gb = mlp.gradient(theta, a, t, 128, hidden, bf16=True)
    E64, g64 = mlp.gradient(theta, a, t, 128, hidden)
    assert np.linalg.norm(g - gb) <= 2e-4 * np.linalg.norm(gb), np.linalg.norm(g - gb) / np.linalg.norm(gb)
    assert abs(E - Eb) <= 1e-4 * Eb
    assert np.linalg.norm(g - g64) <= 1e-2 * np.linalg.norm(g64)
    # element by element against plain FP64: within 6 standard deviations of the error that
    # bf16 operands in the hidden products put on that element (Monte Carlo spread of the
    # oracle), plus float32 rounding elsewhere; the loss likewise
    sE, sg = mlp.rounding_spread(theta, a, t, 128, hidden, runs=32)
    m = np.abs(g64).max()
    bar = 6 * sg + 1e-5 * (np.abs(g64) + m)
    worst = np.argmax(np.abs(g - g64) - bar)
    assert np.all(np.abs(g - g64) <= bar), (worst, g[worst], g64[worst], sg[worst])
    assert abs(E - E64) <= 6 * sE + 1e-6 * E64, (E, E64, sE)
    # every block of the parameter vector carries gradient (no layer left out)
    k = 0
    for o, i in mlp.layer_shapes(128, hidden):
        for size in (o * i, o):
            part, ref = g[k:k + size], gb[k:k + size]
            assert np.linalg.norm(part - ref) <= 1e-3 * np.linalg.norm(ref) + 1e-12, (o, i, size)
            k += size


def test_row_selection_equals_gathered_arrays(F):
    import torch
    theta = f32(W.mlp_params(40))
    a, t = W.mlp_samples(300, 41)
    rows = np.random.default_rng(42).permutation(300)[:200].astype(np.int32)
    net = F.Mlp(params=theta, max_batch=256)
    net.backward(dev(torch, a), dev(torch, t), rows=dev(torch, rows, np.int32))
    g1 = net.grad.clone()
    E1 = net.last_loss()
    net.backward(dev(torch, a[rows]), dev(torch, t[rows]))
    assert torch.equal(g1, net.grad)
    assert E1 == net.last_loss()


def test_adam_matches_oracle(F):
    import torch
    P = mlp.param_count()
    theta = f32(W.mlp_params(50))
    rng = np.random.default_rng(51)
    grads = [f32(rng.standard_normal(P) * 10.0 ** rng.uniform(-4, 0, P)) for _ in range(3)]
    net = F.Mlp(params=theta)
    m = np.zeros(P)
    v = np.zeros(P)
    th = theta.copy()
    for s, g in enumerate(grads, start=1):
        net.grad.copy_(dev(torch, g))
        net.adam_step(1e-3)
        th, m, v = mlp.adam_step(th, g, m, v, s, 1e-3)
    got = net.params.cpu().numpy().astype(np.float64)
    assert np.abs(got - th).max() <= 1e-6 * max(1.0, np.abs(th).max())
    # the first moment is a signed running mean: bound its fp32 error by the gradients' size
    gmax = np.max(np.abs(np.stack(grads)), axis=0)
    assert np.all(np.abs(net.adam_m.cpu().numpy() - m) <= 1e-6 * gmax)


def test_training_lowers_the_loss(F):
    import torch
    a, t = W.mlp_samples(2000, 61)
    net = F.Mlp(seed=7, max_batch=512)
    A, T = dev(torch, a), dev(torch, t)
    net.backward(A[:512], T[:512])
    E0 = net.last_loss()
    for s in range(300):
        k = (s * 512) % 1536
        net.backward(A[k:k + 512], T[k:k + 512])
        net.adam_step(3e-3)
    net.backward(A[:512], T[:512])
    assert net.last_loss() < 0.05 * E0, (E0, net.last_loss())


def test_predict_fields_equals_forward_on_cell_inputs(F):
    import torch
    theta = f32(W.mlp_params(70))
    net = F.Mlp(params=theta)
    kn, nx, ny, uw = 0.37, 37, 29, 0.01
    rho, ux, uy = [x.cpu().numpy() for x in net.predict_fields(kn, nx, ny, uw)]
    xs = (2.0 * (np.arange(nx) + 0.5) / nx - 1.0).astype(np.float32)
    ys = (2.0 * (np.arange(ny) + 0.5) / ny - 1.0).astype(np.float32)
    feats = np.stack([np.full(nx * ny, np.float32((math.log10(kn) + 0.5) / 1.5)),
                      np.tile(xs, ny), np.repeat(ys, nx)], axis=1).astype(np.float32)
    y = net.forward(dev(torch, feats)).cpu().numpy()
    assert np.abs(rho.ravel() - (1 + uw * y[:, 0])).max() <= 1e-6
    assert np.abs(ux.ravel() - uw * y[:, 1]).max() <= 1e-9
    assert np.abs(uy.ravel() - uw * y[:, 2]).max() <= 1e-9


def test_field_samples_of_a_solved_cavity(F):
    case = W.cavity(24, ny=20, kn=0.3, u_w=0.02, order=2)
    p = F.Problem(case, precision="fp64")
    p.init_equilibrium()
    p.solve(1e-9, 100000, check_every=100)
    a, t = [x.cpu().numpy().astype(np.float64) for x in p.field_samples()]
    rho, ux, uy, _ = p.moments()
    assert np.allclose(t[:, 0], (rho.ravel() - 1) / 0.02, rtol=1e-6, atol=1e-7)
    assert np.allclose(t[:, 1], ux.ravel() / 0.02, rtol=1e-6, atol=1e-9)
    assert np.allclose(t[:, 2], uy.ravel() / 0.02, rtol=1e-6, atol=1e-9)
    assert np.allclose(a[:, 0], (math.log10(0.3) + 0.5) / 1.5, rtol=1e-6)
    assert np.allclose(a[:, 1], np.tile(2 * (np.arange(24) + 0.5) / 24 - 1, 20), atol=1e-7)
    assert np.allclose(a[:, 2], np.repeat(2 * (np.arange(20) + 0.5) / 20 - 1, 24), atol=1e-7)


def test_gradient_full_training_batch(F):
    """A full training batch (8,192 samples, the size the warm-start training uses)."""
    import torch
    theta = f32(W.mlp_params(81))
    a, t = W.mlp_samples(8192, 82)
    a, t = f32(a), f32(t)
    net = F.Mlp(params=theta, max_batch=8192)
    net.backward(dev(torch, a), dev(torch, t))
    g = net.grad.cpu().numpy().astype(np.float64)
    Eb, gb = mlp.gradient(theta, a, t, bf16=True)
    assert np.linalg.norm(g - gb) <= 2e-4 * np.linalg.norm(gb)
    assert abs(net.last_loss() - Eb) <= 1e-4 * Eb


def test_train_steps_equals_the_step_by_step_loop(F):
    """fdlb_mlp_train enqueues the same kernels in the same order as backward + adam_step per
    minibatch: parameters, Adam moments and loss agree to the bit (ragged last minibatch)."""
    import torch
    theta = f32(W.mlp_params(90))
    a, t = W.mlp_samples(1000, 91)
    A, T = dev(torch, a), dev(torch, t)
    rows = dev(torch, np.random.default_rng(92).permutation(1000).astype(np.int32), np.int32)
    lrs = [3e-3, 2e-3, 1e-3, 5e-4]           # 4 steps of 300: 300, 300, 300, 100 rows
    n1 = F.Mlp(params=theta, max_batch=512)
    n2 = F.Mlp(params=theta, max_batch=512)
    n1.train_steps(A, T, rows, 300, lrs)
    for s, lr in enumerate(lrs):
        n2.backward(A, T, rows=rows[s * 300:(s + 1) * 300])
        n2.adam_step(lr)
    assert n1.step_count == n2.step_count == 4
    assert torch.equal(n1.params, n2.params)
    assert torch.equal(n1.adam_m, n2.adam_m) and torch.equal(n1.adam_v, n2.adam_v)
    assert n1.last_loss() == n2.last_loss()
    with pytest.raises(F.FdlbError):
        n1.train_steps(A, T, rows, 300, lrs + [1e-4])   # a fifth step would start past the rows


def test_train_and_predict_reject_bad_arguments(F):
    """The minibatch schedule must give every step a row (checked without overflow, before any
    learning rate is read), and the predicted fields need a finite wall speed."""
    import ctypes as C
    import torch
    from paper_1308_0692_amd import _lib
    net = F.Mlp(max_batch=64)
    a, t = W.mlp_samples(17, 3)
    x, y = dev(torch, f32(a)), dev(torch, f32(t))
    rows = torch.arange(17, dtype=torch.int32, device="cuda")
    lr = np.full(4, 1e-3)

    def train(n_rows, batch, steps):
        return _lib.lib.fdlb_mlp_train(net._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                       C.c_void_p(rows.data_ptr()), n_rows, batch, steps, _lib._dp(lr),
                                       0.9, 0.999, 1e-8, 1)

    assert train(17, 8, 3) == 0          # rows 0-7, 8-15, 16
    assert train(16, 8, 3) == _lib.EINVAL  # the third step would start at row 16
    assert train(0, 8, 1) == _lib.EINVAL
    assert train(17, 8, 2 ** 62) == _lib.EINVAL  # (steps - 1) * batch would overflow
    torch.cuda.synchronize()
    for u_w in (float("nan"), float("inf")):
        with pytest.raises(F.FdlbError):
            net.predict_fields(0.1, 8, 8, u_w)


def test_poisoned_workspace_gives_the_same_training(F):
    """Workspace filled with NaN bytes before binding: a read of memory the kernels did not
    write first (activation and gradient transposes past the samples, partials of blocks or
    slices that do not exist) would show up as NaN; gradient, loss and three training steps
    equal those of a clean workspace to the bit (ragged batch, two hidden-layer counts)."""
    import torch
    for hidden, n in ((4, 777), (2, 33)):
        theta = f32(W.mlp_params(100 + hidden, 128, hidden))
        a, t = W.mlp_samples(n, 101)
        A, T = dev(torch, f32(a)), dev(torch, f32(t))
        rows = dev(torch, np.random.default_rng(102).permutation(n).astype(np.int32), np.int32)
        out = []
        for poison in (False, True):
            net = F.Mlp(hidden=hidden, params=theta, max_batch=1024, poison=poison)
            net.backward(A, T)
            g = net.grad.clone()
            E = net.last_loss()
            net.train_steps(A, T, rows, n // 3, [3e-3, 2e-3, 1e-3])
            out.append((g, E, net.params.clone(), net.last_loss()))
            net.close()
        (g0, E0, p0, L0), (g1, E1, p1, L1) = out
        assert torch.isfinite(g1).all() and torch.equal(g0, g1) and E0 == E1
        assert torch.equal(p0, p1) and L0 == L1
