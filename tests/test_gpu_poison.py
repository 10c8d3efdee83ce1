"""Every device buffer the library is given starts filled with 0xFF bytes (NaN as float and
double): a read of memory the library never wrote -- an unused slot, padding, the other
population buffer before its first write, a stale partial sum -- would put a NaN into the
results.  Checked for single problems (every precision, a ragged grid and a Couette column),
a mixed-precision batch with retiring members, and the network."""
import numpy as np
import pytest

import workloads as W
from oracle.scheme import Problem as OP
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_0692_amd as F
    return F


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32", 2e-6), ("mixed", 2e-6)])
@pytest.mark.parametrize("case", [W.cavity(37, ny=29, kn=0.3, order=3), W.couette(50, kn=0.2)],
                         ids=["cavity37x29", "couette50"])
def test_poisoned_buffers_single_problem(F, case, prec, bar):
    op = OP.from_case(case)
    rho, ux, uy = W.random_fields(case.nx, case.ny, seed=8, amp=0.01)
    ref = op.step(op.equilibrium(rho, ux, uy), 23)
    gp = F.Problem(case, precision=prec, poison=True)
    gp.init_equilibrium(rho, ux, uy)
    gp.step(23)
    f = gp.download()
    assert np.all(np.isfinite(f))
    dev = np.abs(ref - op.w[:, None, None]).max()
    assert np.abs(f - ref).max() <= bar * dev
    r, u, v, pxy = gp.moments()
    assert np.all(np.isfinite(r)) and np.all(np.isfinite(pxy))
    # plain float levels off above 1e-8 (the float phase of the mixed path does not)
    rep = gp.solve(1e-6 if prec == "fp32" else 1e-9, 200000, check_every=50)
    assert rep["status"] == 0 and np.isfinite(rep["residual"])


def test_poisoned_buffers_batch(F):
    cases = [W.cavity(40, kn=0.3, order=2), W.cavity(24, ny=56, kn=3.0, order=3), W.cavity(64, kn=0.05, order=2)]
    b = F.Batch(cases, precision="mixed", poison=True)
    b.set_retile(1)
    for i in range(len(cases)):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-9, 200000, check_every=100)
    assert status == 0
    for i, case in enumerate(cases):
        rho, ux, uy, pxy = b.moments(i)
        assert np.all(np.isfinite(rho)) and np.all(np.isfinite(ux)) and np.all(np.isfinite(pxy))


def test_poisoned_buffers_network(F):
    import torch
    theta = np.asarray(W.mlp_params(91), dtype=np.float32).astype(np.float64)
    a, t = W.mlp_samples(333, 92)
    a, t = a.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    net = F.Mlp(params=theta, max_batch=512, poison=True)
    A = torch.as_tensor(a, dtype=torch.float32).cuda()
    T = torch.as_tensor(t, dtype=torch.float32).cuda()
    net.backward(A, T)
    g = net.grad.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(g))
    _, gb = mlp.gradient(theta, a, t, bf16=True)
    assert np.linalg.norm(g - gb) <= 2e-4 * np.linalg.norm(gb)
    y = net.forward(A).cpu().numpy()
    assert np.all(np.isfinite(y))
