"""Edge cases of the HIP path against the oracle: the largest velocity set (16 nodes per half on
both axes, Q = 1024) and the smallest ones (Q = 16 and 8, on every tile shape), a relaxation
rate at its limit (omega = 1), empty calls, and a problem
with no moving wall, which must stay at rest to round-off (the wall constant sqrt(2 pi) A - 1 of
Eq. (9) is zero only in exact arithmetic)."""
import re

import numpy as np
import pytest

import workloads as W
from oracle.scheme import Problem as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_0692_amd as F
    return F


def perturbed(xi_x, xi_y, w, nx, ny, seed):
    rho, ux, uy = W.random_fields(nx, ny, seed, amp=0.01)
    noise = W.random_noise(len(w), nx, ny, seed + 1)
    feq = w[:, None, None] * rho[None] * (1 + xi_x[:, None, None] * ux[None] + xi_y[:, None, None] * uy[None])
    return feq * (1 + 0.02 * noise)


def compare(F, case, prec, steps, bar):
    op = OP.from_case(case)
    gp = F.Problem(case, precision=prec)
    x, y, w = gp.velocities()
    gp.upload(perturbed(x, y, w, case.nx, case.ny, 5))
    gp.step(steps)
    ref = op.step(perturbed(op.xi_x, op.xi_y, op.w, case.nx, case.ny, 5), steps)
    dev = np.abs(ref - op.w[:, None, None]).max()
    assert np.abs(gp.download() - ref).max() <= bar * dev


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_largest_velocity_set(F, prec, bar):
    case = W.cavity(6, ny=5, kn=0.5, order=16)
    assert F.Problem(case, bind=False).q == 1024
    compare(F, case, prec, 5, bar)


@pytest.mark.parametrize("case", [W.cavity(12, ny=10, kn=0.3, order=2),
                                  W.couette(21, kn=0.5, qx=("full", 2), qy=("half", 2))],
                         ids=["cavity_q16", "couette_q8"])
@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_smallest_velocity_sets_every_tile(F, case, prec, bar):
    """The smallest valid velocity sets (two nodes per rule): Q = 16 in the cavity and Q = 8 in
    the channel, two velocities per quadrant, so shapes that split the velocities eight ways
    leave each wave one velocity; every shape that fits must match the oracle."""
    op = OP.from_case(case)
    ref = op.step(perturbed(op.xi_x, op.xi_y, op.w, case.nx, case.ny, 7), 25)
    dev = np.abs(ref - op.w[:, None, None]).max()
    gp = F.Problem(case, precision=prec)
    assert gp.q == op.q
    x, y, w = gp.velocities()
    f0 = perturbed(x, y, w, case.nx, case.ny, 7)
    tiles = []
    for t in range(F.tile_count(prec)):
        try:
            gp.set_tile(t)
        except F.FdlbError:
            continue
        tiles.append(t)
        gp.upload(f0)
        gp.step(25)
        assert np.abs(gp.download() - ref).max() <= bar * dev, (t, F.tile_describe(prec, t))
    assert len(tiles) >= 4


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_relaxation_rate_at_its_limit(F, prec, bar):
    base = W.cavity(24, ny=20, order=2)
    dt = F.Problem(base, bind=False).dt
    case = W.with_(base, kn=dt)          # omega = dt / Kn = 1: full relaxation every step
    p = F.Problem(case, bind=False)
    assert p.omega == 1.0
    compare(F, case, prec, 10, bar)


def test_empty_calls(F):
    case = W.cavity(16, order=2)
    p = F.Problem(case, precision="fp64")
    p.init_equilibrium(*W.random_fields(16, 16, 3, amp=0.01))
    f0 = p.download()
    p.step(0)
    assert np.array_equal(p.download(), f0)
    rep = p.solve(1e-8, 0, check_every=10)
    assert rep["steps"] == 0 and rep["status"] == 1
    assert np.array_equal(p.download(), f0)
    import torch
    net = F.Mlp(max_batch=64)
    y = net.forward(torch.empty((0, 3), dtype=torch.float32, device="cuda"))
    assert y.shape == (0, 3)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_no_moving_wall_stays_at_rest(F, prec):
    case = W.cavity(20, ny=12, kn=0.3, u_w=0.0, order=3)
    p = F.Problem(case, precision=prec)
    p.init_equilibrium()
    p.step(50)
    x, y, w = p.velocities()
    assert np.abs(p.download() - w[:, None, None]).max() <= 1e-13 * w.max()
    rho, ux, uy, pxy = p.moments()
    assert np.abs(rho - 1.0).max() <= 1e-13
    assert np.abs(ux).max() <= 1e-13 and np.abs(uy).max() <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_nan_in_the_state_is_reported_as_divergence(F, prec):
    """A NaN in one population of one cell: the residual of the first step is NaN, which
    the device-side check counts as a runaway, so the solve stops with EDIVERGED at step 1
    instead of returning NaN fields as converged (NaN arithmetic does not fault)."""
    case = W.cavity(33, ny=21, kn=0.2, order=2)
    p = F.Problem(case, precision=prec)
    p.init_equilibrium()
    f = p.download()
    f[3, 10, 17] = np.nan
    p.upload(f)
    rep = p.solve(1e-8, 1000, check_every=25, raise_on_diverge=False)
    assert rep["status"] == F._lib.EDIVERGED
    with pytest.raises(F.FdlbError) as e:
        p.upload(f)
        p.solve(1e-8, 1000, check_every=25)
    assert e.value.code == F._lib.EDIVERGED
    assert re.search(r"diverged at step 1\b", str(e.value)), str(e.value)
    # the problem stays usable: a fresh start converges
    p.init_equilibrium()
    assert p.solve(1e-6, 100000, check_every=50)["status"] == 0


def test_renormalising_a_non_positive_mass(F):
    """The host seed refuses a density field whose sum is not positive; the device seed cannot
    refuse (it is asynchronous), so it leaves a NaN state that the next solve reports as
    divergence at step 1; a valid seed afterwards works."""
    import torch
    case = W.cavity(16, ny=12, kn=0.3, order=2)
    p = F.Problem(case, precision="fp32")
    rho = -np.ones((12, 16))
    with pytest.raises(F.FdlbError) as e:
        p.init_equilibrium(rho, None, None, renormalize=True)
    assert e.value.code == F._lib.EINVAL
    z = torch.zeros((12, 16), dtype=torch.float32, device="cuda")
    for r in (z, z - 1.0):
        p.init_equilibrium_dev(r, z, z, renormalize=True)
        rep = p.solve(1e-8, 1000, check_every=10, raise_on_diverge=False)
        assert rep["status"] == F._lib.EDIVERGED and rep["steps"] == 1
    p.init_equilibrium_dev(z + 1.0, z, z, renormalize=True)
    assert p.solve(1e-6, 100000, check_every=50)["status"] == 0


def test_nan_in_one_batch_member_leaves_the_others(F):
    cases = [W.cavity(32, kn=0.3, order=2), W.cavity(40, kn=0.3, order=2), W.cavity(24, kn=1.0, order=2)]
    b = F.Batch(cases, precision="fp32")
    for i in range(3):
        b.init_equilibrium(i)
    f = b.download(1)
    f[0, 0, 0] = np.nan
    b.upload(1, f)
    status, reps = b.solve(1e-6, 50000, check_every=40)
    assert status == F._lib.EDIVERGED
    assert reps[1]["status"] == F._lib.EDIVERGED
    assert reps[0]["status"] == 0 and reps[2]["status"] == 0
    for i in (0, 2):
        rho, ux, uy, _ = b.moments(i)
        assert np.all(np.isfinite(rho)) and np.all(np.isfinite(ux))
