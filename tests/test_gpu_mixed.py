"""Mixed precision (FDLB_MIXED): float deviations until a steady solve nears its
tolerance, then the state widened to double in place and the double kernels finish.

Checks: the float phase is bit-identical to the FP32 path; after the switch the state
marches exactly as the FP64 oracle does from the widened state (<= 1e-12 relative);
a cavity whose float residual cycles above 1e-8 reaches 1e-8 in mixed precision and
matches the oracle's converged solution to the FP32 bar (2e-5); checkpoints keep the
precision; batch members switch individually and equal their solo runs bit for bit."""
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


def eps_u(ux, uy, uxr, uyr):
    return float(np.hypot(ux - uxr, uy - uyr).max() / np.hypot(uxr, uyr).max())


def test_float_phase_equals_fp32_path(F):
    case = W.cavity(40, ny=36, kn=0.2, order=3)
    m = F.Problem(case, precision="mixed")
    s = F.Problem(case, precision="fp32")
    for p in (m, s):
        p.init_equilibrium()
        p.step(123)
    assert m.active_precision == "fp32"
    assert m.state_bytes == F.Problem(case, precision="fp64", bind=False).state_bytes
    assert np.array_equal(m.download(), s.download())
    assert m.last_residual() == s.last_residual()


def test_switch_then_double_matches_oracle(F):
    case = W.cavity(40, ny=36, kn=0.2, order=3)
    gp = F.Problem(case, precision="mixed")
    gp.init_equilibrium()
    gp.step(150)
    f0 = gp.download()
    gp.promote()
    assert gp.active_precision == "fp64"
    assert np.array_equal(gp.download(), f0)   # widening is exact
    gp.step(100)
    op = OP.from_case(case)
    fo = op.step(f0, 100)
    dev = np.abs(fo - op.w[:, None, None]).max()
    assert np.abs(gp.download() - fo).max() <= 1e-12 * dev
    _, steps = gp.last_residual()
    assert steps == 250
    gp.promote()   # already double: no-op
    assert gp.active_precision == "fp64"
    with pytest.raises(F.FdlbError):
        s = F.Problem(case, precision="fp32")
        s.init_equilibrium()
        s.promote()


def test_mixed_reaches_tolerance_where_float_cycles(F):
    """A 64^2 cavity (8 x 8 velocities, Kn 0.1477) whose float residual settles into a
    rounding cycle near 1.1e-8: the mixed solve switches to double and reaches 1e-8."""
    case = W.cavity(64, kn=0.1477, order=4)
    gp = F.Problem(case, precision="mixed")
    gp.init_equilibrium()
    rep = gp.solve(1e-8, 200000, check_every=200)
    assert rep["status"] == 0, rep["residual"]
    assert gp.active_precision == "fp64"
    assert 0 < rep["steps_fp32"] < rep["steps"]
    assert rep["steps_fp32"] >= 0.5 * rep["steps"], (rep["steps_fp32"], rep["steps"])
    op = OP.from_case(case)
    fo, steps, hist = op.solve(op.equilibrium(), 1e-10, 400000)
    assert hist[-1] < 1e-10
    rho, ux, uy, _ = gp.moments()
    r0, ux0, uy0 = op.moments(fo)
    eu = eps_u(ux, uy, ux0, uy0)
    er = float(np.abs(rho - r0).max())
    print(f"mixed 64^2 Kn 0.1477: {rep['steps']} steps ({rep['steps_fp32']} float), eps_u {eu:.2e}, eps_rho {er:.2e}")
    assert eu <= 2e-5, eu
    assert er <= 2e-5, er


def test_tolerance_above_switch_level_stays_float(F):
    case = W.cavity(32, kn=0.1, order=2)
    gp = F.Problem(case, precision="mixed")
    gp.init_equilibrium()
    rep = gp.solve(1e-6, 100000, check_every=100)
    assert rep["status"] == 0
    assert gp.active_precision == "fp32"
    assert rep["steps_fp32"] == rep["steps"]


def test_checkpoint_keeps_precision(F):
    case = W.cavity(32, ny=24, kn=0.5, order=2)
    a = F.Problem(case, precision="mixed")
    a.init_equilibrium()
    a.step(40)
    a.promote()
    a.step(11)
    ck = a.checkpoint()
    b = F.Problem(case, precision="mixed")
    b.init_equilibrium()
    assert b.active_precision == "fp32"
    b.restore(ck)
    assert b.active_precision == "fp64"
    a.step(20)
    b.step(20)
    assert np.array_equal(a.download(), b.download())
    assert a.last_residual() == b.last_residual()
    b.init_equilibrium()   # a new state starts in float again
    assert b.active_precision == "fp32"


def test_batch_members_switch_individually_and_equal_solo(F):
    # One grid for all members, so that the batch's double-phase tile is the solo default too.
    cases = [W.cavity(48, kn=0.3, order=2), W.cavity(48, kn=2.0, order=3), W.cavity(48, kn=0.05, order=2),
             W.cavity(48, kn=8.0, order=2)]
    b = F.Batch(cases, precision="mixed")
    b.set_retile(0)  # one tile throughout: bit-identical to single solves with that tile
    for i in range(len(cases)):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-9, 200000, check_every=100)
    assert status == 0, [r["status"] for r in reps]
    for i, case in enumerate(cases):
        assert b.active_precision(i) == "fp64", i
        assert 0 < reps[i]["steps_fp32"] < reps[i]["steps"], i
        p = F.Problem(case, precision="mixed")
        p.set_tile(b.tile)
        p.init_equilibrium()
        rep = p.solve(1e-9, 200000, check_every=100)
        assert rep["steps"] == reps[i]["steps"] and rep["steps_fp32"] == reps[i]["steps_fp32"], i
        assert np.array_equal(p.download(), b.download(i, p.q)), i


def test_batch_mixed_matches_oracle(F):
    cases = [W.cavity(40, ny=32, kn=0.4, order=2), W.cavity(24, ny=56, kn=3.0, order=3)]
    b = F.Batch(cases, precision="mixed")
    for i in range(len(cases)):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-9, 200000, check_every=100)
    assert status == 0
    for i, case in enumerate(cases):
        op = OP.from_case(case)
        fo, steps, hist = op.solve(op.equilibrium(), 1e-11, 400000)
        rho, ux, uy, _ = b.moments(i)
        r0, ux0, uy0 = op.moments(fo)
        assert eps_u(ux, uy, ux0, uy0) <= 2e-5, i
        assert float(np.abs(rho - r0).max()) <= 2e-5, i


def test_batch_mixed_autotune_keeps_results(F):
    """Autotuning a mixed batch times both groups' shapes (the double group with every member
    promoted) and re-seeds the members; the solve afterwards still reaches the oracle's
    converged solution within the FP32 bar."""
    cases = [W.cavity(40, ny=32, kn=0.4, order=2), W.cavity(24, ny=56, kn=3.0, order=3),
             W.cavity(32, kn=0.05, order=2)]
    b = F.Batch(cases, precision="mixed")
    assert b.autotune(steps=3) > 0
    for i in range(len(cases)):
        assert b.active_precision(i) == "fp32", i   # re-seeded in float
        b.init_equilibrium(i)
    status, reps = b.solve(1e-9, 300000, check_every=100)
    assert status == 0
    for i, case in enumerate(cases):
        assert b.active_precision(i) == "fp64", i
        op = OP.from_case(case)
        fo, steps, hist = op.solve(op.equilibrium(), 1e-11, 600000)
        rho, ux, uy, _ = b.moments(i)
        r0, ux0, uy0 = op.moments(fo)
        assert eps_u(ux, uy, ux0, uy0) <= 2e-5, i
        assert float(np.abs(rho - r0).max()) <= 2e-5, i
