"""Batched solves: many problems in one launch per step.  Each member must evolve exactly
as it does alone (same tile: bit-identical, including the step at which it stops), match
the oracle, and be isolated from members that diverge."""
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


MIXED = [W.cavity(64, kn=0.3, order=2), W.cavity(48, ny=40, kn=1.0, order=3),
         W.cavity(96, kn=0.1, order=4), W.cavity(32, kn=3.0, order=2),
         W.cavity(40, ny=72, kn=0.05, order=2), W.cavity(64, kn=10.0, order=3)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_members_equal_solo_runs(F, prec):
    b = F.Batch(MIXED, precision=prec)
    b.set_retile(0)  # one tile throughout: bit-identical to single solves with that tile
    for i in range(len(MIXED)):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-7, 60000, check_every=50)
    assert status == 0, [r["status"] for r in reps]
    for i, case in enumerate(MIXED):
        p = F.Problem(case, precision=prec)
        p.set_tile(b.tile)
        p.init_equilibrium()
        rep = p.solve(1e-7, 60000, check_every=50)
        assert rep["steps"] == reps[i]["steps"] == reps[i]["first_below"], i
        assert np.array_equal(p.download(), b.download(i, p.q)), i
        assert np.array_equal(p.moments()[1], b.moments(i)[1]), i


@pytest.mark.parametrize("case", [W.cavity(40, ny=28, kn=0.2, order=3), W.couette(90, kn=0.3)],
                         ids=["cavity", "couette"])
def test_one_member_batch_equals_single_problem(F, case):
    """A batch of one problem (on its built-in shape, column tiles for the channel) marches bit
    for bit like the problem alone on the same shape."""
    b = F.Batch([case], precision="fp32")
    b.init_equilibrium(0)
    status, reps = b.solve(1e-6, 40000, check_every=40)
    assert status == 0
    p = F.Problem(case, precision="fp32")
    p.set_tile(b.tile)
    p.init_equilibrium()
    rep = p.solve(1e-6, 40000, check_every=40)
    assert rep["steps"] == reps[0]["steps"]
    assert np.array_equal(p.download(), b.download(0, p.q))


def test_batch_fp64_matches_oracle_at_fixed_steps(F):
    cases = MIXED[:4]
    b = F.Batch(cases, precision="fp64")
    for i in range(len(cases)):
        b.init_equilibrium(i)
    status, reps = b.solve(0.0, 37, check_every=10)   # tol 0: every member takes 37 steps
    assert status == 1 and all(r["steps"] == 37 for r in reps)
    for i, case in enumerate(cases):
        op = OP.from_case(case)
        fo = op.step(op.equilibrium(), 37)
        f = b.download(i, op.q)
        dev = np.abs(fo - op.w[:, None, None]).max()
        assert np.abs(f - fo).max() <= 1e-12 * dev, i


def test_batch_isolates_a_diverging_member(F):
    good = [W.cavity(48, kn=0.2, order=2), W.cavity(64, kn=1.0, order=2)]
    bad = W.with_(W.cavity(48, kn=0.2, order=2), cfl=2.0)
    b = F.Batch([good[0], bad, good[1]], precision="fp32", allow_unstable=True)
    for i in range(3):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-6, 50000, check_every=40)
    assert status == F._lib.EDIVERGED
    assert reps[1]["status"] == F._lib.EDIVERGED
    assert reps[0]["status"] == 0 and reps[2]["status"] == 0
    for i, j in ((0, 0), (2, 1)):
        p = F.Problem(good[j], precision="fp32")
        p.set_tile(b.tile)
        p.init_equilibrium()
        rep = p.solve(1e-6, 50000, check_every=40)
        assert rep["steps"] == reps[i]["steps"]
        assert np.array_equal(p.download(), b.download(i, p.q))


def test_batch_reports_unconverged_members(F):
    b = F.Batch([W.cavity(32, kn=0.1, order=2), W.cavity(32, kn=5.0, order=2)], precision="fp32")
    for i in range(2):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-12, 30, check_every=10)
    assert status == 1
    assert all(r["status"] == 1 and r["steps"] == 30 for r in reps)


def test_batch_autotune_and_graph_vs_eager(F):
    cases = MIXED[:3]
    a = F.Batch(cases, precision="fp32")
    ms = a.autotune(steps=3)
    assert ms > 0
    b = F.Batch(cases, precision="fp32")
    b.set_tile(a.tile)
    for i in range(3):
        a.init_equilibrium(i)
        b.init_equilibrium(i)
    for rep in range(3):
        a.solve(0.0, 20, check_every=20, use_graph=True)
        b.solve(0.0, 20, check_every=5, use_graph=False)
        for i, c in enumerate(cases):
            assert np.array_equal(a.download(i, c.q), b.download(i, c.q)), (rep, i)


def test_sweep_full_size_sampled_members_match_oracle(F):
    """The 64-cavity sweep at its real sizes, in the launch configuration the benchmark times
    (mixed precision, float phase, the autotuned tile, and every other float shape that fits all
    members, so whichever one the autotuner picks): five steps from seeded non-uniform
    equilibria; the smallest, the largest and one middle instance against the oracle run at
    full size (FP32 bars: 2e-6 on the populations relative to the deviation scale, 2e-5 on
    rho and u)."""
    cases = W.c3_instances()
    b = F.Batch(cases, precision="mixed")
    b.autotune(steps=2)
    tiles = [b.tile]
    for t in range(F.tile_count("fp32")):
        if t != tiles[0]:
            try:
                b.set_tile(t)
                tiles.append(t)
            except F.FdlbError:
                pass
    assert len(tiles) >= 5
    fields = [W.random_fields(c.nx, c.ny, seed=100 + i, amp=0.01) for i, c in enumerate(cases)]
    sizes = [c.nx * c.ny * c.q for c in cases]
    order = np.argsort(sizes)
    refs = {}
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        op = OP.from_case(cases[i])
        fo = op.step(op.equilibrium(*fields[i]), 5)
        refs[i] = (op, fo, op.moments(fo))
    for t in tiles:
        b.set_tile(t)
        for i in range(len(cases)):
            b.init_equilibrium(i, *fields[i])
        status, reps = b.solve(0.0, 5, check_every=5)
        assert all(r["steps"] == 5 for r in reps), t
        for i, (op, fo, (r0, ux0, uy0)) in refs.items():
            assert b.active_precision(i) == "fp32"
            f = b.download(i, op.q)
            dev = np.abs(fo - op.w[:, None, None]).max()
            assert np.abs(f - fo).max() <= 2e-6 * dev, (t, i, cases[i].nx, op.q)
            rho, ux, uy, _ = b.moments(i)
            assert float(np.hypot(ux - ux0, uy - uy0).max() / np.hypot(ux0, uy0).max()) <= 2e-5, (t, i)
            assert float(np.abs(rho - r0).max()) <= 2e-5, (t, i)


def test_sweep_converged_members_match_converged_oracle(F):
    """The whole 64-cavity sweep solved to R < 1e-8 as the benchmark solves it (one mixed-
    precision batch on its autotuned tile, graph-captured chunks, tail re-tiling): three members
    (Kn 0.044 with 12 x 12 velocities, Kn 0.148 and Kn 7.26 with 8 x 8, all 64^2) against the
    oracle converged to 1e-11, within the FP32 bar of 2e-5 on rho and u."""
    cases = W.c3_instances()
    b = F.Batch(cases, precision="mixed")
    b.autotune(steps=2)
    for i in range(len(cases)):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-8, 200000, check_every=200)
    assert status == 0 and all(r["status"] == 0 for r in reps)
    for i in (62, 19, 31):
        c = cases[i]
        assert c.nx == 64
        op = OP.from_case(c)
        fo, n, hist = op.solve(op.equilibrium(), 1e-11, 400000)
        assert hist[-1] < 1e-11
        r0, ux0, uy0 = op.moments(fo)
        rho, ux, uy, _ = b.moments(i)
        eu = float(np.hypot(ux - ux0, uy - uy0).max() / np.hypot(ux0, uy0).max())
        er = float(np.abs(rho - r0).max())
        print(f"member {i} (Kn {c.kn:.4f}, Q {c.q}): eps_u {eu:.2e}, eps_rho {er:.2e}")
        assert eu <= 2e-5 and er <= 2e-5, (i, eu, er)


def test_tail_retiling_keeps_results_and_restores_tiles(F):
    """With tail re-tiling the last instances switch to their single-problem tile:
    every instance still converges to its single-solve answer (the steps differ at most by the
    rounding of the residual), and the batch's tile is restored afterwards."""
    b = F.Batch(MIXED, precision="fp64")
    b.set_retile(4)  # six instances: the last four switch
    tile0 = b.tile
    for i in range(len(MIXED)):
        b.init_equilibrium(i)
    status, reps = b.solve(1e-9, 200000, check_every=50)
    assert status == 0 and b.tile == tile0
    for i, case in enumerate(MIXED):
        p = F.Problem(case, precision="fp64")
        p.set_tile(tile0)
        p.init_equilibrium()
        rep = p.solve(1e-9, 200000, check_every=50)
        assert abs(rep["steps"] - reps[i]["steps"]) <= 1, i
        _, ux, uy, _ = p.moments()
        _, bx, by, _ = b.moments(i)
        assert np.hypot(bx - ux, by - uy).max() <= 1e-7 * np.hypot(ux, uy).max(), i


def test_batch_member_upload_equals_single_problem_upload(F):
    """A member restarted from uploaded populations marches bit for bit as a single problem
    started from the same populations (same tile shape, no tail re-tiling)."""
    cases = [W.cavity(40, kn=0.3, order=2), W.cavity(28, ny=36, kn=0.8, order=3)]
    b = F.Batch(cases, precision="fp32")
    b.set_retile(0)
    rng = np.random.default_rng(5)
    fs = []
    for i, case in enumerate(cases):
        b.init_equilibrium(i)
        f = b.download(i)
        f *= 1 + 0.01 * rng.standard_normal(f.shape)
        b.upload(i, f)
        fs.append(f)
    status, reps = b.solve(1e-7, 50000, check_every=30)
    assert status == 0
    for i, case in enumerate(cases):
        p = F.Problem(case, precision="fp32")
        p.set_tile(b.tile)
        p.upload(fs[i])
        rep = p.solve(1e-7, 50000, check_every=30)
        assert rep["steps"] == reps[i]["steps"]
        assert np.array_equal(p.download(), b.download(i))
