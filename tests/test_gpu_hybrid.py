"""The hybrid half-range / full-range channel (fdlb_hybrid_*) against the oracle
(oracle/hybrid.py): states after equal step counts to 1e-12 relative on layer/bulk set pairs,
x rules, odd and even grids, thin and filling layers, Kn from 0.005 to infinity, one channel
and many per launch; steady solves (step counts, states, residual history); cell moments,
stress, plate faces and interface fluxes; the plain GPU Couette when the layers fill the
channel; grid convergence to the semi-analytic solution of the coupling; and the errors."""
import math

import numpy as np
import pytest

from oracle.hybrid import HybridChannel, HybridSolution

pytestmark = pytest.mark.gpu

CASES = [
    dict(ny=24, layer=5, kn=0.1, n_half=2, n_full=2, qx=("full", 3)),
    dict(ny=37, layer=1, kn=0.05, n_half=4, n_full=3, qx=("full", 3)),
    dict(ny=64, layer=12, kn=math.inf, n_half=4, n_full=4, qx=("half", 2)),
    dict(ny=30, layer=15, kn=0.2, n_half=3, n_full=3, qx=("full", 2)),
    dict(ny=40, layer=7, kn=0.02, n_half=2, n_full=4, qx=("full", 4)),
    dict(ny=33, layer=3, kn=1.0, n_half=8, n_full=2, qx=("full", 3)),
    dict(ny=50, layer=10, kn=0.005, n_half=5, n_full=7, qx=("full", 3)),
]


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_0692_amd as F
    return F


def _oracle(c, u_w):
    return HybridChannel(c["ny"], c["layer"], c["kn"], u_w, n_half=c["n_half"], n_full=c["n_full"], qx=c["qx"])


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("c", CASES, ids=[f"ny{c['ny']}-L{c['layer']}-h{c['n_half']}f{c['n_full']}" for c in CASES])
def test_steps_match_oracle(F, c):
    u_w = (-0.01, 0.02)
    h = F.Hybrid([dict(c, u_w=u_w)])
    o = _oracle(c, u_w)
    assert h.info[0]["dt"] == o.dt and h.info[0]["omega"] == o.omega
    # a seeded non-uniform start exercises every moment and the interface maps in both directions
    rng = np.random.default_rng(c["ny"])
    y = (np.arange(c["ny"]) + 0.5) / c["ny"]
    rho = 1.0 + 0.05 * np.sin(3 * y) + 0.01 * rng.standard_normal(c["ny"])
    ux = 0.01 * np.cos(5 * y)
    uy = 0.003 * rng.standard_normal(c["ny"])
    h.init_equilibrium(0, rho, ux, uy)
    s0 = o.equilibrium(rho, ux, uy)
    assert _rel(h.state(0), o.pack(s0)) <= 1e-15
    for n in (1, 7, 300):
        h.step(n)
        s0 = o.step(s0, n)
        assert _rel(h.state(0), o.pack(s0)) <= 1e-12, n
    h.close()


def test_batch_of_channels_one_launch(F):
    u_w = (-0.01, 0.01)
    h = F.Hybrid([dict(c, u_w=u_w) for c in CASES])
    h.init_all()
    h.step(250)
    for i, c in enumerate(CASES):
        o = _oracle(c, u_w)
        s = o.step(o.equilibrium(), 250)
        assert _rel(h.state(i), o.pack(s)) <= 1e-12, c
    h.close()


@pytest.mark.parametrize("c", [CASES[0], CASES[1], CASES[4]])
def test_solve_matches_oracle(F, c):
    u_w = (-0.01, 0.01)
    h = F.Hybrid([dict(c, u_w=u_w)])
    h.init_all()
    code, reps = h.solve(1e-11, 200000, chunk=997, history_cap=64)
    o = _oracle(c, u_w)
    s, n, hist = o.solve(o.equilibrium(), 1e-11, 200000)
    r = reps[0]
    assert code == 0 and r["status"] == 0
    assert abs(r["steps"] - n) <= 1 and r["first_below"] == r["steps"]
    assert r["residual"] < 1e-11
    if r["steps"] == n:
        assert _rel(h.state(0), o.pack(s)) <= 1e-11
        k = len(r["history"])
        assert k == 64
        # near the tolerance |u^{n+1} - u^n| ~ 1e-13 per cell while u carries rounding of ~1e-16
        # from populations of order 0.1: the residual itself is only good to ~1e-3 there
        assert np.allclose(r["history"], hist[-k:], rtol=5e-3, atol=0)
    rho, ux, uy, pxy = h.moments(0)
    r0, ux0, uy0 = o.moments(s)
    assert _rel(ux, ux0) <= 1e-8 and np.abs(rho - r0).max() <= 1e-12
    h.close()


@pytest.mark.parametrize("c", [CASES[1], CASES[2], CASES[3], CASES[6]])
def test_outputs_match_oracle(F, c):
    u_w = (-0.01, 0.02)
    h = F.Hybrid([dict(c, u_w=u_w)])
    h.init_all()
    h.step(400)
    o = _oracle(c, u_w)
    s = o.step(o.equilibrium(), 400)
    rho, ux, uy, pxy = h.moments(0)
    r0, ux0, uy0 = o.moments(s)
    assert np.abs(rho - r0).max() <= 1e-12
    assert _rel(ux, ux0) <= 1e-12 and np.abs(uy - uy0).max() <= 1e-12 * np.abs(ux0).max()
    # stresses are sums of populations of order 0.1 that cancel to 1e-5 at small Kn: their
    # rounding is set by the populations, 1e-16 x 0.1 per term, hence the absolute floor
    floor = 1e-15
    p0 = o.pxy(s)
    assert np.abs(pxy - p0).max() <= 1e-12 * np.abs(p0).max() + floor
    faces = h.faces(0)
    for wall in (0, 1):
        ut, pw = o.wall_face(s, wall)
        assert abs(faces[2 * wall] - ut) <= 1e-12 * abs(ut) and abs(faces[2 * wall + 1] - pw) <= 1e-12 * abs(pw) + floor
    L, ny = c["layer"], c["ny"]
    if 2 * L < ny:
        ff = o.face_fluxes(s)
        want = [ff[0, L], ff[1, L], ff[0, ny - L], ff[1, ny - L]]
        assert np.allclose(faces[4:], want, rtol=1e-12, atol=floor)
    else:
        assert np.isnan(faces[4:]).all()
    h.close()


def test_layers_filling_the_channel_equal_plain_gpu_couette(F):
    """2 layer == ny: no bulk, the hybrid kernel and the plain library (its general 2-D step
    kernel, FP64) march the same half-range Couette scheme."""
    import workloads as W
    ny = 40
    h = F.Hybrid([dict(ny=ny, layer=ny // 2, kn=0.1, n_half=4, n_full=4, qx=("full", 3))])
    h.init_all()
    h.step(600)
    case = W.couette(ny=ny, kn=0.1)
    p = F.Problem(case, precision="fp64")
    p.init_equilibrium()
    p.step(600)
    rho, ux, uy, pxy = p.moments()
    r1, ux1, uy1, pxy1 = h.moments(0)
    assert _rel(ux1, ux[:, 0]) <= 1e-12 and np.abs(r1 - rho[:, 0]).max() <= 1e-12
    _, ut, pw = p.wall_profile(F.TOP)
    faces = h.faces(0)
    assert abs(faces[2] - ut[0]) <= 1e-12 * abs(ut[0]) and abs(faces[3] - pw[0]) <= 1e-12 * abs(pw[0])
    p.close()
    h.close()


def test_converges_to_semi_analytic_hybrid(F):
    """Kn = 0.1, 4 nodes per half in the layers (thickness 0.2) and the 3-node bulk rule, on
    200 and 400 cells solved to 1e-13 in one batch: the Richardson values of the plate slip
    and of the layer and bulk stresses within 3e-5 of the semi-analytic coupling."""
    kn, delta = 0.1, 0.2
    chans = [dict(ny=n, layer=int(delta * n), kn=kn, u_w=(-1.0, 1.0), n_half=4, n_full=3, qx=("full", 3))
             for n in (200, 400)]
    h = F.Hybrid(chans)
    h.init_all()
    code, reps = h.solve(1e-13, 2_000_000)
    assert code == 0
    vals = []
    for i in range(2):
        f = h.faces(i)
        vals.append((f[0], f[1], f[5]))
    ex = HybridSolution(4, 3, kn, delta, 1.0)
    exact = (ex.wall_u(), ex.pxy_layer(), ex.pxy_bulk())
    for (a, b, e) in zip(vals[0], vals[1], exact):
        assert abs((2 * b - a) - e) <= 3e-5 * abs(e), (a, b, 2 * b - a, e)
    assert abs(exact[1] - exact[2]) > 1e-3 * abs(exact[1])
    h.close()


def test_errors(F):
    from paper_1308_0692_amd import FdlbError
    big = dict(ny=4096, layer=2048, kn=0.1, n_half=8, n_full=8, qx=("full", 3))
    with pytest.raises(FdlbError) as e:
        F.Hybrid([big])
    assert e.value.code == -1 and "LDS" in str(e.value)
    h = F.Hybrid([CASES[0]])
    with pytest.raises(FdlbError):
        h.init_equilibrium(0, rho=np.zeros(CASES[0]["ny"]))
    buf = np.empty(10)
    assert F._lib.lib.fdlb_hybrid_get_state(h._h, 5, F._lib._dp(buf)) == F._lib.EINVAL
    assert F._lib.lib.fdlb_hybrid_step(h._h, -1) == F._lib.EINVAL
    h.close()


def test_poisoned_buffers_give_the_same_results(F):
    """Every device buffer filled with NaN bytes before binding: a read of memory the library
    did not write first (the residual ring before its first block, padding, the unused rows of
    the layout) would show up as NaN; the results equal those of clean buffers bit for bit."""
    chans = [dict(CASES[1], u_w=(-0.01, 0.01)), dict(CASES[4], u_w=(-0.01, 0.01))]
    out = []
    for poison in (False, True):
        h = F.Hybrid(chans, poison=poison)
        h.init_all()
        code, reps = h.solve(1e-10, 100000, chunk=777, history_cap=200)
        assert code == 0
        out.append(([h.state(i) for i in range(2)], [r["history"] for r in reps], [r["steps"] for r in reps]))
        h.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0][1], out[1][1]):
        assert np.isfinite(b).all() and np.array_equal(a, b)
    assert out[0][2] == out[1][2]
