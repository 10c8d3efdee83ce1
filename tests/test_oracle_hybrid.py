"""Pins of the hybrid half-range / full-range oracle (oracle/hybrid.py) against facts fixed
independently of it: polynomial exactness of the maps and Lagrange interpolation for the
bulk -> layer map, the plain half-range scheme (the C oracle) when the layers fill the
channel, the rest state and the symmetries of Couette flow, momentum conservation inside
each zone, and first-order convergence of the fully discrete scheme to the semi-analytic
solution of the same coupling (a different computation: exponential modes of the
discrete-velocity model and a linear solve for their amplitudes), which in turn tends to the
pure half-range solution exponentially as the layers thicken in units of Kn."""
import math

import numpy as np
import pytest

from oracle import quadrature
from oracle.couette import CouetteSolution
from oracle.hybrid import HybridChannel, HybridSolution, maps
from oracle.scheme import TOP, BOTTOM
from oracle.scheme import Problem as Plain


@pytest.mark.parametrize("nh,nf", [(2, 2), (3, 3), (4, 4), (4, 3), (4, 2), (2, 4)])
def test_maps_exact_on_polynomials(nh, nf):
    A, B, ka, kb = maps(nh, nf)
    xh, wh = quadrature.half_range(nh)
    xf, wf = quadrature.full_range(nf)
    rng = np.random.default_rng(nh * 10 + nf)
    for deg in range(ka + 1):
        c = rng.standard_normal(deg + 1)
        assert np.allclose(A @ (wh * np.polyval(c, xh)), wf * np.polyval(c, xf), rtol=0, atol=1e-13 * np.abs(c).sum() * 50)
    for deg in range(kb + 1):
        c = rng.standard_normal(deg + 1)
        assert np.allclose(B @ (wf * np.polyval(c, xf)), wh * np.polyval(c, xh), rtol=0, atol=1e-13 * np.abs(c).sum() * 50)
    # one degree more is no longer carried exactly by the truncated layer -> bulk map
    # (when the bulk rule could still hold it)
    if ka + 1 <= nf - 1:
        c = np.zeros(ka + 2)
        c[0] = 1.0
        assert np.abs(A @ (wh * np.polyval(c, xh)) - wf * np.polyval(c, xf)).max() > 1e-6


@pytest.mark.parametrize("nh,nf", [(2, 2), (4, 4), (4, 3), (3, 2)])
def test_bulk_to_layer_map_is_lagrange_interpolation(nh, nf):
    """B evaluates at the layer nodes the polynomial of degree nf - 1 through the bulk values
    g/w: the Hermite route and Lagrange's formula agree for arbitrary data."""
    _, B, _, _ = maps(nh, nf)
    xh, wh = quadrature.half_range(nh)
    xf, wf = quadrature.full_range(nf)
    g = np.random.default_rng(7).standard_normal(nf) * wf
    phi = g / wf
    lag = np.zeros_like(xh)
    for k in range(nf):
        others = [xf[m] for m in range(nf) if m != k]
        basis = np.prod([(xh - o) / (xf[k] - o) for o in others], axis=0) if others else np.ones_like(xh)
        lag += phi[k] * basis
    assert np.allclose(B @ g, wh * lag, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("nh,qx", [(2, ("full", 3)), (4, ("full", 2))])
def test_layers_filling_the_channel_equal_the_plain_scheme(nh, qx):
    ny, kn = 24, 0.07
    ch = HybridChannel(ny, ny // 2, kn, (-0.01, 0.01), n_half=nh, n_full=nh, qx=qx)
    pl = Plain(1, ny, True, False, (-0.01, 0.01, 0.0, 0.0), kn, qx, ("half", nh))
    assert ch.dt == pl.dt
    s = ch.step(ch.equilibrium(), 300)
    f = pl.step(pl.equilibrium(), 300)
    # plain layout f[alpha][y][x], alpha = y node * Nx + x node
    fh = s[0].reshape(ny, -1).T.reshape(pl.q, ny, 1)
    assert np.abs(fh - f).max() <= 1e-13 * np.abs(f).max()
    r, ux, uy = ch.moments(s)
    r2, ux2, uy2 = pl.moments(f)
    assert np.abs(ux - ux2[:, 0]).max() <= 1e-13 * np.abs(ux2).max()
    for wall, idx in ((BOTTOM, 0), (TOP, 1)):
        _, ut, pw = pl.wall_profile(f, wall)
        u_h, p_h = ch.wall_face(s, idx)
        assert abs(u_h - ut[0]) <= 1e-13 * abs(ut[0]) and abs(p_h - pw[0]) <= 1e-13 * abs(pw[0])


@pytest.mark.parametrize("nh,nf", [(2, 2), (4, 3)])
def test_rest_state_stays_at_rest(nh, nf):
    ch = HybridChannel(20, 4, 0.1, (0.0, 0.0), n_half=nh, n_full=nf)
    s0 = ch.equilibrium(rho=np.full(20, 1.3))
    s = ch.step(s0, 200)
    for a, b in zip(s, s0):
        assert np.abs(a - b).max() <= 1e-15 * 1.3 * 4


def test_couette_invariants():
    ch = HybridChannel(30, 6, 0.1, (-0.01, 0.01), n_half=4, n_full=3)
    s = ch.step(ch.equilibrium(), 500)
    rho, ux, uy = ch.moments(s)
    scale = np.abs(ux).max()
    assert scale > 1e-4
    assert np.abs(rho - 1).max() <= 1e-14
    assert np.abs(uy).max() <= 1e-13 * scale
    assert np.abs(ux + ux[::-1]).max() <= 1e-13 * scale


def test_momentum_flux_uniform_inside_each_zone():
    """At the steady state the y-flux of x-momentum is the same through every face of a zone
    and equals the stress of the wall's face state; the layer and bulk values differ by the
    interface's conservation defect."""
    ny, L = 40, 8
    ch = HybridChannel(ny, L, 0.1, (-0.01, 0.01), n_half=4, n_full=3)
    s, n, hist = ch.solve(ch.equilibrium(), 1e-14, 200000)
    assert hist[-1] < 1e-14
    ff = ch.face_fluxes(s)
    layer_faces = [(0, k) for k in range(0, L + 1)] + [(1, k) for k in range(0, L)]
    layer_faces += [(1, k) for k in range(ny - L, ny + 1)] + [(0, k) for k in range(ny - L + 1, ny + 1)]
    bulk_faces = [(1, k) for k in range(L, ny - L)] + [(0, k) for k in range(L + 1, ny - L + 1)]
    lay = np.array([ff[a, k] for a, k in layer_faces])
    blk = np.array([ff[a, k] for a, k in bulk_faces])
    _, p_wall = ch.wall_face(s, 0)
    assert np.abs(lay - p_wall).max() <= 1e-10 * abs(p_wall)
    assert np.abs(blk - blk.mean()).max() <= 1e-10 * abs(p_wall)
    assert abs(blk.mean() - p_wall) > 1e-4 * abs(p_wall)   # the defect is real at this depth
    pc = ch.pxy(s)
    assert np.isfinite(pc).all()


def _steady(ny, L, kn, nh, nf):
    ch = HybridChannel(ny, L, kn, (-1.0, 1.0), n_half=nh, n_full=nf)
    s, n, hist = ch.solve(ch.equilibrium(), 1e-13, 400000)
    assert hist[-1] < 1e-13
    ff = ch.face_fluxes(s)
    u_wall, p_layer = ch.wall_face(s, 0)
    return u_wall, p_layer, ff[1, ny // 2]


@pytest.mark.parametrize("nh,nf,grids,tol", [(2, 2, (100, 200), 1e-4), (4, 3, (50, 100), 4e-4)])
def test_scheme_converges_to_semi_analytic_hybrid(nh, nf, grids, tol):
    """Kn = 0.1, layers of thickness 0.2: the fully discrete hybrid on N and 2N cells,
    Richardson-extrapolated, against the semi-analytic solution of the coupling (wall slip,
    layer stress, bulk stress); the errors of the slip and of the layer stress halve."""
    kn, delta = 0.1, 0.2
    (n1, n2) = grids
    a = _steady(n1, int(round(delta * n1)), kn, nh, nf)
    b = _steady(n2, int(round(delta * n2)), kn, nh, nf)
    ex = HybridSolution(nh, nf, kn, delta, 1.0)
    # face state at the lower plate moving at -1: u_wall = -(1 - slip)
    exact = (ex.wall_u(), ex.pxy_layer(), ex.pxy_bulk())
    for i, (va, vb, e) in enumerate(zip(a, b, exact)):
        rich = 2 * vb - va
        assert abs(rich - e) <= tol * abs(e), (va, vb, rich, e)
        if i < 2:
            assert 1.6 < (va - e) / (vb - e) < 2.5
    assert abs(exact[1] - exact[2]) > 1e-3 * abs(exact[1]) or (nh, nf) == (2, 2)


def test_semi_analytic_hybrid_tends_to_the_half_range_solution():
    """Kn = 0.02, 2 nodes per half in the layers and 2 full-range nodes in the bulk (the
    paper's N -> N/2 pairing for one axis): the stress and the slip of the hybrid approach
    those of the pure half-range model exponentially in delta/Kn, and the stress defect at
    the interface vanishes with them."""
    kn = 0.02
    pure = CouetteSolution(2, kn, 1.0)
    prev = None
    for delta in (0.05, 0.1, 0.2, 0.3):
        h = HybridSolution(2, 2, kn, delta, 1.0)
        err = max(abs(h.pxy_layer() / pure.pxy() - 1), abs(h.pxy_bulk() / pure.pxy() - 1),
                  abs(h.wall_u() / pure.u(-0.5) - 1))
        if prev is not None:
            assert err < prev / 10, (delta, err, prev)
        prev = err
    assert prev < 1e-9


def test_semi_analytic_hybrid_profile_antisymmetry_and_interface_jump():
    """The profile is antisymmetric; u jumps at the interface by the coupling's defect (the
    two zones see different distributions there), and the jump shrinks as the layer thickens."""
    h = HybridSolution(4, 3, 0.1, 0.2, 1.0)
    assert abs(h.u(0.0)) < 1e-15
    assert abs(h.u(0.3) + h.u(-0.3)) < 1e-15
    jumps = []
    for delta in (0.1, 0.2, 0.3, 0.4):
        h = HybridSolution(4, 3, 0.05, delta, 1.0)
        y1 = 0.5 - delta
        jumps.append(abs(h.u(-y1 - 1e-12) - h.u(-y1 + 1e-12)) / abs(h.u(-0.5) - h.u(-y1)))
    assert all(b < a / 2 for a, b in zip(jumps, jumps[1:])), jumps
    assert jumps[-1] < 1e-3
