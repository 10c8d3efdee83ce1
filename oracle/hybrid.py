"""Hybrid half-range / full-range model of planar Couette flow
(TEST INFRASTRUCTURE ONLY, see oracle/__init__.py).

The paper's closing remarks observe that away from walls a half-range model
with N velocities behaves like a full-range one with N/2^d velocities, and
propose coupling the two: half-range nodes in the Knudsen layers next to the
walls, full-range nodes in the bulk.  The paper gives no coupling; the reading
taken here, for the channel between two plates:

* cells j = 0 .. ny-1 across the channel (y = (j + 1/2)/ny); the first and the
  last ``layer`` cells carry the tensor product of the x rule with a half-range
  y rule of n_h nodes per half-line (the layer set), the cells between carry
  the x rule times an n_f-node full-range y rule (the bulk set); x is periodic
  with one cell, so only y transport acts;
* every cell relaxes with its own set (Eqs. 1, 5: explicit Euler toward the
  linearised equilibrium built from the moments of that set, Eqs. 6-7) and
  then every population moves by the donor cell in y, as in the plain scheme;
* the walls are those of the plain scheme (Eqs. 8-9, the density of the
  emission being the arriving flux over the flux one unit of emitted density
  carries), acting on the layer cells;
* where the donor cell of a population lies in the other zone, its value there
  is the other zone's post-relaxation distribution carried over to this zone's
  nodes through a Hermite expansion in xi_y, for each x node separately: the
  coefficients c_m = (1/m!) sum_a g_a He_m(xi_a) are taken with the source
  rule, and g'_k = w'_k sum_{m<=K} c_m He_m(xi'_k) is evaluated at the target
  nodes.  Bulk -> layer uses K = n_f - 1 (all an n_f-node distribution holds);
  layer -> bulk uses K = min(n_h, n_f) - 1: the half-range rule integrates
  degree 2 n_h - 1 exactly, so the coefficients of a polynomial of degree
  <= K are exact for every m <= K only up to K = n_h - 1.  Both maps carry
  every w * polynomial of degree <= K exactly, the equilibrium w (rho + xi j)
  among them, so a rest state stays at rest and a near-equilibrium bulk
  crosses the interface unchanged;
* time step dt = cfl / (ny max |xi_y|) over the y rules present.

The interface is not exactly conservative: the two zones split a face flux
into half-fluxes with different rules, so the momentum flux seen from either
side differs by an amount that vanishes when the distribution at the
interface is a polynomial of degree <= K in xi_y (far enough from the walls,
in units of Kn).  With 2 * layer == ny there is no bulk and the scheme is the
plain half-range scheme.

``HybridSolution`` is the semi-analytic steady solution of the same coupling
with continuous y (modes of the discrete-velocity model in each zone, the
interface conditions above at y = +-y1), the limit the scheme approaches at
first order in dy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import mpmath as mp
import numpy as np

from . import quadrature
from .couette import _positive_half, _roots

_DPS = 60


def hermite_e(m: int, x):
    """Probabilists' Hermite polynomial He_m(x) by its three-term recurrence
    He_{k+1} = x He_k - k He_{k-1} (works on mpmath numbers and numpy arrays)."""
    if m == 0:
        return x * 0 + 1
    p0, p1 = x * 0 + 1, x
    for k in range(1, m):
        p0, p1 = p1, x * p1 - k * p0
    return p1


def transfer_matrix(src_nodes, dst_nodes, dst_weights, degree: int) -> np.ndarray:
    """T[k, a] such that g'_k = sum_a T[k, a] g_a carries a weighted distribution g on
    src_nodes to dst_nodes through its Hermite expansion truncated at ``degree``.
    Built in mpmath and rounded once."""
    with mp.workdps(_DPS):
        src = [mp.mpf(v) for v in src_nodes]
        dst = [mp.mpf(v) for v in dst_nodes]
        wd = [mp.mpf(v) for v in dst_weights]
        T = np.empty((len(dst), len(src)))
        for k, xk in enumerate(dst):
            for a, xa in enumerate(src):
                s = mp.fsum(hermite_e(m, xk) * hermite_e(m, xa) / mp.factorial(m) for m in range(degree + 1))
                T[k, a] = float(wd[k] * s)
    return T


def _mp_rule(kind: str, n: int):
    """Full node list (ascending) and weights of a y rule in mpmath."""
    if kind == "half":
        x, w = quadrature.half_range_mp(n)
        return [-v for v in reversed(x)] + list(x), list(reversed(w)) + list(w)
    x, w = quadrature.full_range_mp(n)
    xs = [(x[i] - x[n - 1 - i]) / 2 for i in range(n)]
    ws = [(w[i] + w[n - 1 - i]) / 2 for i in range(n)]
    return xs, ws


def maps(n_half: int, n_full: int):
    """(A, B, KA, KB): A carries a layer distribution (2 n_half y nodes) to the bulk nodes,
    B a bulk distribution (n_full nodes) to the layer nodes."""
    ka = min(n_half, n_full) - 1
    kb = n_full - 1
    with mp.workdps(_DPS):
        xh, wh = _mp_rule("half", n_half)
        xf, wf = _mp_rule("full", n_full)
        A = transfer_matrix(xh, xf, wf, ka)
        B = transfer_matrix(xf, xh, wh, kb)
    return A, B, ka, kb


@dataclass
class HybridChannel:
    """The fully discrete hybrid scheme on a channel of ny cells between plates at y = 0
    (speed u_w[0]) and y = 1 (speed u_w[1]).  States are pairs (fh, ff) of arrays of
    shape (ny, Ny, Nx): populations on the layer set and on the bulk set for every cell
    (only the cells of each zone are meaningful; the other rows are kept at zero)."""

    ny: int
    layer: int
    kn: float
    u_w: Tuple[float, float] = (-0.01, 0.01)
    n_half: int = 4
    n_full: Optional[int] = None
    qx: Tuple[str, int] = ("full", 3)
    cfl: float = 0.9
    A: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        if self.n_full is None:
            self.n_full = self.n_half
        if not (1 <= self.layer and 2 * self.layer <= self.ny):
            raise ValueError("need 1 <= layer <= ny / 2")
        self.xx, self.wx = quadrature.rule(*self.qx)
        self.yh, self.wh = quadrature.half_range(self.n_half)
        self.yf, self.wf = quadrature.full_range(self.n_full)
        self.dy = 1.0 / self.ny
        self.has_bulk = 2 * self.layer < self.ny
        vmax = np.max(np.abs(self.yh))
        if self.has_bulk:
            vmax = max(vmax, np.max(np.abs(self.yf)))
        self.dt = self.cfl / (float(vmax) * self.ny)
        self.omega = 0.0 if math.isinf(self.kn) else self.dt / self.kn
        self.A, self.B, self.ka, self.kb = maps(self.n_half, self.n_full)
        j = np.arange(self.ny)
        self.in_layer = (j < self.layer) | (j >= self.ny - self.layer)
        # per-set velocity grids (y index major, x fastest) with tensor weights
        self.sets = {}
        for name, (yn, yw) in (("h", (self.yh, self.wh)), ("f", (self.yf, self.wf))):
            XI_Y, XI_X = np.meshgrid(yn, self.xx, indexing="ij")
            W = np.outer(yw, self.wx)
            self.sets[name] = (XI_X, XI_Y, W)

    # -- states -------------------------------------------------------------
    def equilibrium(self, rho=None, ux=None, uy=None):
        """f = w (rho + xi . rho u) on each cell's own set (Eqs. 3, 5)."""
        rho = np.ones(self.ny) if rho is None else np.asarray(rho, float)
        ux = np.zeros(self.ny) if ux is None else np.asarray(ux, float)
        uy = np.zeros(self.ny) if uy is None else np.asarray(uy, float)
        out = []
        for name, mask in (("h", self.in_layer), ("f", ~self.in_layer)):
            XI_X, XI_Y, W = self.sets[name]
            f = W[None] * (rho[:, None, None] + XI_X[None] * (rho * ux)[:, None, None]
                           + XI_Y[None] * (rho * uy)[:, None, None])
            f[~mask] = 0.0
            out.append(f)
        return tuple(out)

    def _moments_of(self, name, f):
        XI_X, XI_Y, _ = self.sets[name]
        return f.sum(axis=(1, 2)), (XI_X[None] * f).sum(axis=(1, 2)), (XI_Y[None] * f).sum(axis=(1, 2))

    def moments(self, state):
        """rho, u_x, u_y per cell (Eqs. 6-7 over each cell's own set)."""
        rho, jx, jy = np.zeros(self.ny), np.zeros(self.ny), np.zeros(self.ny)
        for name, f, mask in (("h", state[0], self.in_layer), ("f", state[1], ~self.in_layer)):
            r, a, b = self._moments_of(name, f)
            rho[mask], jx[mask], jy[mask] = r[mask], a[mask], b[mask]
        return rho, jx / rho, jy / rho

    def relax(self, state):
        """Post-relaxation populations g = (1 - omega) f + omega w (rho + xi . j)."""
        out = []
        for name, f, mask in (("h", state[0], self.in_layer), ("f", state[1], ~self.in_layer)):
            XI_X, XI_Y, W = self.sets[name]
            r, a, b = self._moments_of(name, f)
            feq = W[None] * (r[:, None, None] + XI_X[None] * a[:, None, None] + XI_Y[None] * b[:, None, None])
            g = (1.0 - self.omega) * f + self.omega * feq
            g[~mask] = 0.0
            out.append(g)
        return tuple(out)

    def wall_emission(self, gh, wall: int):
        """(rho_w, emitted populations on the layer set) at the bottom (0) or top (1) plate."""
        XI_X, XI_Y, W = self.sets["h"]
        if wall == 0:
            cell, arriving, leaving = gh[0], XI_Y < 0, XI_Y > 0
        else:
            cell, arriving, leaving = gh[self.ny - 1], XI_Y > 0, XI_Y < 0
        flux_in = np.sum(np.abs(XI_Y[arriving]) * cell[arriving])
        per_density = np.sum(np.abs(XI_Y[leaving]) * W[leaving])
        rho_w = flux_in / per_density
        ghost = W * rho_w * (1.0 + XI_X * self.u_w[wall])
        return rho_w, ghost

    def carried(self, g_src, to: str):
        """A post-relaxation distribution of one cell carried to the other zone's nodes
        (y index major: the map acts on the y index for every x node)."""
        T = self.A if to == "f" else self.B
        return T @ g_src

    def step(self, state, nsteps: int = 1):
        s = (state[0].copy(), state[1].copy())
        for _ in range(int(nsteps)):
            s = self._one_step(s)
        return s

    def _one_step(self, state):
        gh, gf = self.relax(state)
        _, ghost_b = self.wall_emission(gh, 0)
        _, ghost_t = self.wall_emission(gh, 1)
        ny = self.ny
        new = []
        for name, g, own in (("h", gh, self.in_layer), ("f", gf, ~self.in_layer)):
            XI_X, XI_Y, W = self.sets[name]
            # upwind values seen in this zone's representation, cells -1 .. ny
            ext = np.zeros((ny + 2,) + g.shape[1:])
            ext[1:-1][own] = g[own]
            other = gf if name == "h" else gh
            for j in np.nonzero(~own)[0]:
                # only a cell next to this zone is ever an upwind cell of it
                if (j > 0 and own[j - 1]) or (j + 1 < ny and own[j + 1]):
                    ext[1 + j] = self.carried(other[j], name)
            if name == "h":
                ext[0], ext[-1] = ghost_b, ghost_t
            nu = self.dt * np.abs(XI_Y) / self.dy
            up = np.where(XI_Y[None] > 0, ext[:-2], np.where(XI_Y[None] < 0, ext[2:], g))
            f = g - nu[None] * (g - up)
            f[~own] = 0.0
            new.append(f)
        return tuple(new)

    def residual(self, old, new) -> float:
        """R = ||u^{n+1} - u^n||_2 / ||u^{n+1}||_2 over cells, both components."""
        _, ux0, uy0 = self.moments(old)
        _, ux1, uy1 = self.moments(new)
        num = np.sum((ux1 - ux0) ** 2 + (uy1 - uy0) ** 2)
        den = np.sum(ux1 ** 2 + uy1 ** 2)
        return math.sqrt(num) / math.sqrt(den) if den > 0 else (0.0 if num == 0 else math.inf)

    def solve(self, state, tol: float, max_steps: int):
        """March until the first step whose residual is below tol.  (state, steps, history)."""
        s = (state[0].copy(), state[1].copy())
        hist = []
        for n in range(int(max_steps)):
            t = self._one_step(s)
            r = self.residual(s, t)
            hist.append(r)
            s = t
            if r < tol:
                break
        return s, len(hist), np.array(hist)

    # -- outputs ------------------------------------------------------------
    def pxy(self, state) -> np.ndarray:
        """xy stress of the post-relaxation state per cell."""
        gh, gf = self.relax(state)
        out = np.zeros(self.ny)
        for name, g, mask in (("h", gh, self.in_layer), ("f", gf, ~self.in_layer)):
            XI_X, XI_Y, _ = self.sets[name]
            p = (XI_X[None] * XI_Y[None] * g).sum(axis=(1, 2))
            out[mask] = p[mask]
        return out

    def face_fluxes(self, state) -> np.ndarray:
        """y-flux of x-momentum through every face y = k dy, k = 0..ny, as the donor cell of
        each side transports it: row 0 from the cell below the face, row 1 from the cell
        above (equal except at the two interfaces; at the plates the face state of the wall
        cell, arriving populations and the emission)."""
        gh, gf = self.relax(state)
        _, ghost_b = self.wall_emission(gh, 0)
        _, ghost_t = self.wall_emission(gh, 1)
        ny = self.ny
        out = np.zeros((2, ny + 1))
        for side in (0, 1):
            for k in range(ny + 1):
                cell = k - 1 if side == 0 else k      # the cell whose update this face belongs to
                cell = min(max(cell, 0), ny - 1)
                name = "h" if self.in_layer[cell] else "f"
                XI_X, XI_Y, _ = self.sets[name]
                g_own = (gh if name == "h" else gf)

                def seen(j):
                    if j < 0:
                        return ghost_b
                    if j >= ny:
                        return ghost_t
                    if self.in_layer[j] == (name == "h"):
                        return g_own[j]
                    return self.carried((gf if name == "h" else gh)[j], name)

                below, above = seen(k - 1), seen(k)
                flux = np.where(XI_Y > 0, below, np.where(XI_Y < 0, above, 0.0))
                out[side, k] = np.sum(XI_X * XI_Y * flux)
        return out

    def wall_face(self, state, wall: int):
        """(u_t, p_xy) of the face state at a plate: arriving populations of the wall cell
        (post-relaxation) and the emission."""
        gh, _ = self.relax(state)
        XI_X, XI_Y, _ = self.sets["h"]
        _, ghost = self.wall_emission(gh, wall)
        cell = gh[0] if wall == 0 else gh[self.ny - 1]
        arriving = XI_Y < 0 if wall == 0 else XI_Y > 0
        face = np.where(arriving, cell, ghost)
        rho = face.sum()
        return float((XI_X * face).sum() / rho), float((XI_X * XI_Y * face).sum())

    def pack(self, state) -> np.ndarray:
        """Flat layout shared with the library: the layer cells' populations velocity-plane by
        plane ([alpha][cell], alpha = y node * Nx + x node; cells ascending, bottom layer
        then top layer), then the bulk cells' populations the same way."""
        lay = np.nonzero(self.in_layer)[0]
        blk = np.nonzero(~self.in_layer)[0]
        h = state[0][lay].reshape(len(lay), state[0].shape[1] * state[0].shape[2]).T
        f = state[1][blk].reshape(len(blk), state[1].shape[1] * state[1].shape[2]).T
        return np.concatenate([h.ravel(), f.ravel()])

    def unpack(self, flat: np.ndarray):
        lay = np.nonzero(self.in_layer)[0]
        blk = np.nonzero(~self.in_layer)[0]
        qh, qf = len(self.yh) * len(self.xx), len(self.yf) * len(self.xx)
        fh = np.zeros((self.ny, len(self.yh), len(self.xx)))
        ff = np.zeros((self.ny, len(self.yf), len(self.xx)))
        nh = qh * len(lay)
        fh[lay] = flat[:nh].reshape(qh, len(lay)).T.reshape(len(lay), len(self.yh), len(self.xx))
        ff[blk] = flat[nh:nh + qf * len(blk)].reshape(qf, len(blk)).T.reshape(len(blk), len(self.yf), len(self.xx))
        return fh, ff


class HybridSolution:
    """Semi-analytic steady Couette solution of the hybrid model with continuous y:
    plates at y = -1/2 (-u_w) and +1/2 (+u_w), layers of thickness ``delta`` next to each
    plate on n_half nodes per half-line, the bulk |y| < y1 = 1/2 - delta on n_full
    full-range nodes, the interface conditions of the maps at y = -y1 (and by
    antisymmetry at +y1).

    With rho = 1 and u_y = 0 the populations are w (1 + xi_x B_k(y)) and each zone's
    amplitudes solve xi_k B_k' = -(B_k - u_x)/Kn with u_x = sum_k w_k B_k over its own
    nodes.  Layer zone (general solution): B_a = c + C_h (y - Kn xi_a)
      + sum_i [P_i e^{mu_i (y + y1)/Kn} / (1 + mu_i xi_a) + M_i e^{-mu_i (y + 1/2)/Kn} / (1 - mu_i xi_a)],
    mu_i the roots of the layer rule's dispersion relation; bulk zone (antisymmetric):
    B_k = C_f (y - Kn xi_k) + sum_i E_i [e^{nu_i (y - y1)/Kn}/(1 + nu_i xi_k)
      - e^{-nu_i (y + y1)/Kn}/(1 - nu_i xi_k)].
    Conditions: emission B_a(-1/2) = -u_w for xi_a > 0; bulk inflow B_k(-y1) = (A-hat B_h)(-y1)
    for xi_k > 0; layer inflow B_a(-y1) = (B-hat B_f)(-y1) for xi_a < 0, where the hatted
    maps act on amplitudes (the weights divided out).  The xy stress is -Kn C in each zone
    (the exponential modes carry none)."""

    def __init__(self, n_half: int, n_full: int, kn: float, delta: float, u_w: float = 1.0):
        with mp.workdps(_DPS):
            self.kn = kn_ = mp.mpf(kn)
            self.u_w = mp.mpf(u_w)
            self.y1 = y1 = mp.mpf(1) / 2 - mp.mpf(delta)
            if not (0 < self.y1 < mp.mpf(1) / 2):
                raise ValueError("need 0 < delta < 1/2")
            self.xh, self.wh = _mp_rule("half", n_half)
            self.xf, self.wf = _mp_rule("full", n_full)
            xp, wp = _positive_half("half", n_half)
            self.mu = _roots(xp, wp)
            xq, wq = _positive_half("full", n_full)
            self.nu = _roots(xq, wq) if len(xq) > 1 else []
            ka = min(n_half, n_full) - 1
            kb = n_full - 1

            def hat(src, dst, degree):
                # amplitude map: phi'_k = sum_a (sum_m He_m(x'_k) He_m(x_a) w_a / m!) phi_a
                src_x, src_w = src
                return [[mp.fsum(hermite_e(m, xk) * hermite_e(m, xa) / mp.factorial(m)
                                 for m in range(degree + 1)) * wa
                         for xa, wa in zip(src_x, src_w)] for xk in dst]

            self.Ahat = hat((self.xh, self.wh), self.xf, ka)
            self.Bhat = hat((self.xf, self.wf), self.xh, kb)
            nh_modes = 2 + 2 * len(self.mu)
            nf_modes = 1 + len(self.nu)
            n = nh_modes + nf_modes
            M = mp.matrix(n, n)
            rhs = mp.matrix(n, 1)
            r = 0
            # emission at the lower plate
            for a, xa in enumerate(self.xh):
                if xa > 0:
                    row = self._h_row(xa, -mp.mpf(1) / 2)
                    for c, v in enumerate(row):
                        M[r, c] = v
                    rhs[r] = -self.u_w
                    r += 1
            # bulk inflow at -y1: B_f,k(-y1) - sum_a Ahat[k][a] B_h,a(-y1) = 0 for xi_k > 0
            for k, xk in enumerate(self.xf):
                if xk > 0:
                    frow = self._f_row(xk, -y1)
                    for c, v in enumerate(frow):
                        M[r, nh_modes + c] += v
                    for a, xa in enumerate(self.xh):
                        hrow = self._h_row(xa, -y1)
                        for c, v in enumerate(hrow):
                            M[r, c] -= self.Ahat[k][a] * v
                    r += 1
            # layer inflow at -y1: B_h,a(-y1) - sum_k Bhat[a][k] B_f,k(-y1) = 0 for xi_a < 0
            for a, xa in enumerate(self.xh):
                if xa < 0:
                    hrow = self._h_row(xa, -y1)
                    for c, v in enumerate(hrow):
                        M[r, c] += v
                    for k, xk in enumerate(self.xf):
                        frow = self._f_row(xk, -y1)
                        for c, v in enumerate(frow):
                            M[r, nh_modes + c] -= self.Bhat[a][k] * v
                    r += 1
            assert r == n
            sol = mp.lu_solve(M, rhs)
            self.coef_h = [sol[i] for i in range(nh_modes)]
            self.coef_f = [sol[nh_modes + i] for i in range(nf_modes)]

    # mode rows: amplitude of node xi at y as a linear form in the zone's coefficients
    def _h_row(self, xi, y):
        kn_, y1 = self.kn, self.y1
        row = [mp.mpf(1), y - kn_ * xi]
        for mu in self.mu:
            row.append(mp.exp(mu * (y + y1) / kn_) / (1 + mu * xi))
        for mu in self.mu:
            row.append(mp.exp(-mu * (y + mp.mpf(1) / 2) / kn_) / (1 - mu * xi))
        return row

    def _f_row(self, xi, y):
        kn_, y1 = self.kn, self.y1
        row = [y - kn_ * xi]
        for nu in self.nu:
            row.append(mp.exp(nu * (y - y1) / kn_) / (1 + nu * xi)
                       - mp.exp(-nu * (y + y1) / kn_) / (1 - nu * xi))
        return row

    def amplitude(self, xi, y, zone: str) -> float:
        """B of node xi at y (y <= 0 for the layer zone; the top half by antisymmetry)."""
        with mp.workdps(_DPS):
            y, xi = mp.mpf(y), mp.mpf(xi)
            if zone == "h":
                return float(mp.fsum(c * v for c, v in zip(self.coef_h, self._h_row(xi, y))))
            return float(mp.fsum(c * v for c, v in zip(self.coef_f, self._f_row(xi, y))))

    def u(self, y) -> float:
        """u_x at y in [-1/2, 1/2] (antisymmetric)."""
        with mp.workdps(_DPS):
            y = mp.mpf(y)
            if y > 0:
                return -self.u(-y)
            if y < -self.y1:
                return float(mp.fsum(w * mp.fsum(c * v for c, v in zip(self.coef_h, self._h_row(x, y)))
                                     for x, w in zip(self.xh, self.wh)))
            return float(mp.fsum(w * mp.fsum(c * v for c, v in zip(self.coef_f, self._f_row(x, y)))
                                 for x, w in zip(self.xf, self.wf)))

    def wall_u(self) -> float:
        """u_x of the face state at the lower plate (emission for xi > 0, arriving B(-1/2))."""
        with mp.workdps(_DPS):
            y = -mp.mpf(1) / 2
            s = mp.mpf(0)
            for x, w in zip(self.xh, self.wh):
                b = -self.u_w if x > 0 else mp.fsum(c * v for c, v in zip(self.coef_h, self._h_row(x, y)))
                s += w * b
            return float(s)

    def pxy_layer(self) -> float:
        return float(-self.kn * self.coef_h[1])

    def pxy_bulk(self) -> float:
        return float(-self.kn * self.coef_f[0])
