"""Steady planar Couette flow of the discrete-velocity model, solved analytically
(TEST INFRASTRUCTURE ONLY, see oracle/__init__.py).

Semi-discrete problem (continuous y, discrete velocities): plates at
y = -1/2 (speed -u_w) and y = +1/2 (+u_w), diffuse walls (Eqs. 8-9), steady
linearised BGKW model (Eq. 1 with Eq. 5).  The paper states such a closed form
for the 2-nodes-per-half set (Eqs. 10-11, obtained along the lines of its
moment-method reference); this module derives it for any number n of nodes
per half-line, and also evaluates the printed Eqs. (10)-(11).

The same derivation holds for a full-range xi_y rule (the paper's standard
lattice) with the wall density read as the impermeability condition: the
modes pair +xi_k with -xi_k over the positive nodes, and a zero node (odd
full-range rules) adds w_0 to both sides of sum_k w_k / (1 + mu xi_k) = 1 and
drops out of the dispersion relation; its amplitude is B_0 = u_x.

Derivation (own).  With rho = 1 and u_y = 0 the populations are
f_alpha = w_alpha (1 + xi_x,alpha B_k(y)), k the index of xi_y,alpha, and the
x-momentum part obeys  xi_k B_k' = -(B_k - u_x)/Kn,  u_x = sum_k w_k B_k.
Exponential modes B_k = S e^{mu y/Kn} / (1 + mu xi_k) require
sum_k w_k / (1 + mu xi_k) = 1, i.e. (pairing +xi and -xi)
    sum_{xi_k > 0} w_k xi_k^2 / (1 - mu^2 xi_k^2) = 0,
whose n - 1 positive roots mu_i lie one between consecutive poles
1/xi_k^2 (in mu^2).  mu = 0 is a double root giving B_k = C (y - Kn xi_k).
Antisymmetry about the mid-plane pairs the modes:
    B_k(y) = C (y - Kn xi_k)
             + sum_i D_i [ e^{mu_i y/Kn}/(1 + mu_i xi_k) - e^{-mu_i y/Kn}/(1 - mu_i xi_k) ],
and the n wall conditions B_k(1/2) = u_w for the xi_k < 0 fix C and D_i.  Then
    u_x(y) = C y + 2 sum_i D_i sinh(mu_i y / Kn),      p_xy = -Kn C.
Kn is the paper's Eq. (1) Knudsen number throughout.
"""
from __future__ import annotations

from typing import Sequence

import mpmath as mp

from . import quadrature

_DPS = 60


def _roots(xk, wk):
    """The n-1 positive roots mu_i of sum_k w_k xi_k^2 / (1 - mu^2 xi_k^2) = 0 (xk > 0 ascending)."""
    def F(nu):
        return mp.fsum(w * x * x / (1 - nu * x * x) for x, w in zip(xk, wk))

    poles = sorted(1 / (x * x) for x in xk)  # ascending in nu = mu^2
    out = []
    for lo, hi in zip(poles[:-1], poles[1:]):
        eps = (hi - lo) * mp.mpf(10) ** (-40)
        a, b = lo + eps, hi - eps
        # F -> -inf just above a pole and +inf just below the next one: bisect, then polish.
        fa, fb = F(a), F(b)
        assert fa < 0 < fb
        for _ in range(200):
            m = (a + b) / 2
            if F(m) < 0:
                a = m
            else:
                b = m
        nu = mp.findroot(F, (a + b) / 2)
        out.append(mp.sqrt(nu))
    return out


def _positive_half(kind: str, n: int):
    """Positive nodes (ascending) and their weights of a xi_y rule, in mpmath."""
    if kind == "half":
        x, w = quadrature.half_range_mp(n)
        return list(x), list(w)
    if kind == "full":
        x, w = quadrature.full_range_mp(n)
        pairs = [(xi, wi) for xi, wi in zip(x, w) if xi > mp.mpf(10) ** (-30)]
        return [p[0] for p in pairs], [p[1] for p in pairs]
    raise ValueError(f"unknown rule kind {kind!r}")


class CouetteSolution:
    """Semi-analytic steady Couette solution for a xi_y rule: n nodes per half-line
    (kind "half", the default) or an n-node full-range rule (kind "full").

    Only the xi_y rule matters: the odd-in-xi_x part of f is linear in xi_x, so any
    xi_x rule that integrates xi_x^2 exactly gives the same solution."""

    def __init__(self, n_per_half: int, kn: float, u_w: float = 1.0, kind: str = "half"):
        with mp.workdps(_DPS):
            self.kn = mp.mpf(kn)
            self.u_w = mp.mpf(u_w)
            self.xk, self.wk = _positive_half(kind, n_per_half)   # positive nodes and weights
            self.mu = _roots(self.xk, self.wk)
            kn_ = self.kn
            # Unknowns: C, D_1..D_{m-1} (m positive nodes).  Conditions at y = 1/2 for the
            # arriving nodes -xi_k.
            n = len(self.xk)
            A = mp.matrix(n, n)
            rhs = mp.matrix(n, 1)
            for r, xpos in enumerate(self.xk):
                xi = -xpos
                A[r, 0] = mp.mpf(1) / 2 - kn_ * xi
                for i, mu in enumerate(self.mu):
                    # scaled by e^{-mu/(2Kn)} to keep the system well conditioned for small Kn
                    A[r, 1 + i] = 1 / (1 + mu * xi) - mp.exp(-mu / kn_) / (1 - mu * xi)
                rhs[r] = self.u_w
            sol = mp.lu_solve(A, rhs)
            self.C = sol[0]
            self.E = [sol[1 + i] for i in range(n - 1)]   # D_i = E_i e^{-mu_i/(2 Kn)}

    def _mode(self, i, y):
        mu, kn_ = self.mu[i], self.kn
        # 2 D_i sinh(mu y/Kn) with D_i = E_i e^{-mu/(2Kn)}
        return self.E[i] * (mp.exp(mu * (y - mp.mpf(1) / 2) / kn_) - mp.exp(-mu * (y + mp.mpf(1) / 2) / kn_))

    def u(self, y) -> float:
        """u_x at y in [-1/2, 1/2] (the face value at y = +-1/2)."""
        with mp.workdps(_DPS):
            y = mp.mpf(y)
            return float(self.C * y + mp.fsum(self._mode(i, y) for i in range(len(self.mu))))

    def pxy(self) -> float:
        """xy stress, uniform across the channel: -Kn C."""
        with mp.workdps(_DPS):
            return float(-self.kn * self.C)

    def B(self, y, xi_k) -> float:
        """Odd-in-xi_x amplitude of the population with xi_y = xi_k at y."""
        with mp.workdps(_DPS):
            y, xi = mp.mpf(y), mp.mpf(xi_k)
            s = self.C * (y - self.kn * xi)
            for i, mu in enumerate(self.mu):
                s += self.E[i] * (mp.exp(mu * (y - mp.mpf(1) / 2) / self.kn) / (1 + mu * xi)
                                  - mp.exp(-mu * (y + mp.mpf(1) / 2) / self.kn) / (1 - mu * xi))
            return float(s)


def free_molecular_pxy(u_w: float = 1.0) -> float:
    """Kn -> infinity: each plate's emission crosses the gap unchanged and
    p_xy = -2 u_w sum_{xi>0} w xi = -sqrt(2/pi) u_w, for any half-range set
    (the rule integrates xi on the half-line exactly: 1/sqrt(2 pi)).  A full-range
    rule gives -2 u_w sum_{xi>0} w xi with its own half-line sum."""
    return float(-mp.sqrt(2 / mp.pi) * u_w)


# ---------------------------------------------------------------------------
# The paper's printed closed form for 2 nodes per half (Eqs. 10-11).
# ---------------------------------------------------------------------------

def printed_eq10(y_over_l: float, kn_printed: float, u_w: float = 1.0,
                 a_num: float = 0.9494) -> float:
    """Eq. (10) exactly as printed (y measured from the mid-plane).  ``a_num`` is the
    argument constant of the first sinh in the numerator (printed 0.9494)."""
    k = kn_printed
    num = (mp.sinh(a_num / k) + 0.7978 * mp.cosh(0.9404 / k)) * y_over_l \
        + 0.5642 * k * mp.sinh(1.881 / k * y_over_l)
    den = (0.7071 * k + 0.3989) * mp.cosh(0.9404 / k) + (1.128 * k + 0.5) * mp.sinh(0.9404 / k)
    return float(u_w * num / den)


def printed_eq11(kn_printed: float, a_num: float = 0.9494) -> float:
    """Eq. (11) exactly as printed: sqrt(R T0) p_xy / (u_w p0)."""
    k = kn_printed
    num = mp.sinh(a_num / k) + 0.7979 * mp.cosh(0.9404 / k)
    den = (0.7071 * k + 0.3989) * mp.cosh(0.9404 / k) + (1.128 * k + 0.5) * mp.sinh(0.9404 / k)
    return float(-k * num / den)
