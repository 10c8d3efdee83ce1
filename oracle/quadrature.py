"""Gauss-Hermite velocity quadratures, computed in high precision (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper (Eq. 4 and Table I) weighs velocities with
omega(xi) = (2 pi)^(-d/2) exp(-xi^2/2).  A half-range rule with n nodes per
half-line is the n-point Gauss rule for that weight restricted to [0, inf),
mirrored onto (-inf, 0]; the full-range rule is the ordinary Gauss rule for
the weight on the whole line (probabilists' Hermite roots).  Two-dimensional
sets are tensor products (text after Table I).

Method used here (kept deliberately different from the library's):
  1. exact moments m_k of the weight, as closed forms in mpmath;
  2. Chebyshev's algorithm: moments -> three-term recurrence of the monic
     orthogonal polynomials;
  3. nodes = eigenvalues of the Jacobi matrix (mpmath eigsy);
  4. weights from the definition of an interpolatory rule: solve the
     Vandermonde system sum_i w_i x_i^k = m_k, k < n, in high precision.
Exactness for degrees n .. 2n-1 is then a property the tests check, not an
input.
"""
from __future__ import annotations

from functools import lru_cache
from typing import Tuple

import mpmath as mp
import numpy as np

_DPS = 80


def half_moment(k: int):
    """m_k = int_0^inf xi^k (2 pi)^(-1/2) exp(-xi^2/2) dxi = 2^((k-1)/2) Gamma((k+1)/2) / sqrt(2 pi)."""
    return mp.power(2, mp.mpf(k - 1) / 2) * mp.gamma(mp.mpf(k + 1) / 2) / mp.sqrt(2 * mp.pi)


def full_moment(k: int):
    """Moments of the normalised Gaussian on the whole line: (k-1)!! for even k, 0 for odd k."""
    if k % 2:
        return mp.mpf(0)
    return mp.fac2(k - 1) if k > 0 else mp.mpf(1)


def _chebyshev(moments, n):
    """Chebyshev's algorithm: recurrence coefficients (a_k, b_k), k < n, of the monic
    polynomials orthogonal for the measure with the given 2n moments."""
    sig_prev = [mp.mpf(0)] * (2 * n)
    sig = [moments[l] for l in range(2 * n)]
    a = [moments[1] / moments[0]]
    b = [moments[0]]
    for k in range(1, n):
        sig_new = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            sig_new[l] = sig[l + 1] - a[k - 1] * sig[l] - b[k - 1] * sig_prev[l]
        a.append(sig_new[k + 1] / sig_new[k] - sig[k] / sig[k - 1])
        b.append(sig_new[k] / sig[k - 1])
        sig_prev, sig = sig, sig_new
    return a, b


def _gauss(moment, n):
    with mp.workdps(_DPS):
        m = [moment(k) for k in range(2 * n)]
        a, b = _chebyshev(m, n)
        J = mp.matrix(n, n)
        for i in range(n):
            J[i, i] = a[i]
            if i + 1 < n:
                J[i, i + 1] = J[i + 1, i] = mp.sqrt(b[i + 1])
        evals, _ = mp.eigsy(J)
        x = sorted(evals[i] for i in range(n))
        V = mp.matrix(n, n)
        for k in range(n):
            for i in range(n):
                V[k, i] = x[i] ** k
        w = mp.lu_solve(V, mp.matrix(m[:n]))
        return x, [w[i] for i in range(n)]


@lru_cache(maxsize=None)
def half_range_mp(n: int):
    """Nodes (ascending, positive) and weights of the n-point rule on [0, inf), in mpmath."""
    if not 1 <= n <= 16:
        raise ValueError("half-range order must be in 1..16 nodes per half")
    return _gauss(half_moment, n)


@lru_cache(maxsize=None)
def full_range_mp(n: int):
    """Nodes (ascending) and weights of the n-point full-range Gauss-Hermite rule, in mpmath."""
    if not 1 <= n <= 32:
        raise ValueError("full-range order must be in 1..32 nodes")
    return _gauss(full_moment, n)


def half_range(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Mirrored half-range rule: 2n nodes ascending (-xi_n..-xi_1, xi_1..xi_n), weights summing to 1."""
    x, w = half_range_mp(n)
    nodes = [-v for v in reversed(x)] + list(x)
    weights = list(reversed(w)) + list(w)
    return (np.array([float(v) for v in nodes]), np.array([float(v) for v in weights]))


def full_range(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Full-range rule: n nodes ascending, weights summing to 1."""
    x, w = full_range_mp(n)
    # The weight is even, so the rule is symmetric: impose it exactly (an odd n has
    # the node 0, which must come out as 0 and not as a rounding residue).
    xs = [(x[i] - x[n - 1 - i]) / 2 for i in range(n)]
    ws = [(w[i] + w[n - 1 - i]) / 2 for i in range(n)]
    return np.array([float(v) for v in xs]), np.array([float(v) for v in ws])


def rule(kind: str, n: int) -> Tuple[np.ndarray, np.ndarray]:
    if kind == "half":
        return half_range(n)
    if kind == "full":
        return full_range(n)
    raise ValueError(f"unknown quadrature kind {kind!r}")


def velocity_set(qx: Tuple[str, int], qy: Tuple[str, int]):
    """Tensor-product set (text after Table I): xi_alpha = (xi_i, xi_j), w_alpha = w_i w_j,
    ordered alpha = j * Q_x + i (x index fastest), 1-D nodes ascending."""
    x, wx = rule(*qx)
    y, wy = rule(*qy)
    xi_x = np.tile(x, len(y))
    xi_y = np.repeat(y, len(x))
    w = np.repeat(wy, len(x)) * np.tile(wx, len(y))
    return xi_x, xi_y, w
