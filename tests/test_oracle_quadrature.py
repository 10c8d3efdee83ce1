"""Pins of the oracle's velocity quadrature (Eq. 4, Table I, text after Table I)."""
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_half_range.txt")


def _table1():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        n, x, w = line.split()
        rows.append((int(n), x, w))
    return rows


def _half_ulp_of_print(s: str) -> float:
    decimals = len(s.split(".")[1]) if "." in s else 0
    return 0.5 * 10.0 ** (-decimals)


def test_table1_printed_digits():
    """Every printed node and weight of Table I is reproduced to the printed digit."""
    rows = _table1()
    assert len(rows) == 9
    for n in (2, 3, 4):
        x, w = quadrature.half_range(n)
        mine = [(xi, wi) for xi, wi in zip(x[n:], w[n:])]
        printed = [(xs, ws) for (nn, xs, ws) in rows if nn == n]
        assert len(printed) == n
        for (xi, wi), (xs, ws) in zip(mine, printed):
            assert abs(xi - float(xs)) <= _half_ulp_of_print(xs) * 1.0001, (n, xi, xs)
            assert abs(wi - float(ws)) <= _half_ulp_of_print(ws) * 1.0001, (n, wi, ws)


def _exact_half_moment(k):
    # int_0^inf xi^k exp(-xi^2/2) dxi / sqrt(2 pi): even k -> (k-1)!!/2, odd k -> 2^((k-1)/2) ((k-1)/2)! / sqrt(2 pi)
    if k % 2 == 0:
        return float(mp.fac2(k - 1) / 2) if k > 0 else 0.5
    j = (k - 1) // 2
    return float(mp.mpf(2) ** j * mp.factorial(j) / mp.sqrt(2 * mp.pi))


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_half_range_gauss_exactness(n):
    """An n-point Gauss rule on the half-line is exact for degree <= 2n-1 (and not 2n)."""
    x, w = quadrature.half_range(n)
    xp, wp = x[n:], w[n:]
    assert np.all(xp > 0) and np.all(np.diff(xp) > 0)
    assert np.allclose(x[:n], -xp[::-1], rtol=0, atol=0)
    for k in range(2 * n):
        got = math.fsum(wp * xp ** k)
        want = _exact_half_moment(k)
        assert abs(got - want) <= 2e-14 * want * (1 + k), (n, k, got, want)
    # degree 2n is not integrated exactly by a Gauss rule (checked at 80 digits)
    with mp.workdps(80):
        xm, wm = quadrature.half_range_mp(n)
        got = mp.fsum(wi * xi ** (2 * n) for xi, wi in zip(xm, wm))
        want = quadrature.half_moment(2 * n)
        assert abs(got - want) > mp.mpf(10) ** -30 * want


@pytest.mark.parametrize("n", [2, 4, 6, 8, 16])
def test_half_range_normalisation(n):
    """Eq. (4) normalisation on the whole line: sum w = 1, sum w xi = 0, sum w xi^2 = 1,
    and the half-range flux sum_{xi>0} w xi = (2 pi)^(-1/2) used by Eq. (9)."""
    x, w = quadrature.half_range(n)
    assert abs(math.fsum(w) - 1) < 1e-15
    assert abs(math.fsum(w * x)) < 1e-16
    assert abs(math.fsum(w * x * x) - 1) < 1e-14
    assert abs(math.fsum((w * x)[x > 0]) * math.sqrt(2 * math.pi) - 1) < 1e-15


def test_full_range_gh3_textbook():
    x, w = quadrature.full_range(3)
    assert x[1] == 0.0
    assert np.allclose(x, [-math.sqrt(3), 0, math.sqrt(3)], rtol=1e-15, atol=0)
    assert np.allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 12, 16, 20])
def test_full_range_matches_numpy_hermegauss(n):
    xr, wr = np.polynomial.hermite_e.hermegauss(n)
    wr = wr / math.sqrt(2 * math.pi)
    x, w = quadrature.full_range(n)
    assert np.allclose(x, xr, rtol=1e-13, atol=1e-14)
    assert np.allclose(w, wr, rtol=1e-11, atol=1e-300)


def test_tensor_product_and_ordering():
    xi_x, xi_y, w = quadrature.velocity_set(("full", 3), ("half", 4))
    assert len(w) == 24
    x, wx = quadrature.full_range(3)
    y, wy = quadrature.half_range(4)
    for a in range(24):
        i, j = a % 3, a // 3
        assert xi_x[a] == x[i] and xi_y[a] == y[j]
        assert w[a] == wy[j] * wx[i]
    assert abs(w.sum() - 1) < 1e-15
    assert abs((w * xi_x * xi_y).sum()) < 1e-16


def test_invalid_orders():
    with pytest.raises(ValueError):
        quadrature.half_range(0)
    with pytest.raises(ValueError):
        quadrature.half_range(17)
    with pytest.raises(ValueError):
        quadrature.full_range(33)
