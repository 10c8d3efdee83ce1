"""Python driver of the C oracle (TEST INFRASTRUCTURE ONLY, see oracle/__init__.py).

Sets up a problem exactly as the paper's method needs it — velocity set from
``oracle.quadrature``, cell-centred grid on the unit square (l = 1), time
step from the Courant number, omega = dt / Kn — and calls ``fdlb_oracle.c``.

Time step (reading; the paper gives none): the unsplit two-dimensional donor
cell is stable for  dt * max_alpha(|xi_x| N_x + |xi_y| N_y) <= 1,  so
dt = CFL / max_alpha(|xi_x| N_x [x active] + |xi_y| N_y [y active]), where an
axis is active unless it is periodic with a single cell (then transport along
it vanishes identically).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

from . import quadrature
from .build import LIB, build

BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3


class _CProblem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("q", C.c_int32), ("order", C.c_int32),
        ("wall_u", C.c_double * 4),
        ("dt", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
        ("omega", C.c_double),
        ("xi_x", C.POINTER(C.c_double)), ("xi_y", C.POINTER(C.c_double)),
        ("w", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build(force=False)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(_CProblem)
        L.oracle_moments.argtypes = [pp, dp, dp, dp, dp]
        L.oracle_step.argtypes = [pp, dp, dp, dp]
        L.oracle_work_doubles.argtypes = [pp]
        L.oracle_work_doubles.restype = C.c_size_t
        L.oracle_solve.argtypes = [pp, dp, C.c_int64, C.c_double, dp]
        L.oracle_solve.restype = C.c_int64
        L.oracle_pxy.argtypes = [pp, dp, dp]
        L.oracle_wall_profile.argtypes = [pp, dp, C.c_int, dp, dp, dp]
        L.oracle_wall_profile.restype = C.c_int
        L.oracle_equilibrium.argtypes = [pp, dp, dp, dp, dp]
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Problem:
    """A discretised boundary-value problem on an l_x x l_y rectangle (the unit square by
    default; lengths in units of the length l that defines Kn)."""

    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    wall_u: Tuple[float, float, float, float]
    kn: float
    qx: Tuple[str, int]
    qy: Tuple[str, int]
    cfl: float = 0.9
    order: int = 0           # 0: relax then transport, 1: transport then relax
    dt_override: Optional[float] = None
    lx: float = 1.0          # domain lengths in units of the length of Kn
    ly: float = 1.0

    def __post_init__(self):
        self.xi_x, self.xi_y, self.w = quadrature.velocity_set(self.qx, self.qy)
        self.q = len(self.w)
        self.dx = self.lx / self.nx
        self.dy = self.ly / self.ny
        ax = 0.0 if (self.periodic_x and self.nx == 1) else 1.0
        ay = 0.0 if (self.periodic_y and self.ny == 1) else 1.0
        speed = np.max(np.abs(self.xi_x) * (self.nx / self.lx) * ax + np.abs(self.xi_y) * (self.ny / self.ly) * ay)
        self.dt = float(self.dt_override) if self.dt_override is not None else self.cfl / float(speed)
        self.omega = 0.0 if math.isinf(self.kn) else self.dt / self.kn
        self._keep = [np.ascontiguousarray(a, dtype=np.float64) for a in (self.xi_x, self.xi_y, self.w)]
        self._c = _CProblem(self.nx, self.ny, int(self.periodic_x), int(self.periodic_y), self.q,
                            self.order, (C.c_double * 4)(*self.wall_u), self.dt, self.dx, self.dy,
                            self.omega, _dp(self._keep[0]), _dp(self._keep[1]), _dp(self._keep[2]))

    @classmethod
    def from_case(cls, case, **kw) -> "Problem":
        kw.setdefault("lx", getattr(case, "lx", 1.0))
        kw.setdefault("ly", getattr(case, "ly", 1.0))
        return cls(case.nx, case.ny, case.periodic_x, case.periodic_y, tuple(case.wall_u), case.kn,
                   tuple(case.qx), tuple(case.qy), case.cfl, **kw)

    @property
    def shape(self):
        return (self.q, self.ny, self.nx)

    # -- state construction ------------------------------------------------
    def equilibrium(self, rho=None, ux=None, uy=None, renormalize: bool = False) -> np.ndarray:
        """f_alpha = w_alpha rho (1 + xi_alpha . u) (Eqs. 3, 5); rho = 1 and u = 0 by default.
        With renormalize, rho is scaled so that its sum over cells is nx * ny."""
        cells = (self.ny, self.nx)
        rho = np.ones(cells) if rho is None else np.array(rho, dtype=np.float64).reshape(cells)
        ux = np.zeros(cells) if ux is None else np.array(ux, dtype=np.float64).reshape(cells)
        uy = np.zeros(cells) if uy is None else np.array(uy, dtype=np.float64).reshape(cells)
        if renormalize:
            rho = rho * (self.nx * self.ny / rho.sum())
        f = np.empty(self.shape)
        lib().oracle_equilibrium(C.byref(self._c), _dp(np.ascontiguousarray(rho)),
                                 _dp(np.ascontiguousarray(ux)), _dp(np.ascontiguousarray(uy)), _dp(f))
        return f

    # -- time marching -------------------------------------------------------
    def step(self, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
        """f after nsteps steps (input untouched)."""
        out = np.array(f, dtype=np.float64, order="C", copy=True)
        n = lib().oracle_solve(C.byref(self._c), _dp(out), int(nsteps), 0.0, None)
        if n != nsteps:
            raise MemoryError("oracle allocation failed")
        return out

    def solve(self, f: np.ndarray, tol: float, max_steps: int):
        """March until the per-step residual R = ||u^{n+1}-u^n|| / ||u^{n+1}|| drops below tol.
        Returns (f, steps taken, residual history)."""
        out = np.array(f, dtype=np.float64, order="C", copy=True)
        hist = np.zeros(int(max_steps))
        n = lib().oracle_solve(C.byref(self._c), _dp(out), int(max_steps), float(tol), _dp(hist))
        if n < 0:
            raise MemoryError("oracle allocation failed")
        return out, int(n), hist[:n]

    # -- outputs ---------------------------------------------------------------
    def moments(self, f: np.ndarray):
        """Density and velocity per cell (Eqs. 6-7), arrays of shape (ny, nx)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho, ux, uy = (np.empty((self.ny, self.nx)) for _ in range(3))
        lib().oracle_moments(C.byref(self._c), _dp(f), _dp(rho), _dp(ux), _dp(uy))
        return rho, ux, uy

    def pxy(self, f: np.ndarray) -> np.ndarray:
        """xy stress of the post-relaxation state per cell."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.empty((self.ny, self.nx))
        lib().oracle_pxy(C.byref(self._c), _dp(f), _dp(out))
        return out

    def wall_profile(self, f: np.ndarray, wall: int):
        """(rho, u_t, p_xy) of the face state along a wall (post-relaxation, Eq. 8 emission)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        n = self.nx if wall in (BOTTOM, TOP) else self.ny
        r, u, p = np.empty(n), np.empty(n), np.empty(n)
        if lib().oracle_wall_profile(C.byref(self._c), _dp(f), int(wall), _dp(r), _dp(u), _dp(p)) != 0:
            raise ValueError("wall not present")
        return r, u, p

    def step_matrix(self) -> np.ndarray:
        """The one-step map as a dense matrix (the scheme is linear and homogeneous in f);
        only for tiny problems."""
        n = self.q * self.nx * self.ny
        if n > 4096:
            raise ValueError("step_matrix is for tiny problems")
        # Columns as differences around the rest state: the relaxation divides by rho,
        # so a bare unit vector (rho = 0 in most cells) is not a valid input, while
        # linearity makes step(base + e_k) - step(base) the k-th column.
        base = self.equilibrium()
        s0 = self.step(base, 1).ravel()
        M = np.empty((n, n))
        for k in range(n):
            e = base.ravel().copy()
            e[k] += 1.0
            M[:, k] = self.step(e.reshape(self.shape), 1).ravel() - s0
        return M


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the number in effect."""
    return int(lib().oracle_set_threads(int(n)))
