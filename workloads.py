"""Seeded synthetic workloads for the finite-difference lattice Boltzmann solver.

This module is shared by the test oracle and by the GPU library's callers
(tests, benchmark).  It defines problem *inputs* only — grid sizes, Knudsen
numbers, wall speeds, velocity-set orders, random draws — and holds none of
the method's arithmetic (no quadrature, no equilibrium, no transport).

The paper's two boundary-value problems are fully defined by geometry, Kn,
the wall speed and the velocity set (planar Couette flow between plates at
distance l moving at -u_w / +u_w with periodic ends; square lid-driven cavity
with the top wall sliding at +u_w), so no dataset stands behind them: every
input here is synthetic and seeded.

Velocity sets are named by the number of nodes per half-line for half-range
Gauss-Hermite rules ("half", n) — the paper's D1Q^h_{2n} — and by the total
node count for full-range rules ("full", n).
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Optional, Tuple

import numpy as np

# Wall indices used throughout: tangential speed of each wall.  Bottom/top
# walls slide along +x, left/right walls along +y.
BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3


@dataclass(frozen=True)
class Case:
    """One boundary-value problem instance (inputs only)."""

    name: str
    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    wall_u: Tuple[float, float, float, float]  # bottom, top, left, right
    kn: float                                   # Kn of the kinetic equation's own definition; inf allowed
    qx: Tuple[str, int]                         # ("half", n per half) or ("full", n)
    qy: Tuple[str, int]
    cfl: float = 0.9
    tol: float = 1e-8
    precision: str = "fp32"                     # "fp32" (deviation storage) or "fp64"
    lx: float = 1.0                             # domain lengths in units of the length of Kn
    ly: float = 1.0

    @property
    def q(self) -> int:
        def cnt(r):
            return 2 * r[1] if r[0] == "half" else r[1]
        return cnt(self.qx) * cnt(self.qy)

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def couette(ny: int = 200, kn: float = 0.1, u_w: float = 0.01,
            qy: Tuple[str, int] = ("half", 4), qx: Tuple[str, int] = ("full", 3),
            **kw) -> Case:
    """Planar Couette flow: plates at y=0 (speed -u_w) and y=1 (+u_w), x periodic with one cell."""
    return Case(name=kw.pop("name", f"couette{ny}"), nx=1, ny=ny, periodic_x=True,
                periodic_y=False, wall_u=(-u_w, u_w, 0.0, 0.0), kn=kn, qx=qx, qy=qy, **kw)


def couette_x(nx: int = 200, kn: float = 0.1, u_w: float = 0.01,
              qx: Tuple[str, int] = ("half", 4), qy: Tuple[str, int] = ("full", 3),
              **kw) -> Case:
    """Couette flow turned by 90 degrees: plates at x=0 (speed -u_w along y) and x=1 (+u_w)."""
    return Case(name=kw.pop("name", f"couettex{nx}"), nx=nx, ny=1, periodic_x=False,
                periodic_y=True, wall_u=(0.0, 0.0, -u_w, u_w), kn=kn, qx=qx, qy=qy, **kw)


def cavity(n: int = 128, kn: float = 0.1, u_w: float = 0.01, order: int = 4,
           ny: Optional[int] = None, **kw) -> Case:
    """Lid-driven cavity: all walls fixed except the top one, which slides at +u_w along x."""
    return Case(name=kw.pop("name", f"cavity{n}"), nx=n, ny=(ny or n), periodic_x=False,
                periodic_y=False, wall_u=(0.0, u_w, 0.0, 0.0), kn=kn,
                qx=("half", order), qy=("half", order), **kw)


# ---------------------------------------------------------------------------
# The five named workloads.
# ---------------------------------------------------------------------------

#: Couette, 4 nodes per half in xi_y x 3-node full-range rule in xi_x (24 velocities),
#: 200 cells, Kn = 0.1, plates at -/+0.01, FP64, stepped to residual 1e-10.
C1 = couette(200, kn=0.1, u_w=0.01, qy=("half", 4), qx=("full", 3), tol=1e-10,
             precision="fp64", name="couette200_q24_fp64")

#: Lid-driven cavity 128 x 128, 8 x 8 = 64 velocities, Kn = 0.1, lid 0.01, to residual 1e-8.
C2 = cavity(128, kn=0.1, u_w=0.01, order=4, tol=1e-8, name="cavity128_q64")

#: Large cavity 1024 x 1024, 16 x 16 = 256 velocities, Kn = 1, lid 0.01, FP32 state.
C4 = cavity(1024, kn=1.0, u_w=0.01, order=8, tol=1e-8, name="cavity1024_q256_fp32")


def c3_instances(count: int = 64, seed: int = 13080692) -> List[Case]:
    """Batched sweep: Kn log-uniform in [0.01, 10], N from {64, 96, 128, 192},
    half-range order 4 or 6 per half; draws taken per instance in the order Kn, N, order."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kn = float(10.0 ** rng.uniform(-2.0, 1.0))
        n = int(rng.choice([64, 96, 128, 192]))
        order = int(rng.choice([4, 6]))
        out.append(cavity(n, kn=kn, u_w=0.01, order=order, tol=1e-8, name=f"batch{i:02d}"))
    return out


def c5_training_kn(count: int = 2000, seed: int = 1308) -> np.ndarray:
    """Knudsen numbers of the warm-start training cavities (log-uniform in [0.01, 10])."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-2.0, 1.0, size=count)


def c5_heldout_kn(count: int = 16, seed: int = 692, training: Optional[np.ndarray] = None,
                  min_rel_gap: float = 0.001) -> np.ndarray:
    """Held-out Knudsen numbers, rejecting draws within 0.1 % of any training value (2,000
    log-uniform training values are ~0.35 % apart on average, so a wider exclusion would
    leave only the few widest gaps)."""
    rng = np.random.default_rng(seed)
    train = np.asarray(training if training is not None else c5_training_kn())
    out: List[float] = []
    while len(out) < count:
        kn = 10.0 ** rng.uniform(-2.0, 1.0)
        if np.min(np.abs(train - kn) / kn) > min_rel_gap:
            out.append(kn)
    return np.asarray(out)


# ---------------------------------------------------------------------------
# Seeded perturbations for parity tests (plain random numbers, no physics).
# ---------------------------------------------------------------------------

def random_fields(nx: int, ny: int, seed: int, amp: float = 1e-2):
    """Smooth-ish random macroscopic fields: rho = 1 + amp*r0, ux = amp*r1, uy = amp*r2,
    arrays of shape (ny, nx), float64."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(-1.0, 1.0, size=(3, ny, nx))
    return 1.0 + amp * r[0], amp * r[1], amp * r[2]


def random_noise(q: int, nx: int, ny: int, seed: int) -> np.ndarray:
    """Uniform noise in [-1, 1] of shape (q, ny, nx), float64 (population index first)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(q, ny, nx))


def with_(case: Case, **kw) -> Case:
    """Copy of a case with some fields replaced."""
    return replace(case, **kw)


# ---------------------------------------------------------------------------
# Warm-start network: seeded parameters and samples (inputs only; no arithmetic of the method).
# ---------------------------------------------------------------------------

def mlp_params(seed: int, width: int = 128, hidden: int = 4, scale: float = 1.0) -> np.ndarray:
    """Flat parameter vector, layer by layer (W row-major by output, then b): weights uniform in
    +-scale*sqrt(6 / (fan_in + fan_out)), biases uniform in +-0.1."""
    rng = np.random.default_rng(seed)
    shapes = [(width, 3)] + [(width, width)] * (hidden - 1) + [(3, width)]
    parts = []
    for o, i in shapes:
        lim = scale * np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(rng.uniform(-0.1, 0.1, size=o))
    return np.concatenate(parts)


def mlp_samples(n: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Encoded inputs in [-1, 1]^3 and smooth targets of order one, shape (n, 3) each."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(n, 3))
    t = np.stack([np.sin(2 * a[:, 1]) * a[:, 0], a[:, 2] ** 2 - 0.3, np.cos(a[:, 0] + a[:, 1])], axis=1)
    return a, t


def random_cases(count: int, seed: int) -> List[Case]:
    """Seeded assorted problems for broad parity checks: grids 2..70 (or a periodic single cell on
    one axis), half-range rules of 2..5 nodes per half on bounded axes (walls need them) and half-
    or full-range rules (full: 2..6 nodes) on a periodic axis, Kn log-uniform in [0.02, 50] or
    infinite, every wall speed in [-0.02, 0.02], domain lengths in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = int(rng.integers(0, 3))  # 0 box, 1 periodic x, 2 periodic y
        nx = 1 if kind == 1 else int(rng.integers(2, 71))
        ny = 1 if kind == 2 else int(rng.integers(2, 71))

        def rule(axis_periodic: bool):
            if not axis_periodic or rng.random() < 0.5:
                return ("half", int(rng.integers(2, 6)))
            return ("full", int(rng.integers(2, 7)))

        qx, qy = rule(kind == 1), rule(kind == 2)
        kn = float("inf") if rng.random() < 0.1 else float(10.0 ** rng.uniform(np.log10(0.02), np.log10(50.0)))
        wall = tuple(float(v) for v in rng.uniform(-0.02, 0.02, size=4))
        out.append(Case(name=f"random{i:02d}", nx=nx, ny=ny, periodic_x=kind == 1, periodic_y=kind == 2,
                        wall_u=wall, kn=kn, qx=qx, qy=qy, lx=float(rng.uniform(0.5, 2.0)),
                        ly=float(rng.uniform(0.5, 2.0))))
    return out
