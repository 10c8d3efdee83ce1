"""Knudsen-number sweeps of the paper's two flows, solved as batches on the GPU.

Couette flow (plates at y = 0 and 1 sliding at -u_w and +u_w): the slip at the plate and the
shear stress against the free-molecular value, the quantities of the paper's Couette figures,
for a half-range lattice (the paper's method) or the standard full-range one.  Lid-driven
cavity: the drag on the lid and the recirculating flow rate through the vertical mid-line, the
quantities of the paper's cavity table, and the mid-line velocity profile.  Couette flow on the
half-range / full-range hybrid that the paper proposes (the library's fdlb_hybrid_* channels).

Conventions (all in the units of Eq. (1); Kn is Eq. (1)'s Knudsen number):
  slip          1 - u_t(wall) / u_w at the upper plate, u_t the tangential velocity of the face
                state (arriving populations from the wall cell, leaving ones from Eq. (8))
  p_fm          free-molecular shear stress of the continuous model, -sqrt(2/pi) u_w (the
                paper prints the same quantity with Kn and stress in units that differ by sqrt 2:
                its Kn is sqrt(2) times this one, reported as ``kn_printed``)
  D             drag on the lid: -(1/u_w) times the mean over the lid's faces of the face xy
                stress (the tangential force per unit lid length; > 0)
  G             recirculating flow rate: (1/u_w) times the integral over the vertical mid-line
                of |u_x| (the net flux through the line is zero at steady state, so this is twice
                the flow carried each way); on an even grid the mid-line is the average of
                columns N/2 - 1, N/2
The paper's own definitions of D and G are in a cited work it does not reproduce, so these are
stated here rather than taken from it.

First-order grid convergence: with ``refine`` every case is also solved on the doubled grid and
the Richardson value 2 v(2N) - v(N) is reported beside the values of both grids.
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import BOTTOM, TOP, Batch

Rule = Tuple[str, int]

#: Named lattices: (x rule, y rule).  The paper's D2Q^h_16 is two nodes per half-line on each
#: axis; its standard lattice D2Q_16 is the four-node full-range rule on each axis.
LATTICES: Dict[str, Tuple[Rule, Rule]] = {
    "D2Qh16": (("half", 2), ("half", 2)),
    "D2Qh64": (("half", 4), ("half", 4)),
    "D2Q16": (("full", 4), ("full", 4)),
    "D2Q36": (("full", 6), ("full", 6)),
    "D2Q64": (("full", 8), ("full", 8)),
}


def lattice_rules(lattice) -> Tuple[Rule, Rule]:
    """A name of LATTICES, or an explicit ((kind, n), (kind, n)) pair of x and y rules."""
    if isinstance(lattice, str):
        try:
            return LATTICES[lattice]
        except KeyError:
            raise ValueError(f"unknown lattice {lattice!r}; known: {sorted(LATTICES)}") from None
    qx, qy = lattice
    return (str(qx[0]), int(qx[1])), (str(qy[0]), int(qy[1]))


def p_free_molecular(u_w: float = 1.0) -> float:
    """Free-molecular shear stress between plates at -u_w and +u_w (Eq. 1 units)."""
    return -math.sqrt(2.0 / math.pi) * u_w


class _Case:
    """Inputs of one problem in the form the batch takes (duck-typed like workloads.Case)."""

    def __init__(self, nx, ny, periodic_x, periodic_y, wall_u, kn, qx, qy, cfl=0.9):
        self.nx, self.ny = nx, ny
        self.periodic_x, self.periodic_y = periodic_x, periodic_y
        self.wall_u = tuple(wall_u)
        self.kn = kn
        self.qx, self.qy = qx, qy
        self.cfl = cfl
        self.lx = self.ly = 1.0


def _solve(cases: Sequence[_Case], precision, tol, max_steps, check_every, device, autotune):
    b = Batch(cases, precision=precision, device=device)
    if autotune:
        b.autotune(steps=2)
    for i in range(len(cases)):
        b.init_equilibrium(i)
    status, reps = b.solve(tol, max_steps, check_every=check_every)
    bad = [i for i, r in enumerate(reps) if r["status"] != 0]
    if bad:
        raise RuntimeError(f"sweep members {bad} did not converge to {tol:g} "
                           f"(status {[reps[i]['status'] for i in bad]})")
    return b, reps


def _richardson(rows: List[dict], keys: Iterable[str]):
    for r in rows:
        for k in keys:
            r[k] = 2.0 * r[k + "_2N"] - r[k + "_N"]


def couette_sweep(kns: Sequence[float], lattice="D2Qh16", ny: int = 100, refine: bool = True,
                  u_w: float = 0.01, precision: str = "fp64", tol: float = 1e-11,
                  max_steps: int = 4_000_000, check_every: int = 500, device="cuda:0") -> List[dict]:
    """Slip and shear stress of planar Couette flow for every Kn, one batch for all of them.

    Per Kn: ``slip`` and ``pxy_over_pfm`` (Richardson values when ``refine``, else those of the
    ny grid), the values of each grid (``*_N``, ``*_2N``), the steps taken and ``kn_printed``."""
    (qx, qy) = lattice_rules(lattice)
    grids = [ny, 2 * ny] if refine else [ny]
    cases = [_Case(1, n, True, False, (-u_w, u_w, 0.0, 0.0), float(kn), qx, qy) for n in grids for kn in kns]
    b, reps = _solve(cases, precision, tol, max_steps, check_every, device, autotune=False)
    pfm = p_free_molecular(u_w)
    rows = []
    for j, kn in enumerate(kns):
        row = {"kn": float(kn), "kn_printed": math.sqrt(2.0) * float(kn)}
        for g, tag in zip(range(len(grids)), ("_N", "_2N")):
            i = g * len(kns) + j
            _, ut, pw = b.wall_profile(i, TOP)
            row["slip" + tag] = 1.0 - float(ut[0]) / u_w
            row["pxy_over_pfm" + tag] = float(pw[0]) / pfm
            row["steps" + tag] = int(reps[i]["steps"])
        rows.append(row)
    if refine:
        _richardson(rows, ("slip", "pxy_over_pfm"))
    else:
        for r in rows:
            r["slip"], r["pxy_over_pfm"] = r["slip_N"], r["pxy_over_pfm_N"]
    b.close()
    return rows


def _midline(a: np.ndarray) -> np.ndarray:
    n = a.shape[1]
    return 0.5 * (a[:, n // 2 - 1] + a[:, n // 2]) if n % 2 == 0 else a[:, n // 2]


def cavity_sweep(kns: Sequence[float], lattice="D2Qh16", n: int = 64, refine: bool = False,
                 u_w: float = 0.01, precision: str = "mixed", tol: float = 1e-8,
                 max_steps: int = 4_000_000, check_every: int = 200, device="cuda:0",
                 autotune: bool = True) -> List[dict]:
    """Drag on the lid and recirculating flow rate of the lid-driven cavity for every Kn, one
    batch for all of them.  Per Kn: ``D``, ``G`` (Richardson values when ``refine``), the values
    of each grid, the mid-line profile ``u_mid`` (u_x / u_w at the cell centres of the n grid,
    bottom to top) and the steps taken."""
    (qx, qy) = lattice_rules(lattice)
    grids = [n, 2 * n] if refine else [n]
    cases = [_Case(m, m, False, False, (0.0, u_w, 0.0, 0.0), float(kn), qx, qy) for m in grids for kn in kns]
    b, reps = _solve(cases, precision, tol, max_steps, check_every, device, autotune)
    rows = []
    for j, kn in enumerate(kns):
        row = {"kn": float(kn), "kn_printed": math.sqrt(2.0) * float(kn)}
        for g, tag in zip(range(len(grids)), ("_N", "_2N")):
            i = g * len(kns) + j
            m = grids[g]
            _, _, pw = b.wall_profile(i, TOP)
            _, ux, _, _ = b.moments(i)
            mid = _midline(ux) / u_w
            row["D" + tag] = -float(np.mean(pw)) / u_w
            row["G" + tag] = float(np.sum(np.abs(mid)) / m)
            row["steps" + tag] = int(reps[i]["steps"])
            if g == 0:
                row["u_mid"] = mid.tolist()
        rows.append(row)
    if refine:
        _richardson(rows, ("D", "G"))
    else:
        for r in rows:
            r["D"], r["G"] = r["D_N"], r["G_N"]
    b.close()
    return rows


def hybrid_couette_sweep(kns: Sequence[float], delta: float = 0.2, ny: int = 200, n_half: int = 4,
                         n_full: Optional[int] = None, qx: Rule = ("full", 3), refine: bool = True,
                         u_w: float = 0.01, tol: float = 1e-12, max_steps: int = 4_000_000,
                         device="cuda:0") -> List[dict]:
    """Couette flow on the half-range / full-range hybrid (layers of thickness ``delta`` next to
    the plates on ``n_half`` nodes per half-line, the bulk on ``n_full`` full-range nodes), every
    Kn and grid one channel of a single hybrid launch.

    Per Kn: ``slip`` and ``pxy_over_pfm`` at the upper plate (Richardson values from ny and 2 ny
    cells when ``refine``), ``defect`` = the relative difference of the momentum flux through the
    upper interface as the bulk and the layer see it (the coupling's conservation defect; 0
    without a bulk), the values of each grid and the steps taken."""
    from . import Hybrid
    if n_full is None:
        n_full = n_half
    grids = [ny, 2 * ny] if refine else [ny]
    chans = [dict(ny=n, layer=max(1, int(round(delta * n))), kn=float(kn), u_w=(-u_w, u_w), n_half=n_half,
                  n_full=n_full, qx=qx) for n in grids for kn in kns]
    h = Hybrid(chans, device=device)
    h.init_all()
    code, reps = h.solve(tol, max_steps)
    bad = [i for i, r in enumerate(reps) if r["status"] != 0]
    if bad:
        h.close()
        raise RuntimeError(f"hybrid channels {bad} did not converge to {tol:g}")
    pfm = p_free_molecular(u_w)
    rows = []
    for j, kn in enumerate(kns):
        row = {"kn": float(kn), "kn_printed": math.sqrt(2.0) * float(kn)}
        for g, tag in zip(range(len(grids)), ("_N", "_2N")):
            i = g * len(kns) + j
            f = h.faces(i)
            row["slip" + tag] = 1.0 - float(f[2]) / u_w
            row["pxy_over_pfm" + tag] = float(f[3]) / pfm
            row["defect" + tag] = 0.0 if math.isnan(f[6]) else abs(float(f[6]) / float(f[7]) - 1.0)
            row["steps" + tag] = int(reps[i]["steps"])
        rows.append(row)
    if refine:
        _richardson(rows, ("slip", "pxy_over_pfm", "defect"))
    else:
        for r in rows:
            r["slip"], r["pxy_over_pfm"], r["defect"] = r["slip_N"], r["pxy_over_pfm_N"], r["defect_N"]
    h.close()
    return rows
