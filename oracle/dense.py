"""Steady state of the fully discrete scheme by a dense linear solve
(TEST INFRASTRUCTURE ONLY, see oracle/__init__.py).

The scheme is linear and homogeneous in f (the equilibrium of Eq. 5 in
weighted form is w_alpha (rho + xi_alpha . rho u), and the wall emission of
Eq. 8 is proportional to rho_w, itself linear in f by Eq. 9), so one step is
f^{n+1} = M f^n.  A steady state is a null vector of M - I; the total mass
(conserved by the scheme) fixes its scale.  This route shares nothing with the
time marching's stopping logic or residual, so it checks them.
"""
from __future__ import annotations

import numpy as np


def steady_state(problem, total_mass: float) -> np.ndarray:
    """Null vector of (M - I) scaled to the given total mass sum_cells rho.
    Requires a one-dimensional null space (a connected domain with walls)."""
    M = problem.step_matrix()
    n = M.shape[0]
    A = M - np.eye(n)
    _, s, vt = np.linalg.svd(A)
    if s[-1] > 1e-9 * s[0] or s[-2] < 1e-8 * s[0]:
        raise ValueError(f"null space is not one-dimensional (singular values {s[-2]:.3e}, {s[-1]:.3e})")
    v = vt[-1]
    f = v.reshape(problem.shape)
    return f * (total_mass / f.sum())
