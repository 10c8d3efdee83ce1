"""Test oracle for the finite-difference lattice Boltzmann method (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
the benchmark's CPU-baseline leg may import, call, link or run anything in
this directory.  The GPU library never does, and this directory never
imports the GPU library: the two share no code, only the seeded input
generators of ``workloads.py``.

Contents
--------
quadrature.py  half-range and full-range Gauss-Hermite rules from exact moments (mpmath)
fdlb_oracle.c  the fully discrete scheme on raw populations, plain C, FP64
scheme.py      ctypes driver of fdlb_oracle.c, problem setup, moments and wall profiles
couette.py     semi-analytic steady Couette solution of the discrete-velocity model
               and the paper's printed closed form (Eqs. 10-11)
hybrid.py      half-range layers coupled to a full-range bulk in the Couette channel:
               the fully discrete scheme (numpy) and its semi-analytic steady solution
dense.py       steady state by a dense null-space solve on tiny grids
mlp.py         FP64 forward/backward/Adam of the warm-start network
build.py       compiles fdlb_oracle.c with gcc

Parity status: every function here is pinned by tests against facts the paper
or mathematics fixes (printed Table I, closed-form moments, closed-form
relaxation and transport responses, the residual of every step in closed form
for free-molecular flow on a periodic box, conservation with half- and
full-range walls, free-molecular Couette, convergence to the semi-analytic
Couette solution for half- and full-range rules, the printed Eqs. 10-11,
symmetries, grid self-convergence of the cavity, dense solves; for the hybrid:
polynomial exactness and Lagrange interpolation of the interface maps, equality
with the plain scheme when the layers fill the channel, the rest state,
momentum conservation inside each zone, first-order convergence to the
semi-analytic solution of the coupling and its exponential approach to the
pure half-range solution).  The figure curves are parity unpinned (their
reference solvers are not in the paper); the drag and flow rate of Table II
are defined by this project (the paper cites their definitions), and the GPU
sweep is held to the printed table within 3 %.
"""
