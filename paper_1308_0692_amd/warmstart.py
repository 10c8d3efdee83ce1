"""Learned warm start of steady solves (fdlb_mlp_* and fdlb_field_samples).

The solver generates its own training data: a batch of cavities with Knudsen numbers
spread over the range of interest is solved to the tolerance, and every cell of every
solution becomes a sample (inputs: encoded log10 Kn and cell centre; targets: the fields
scaled by the lid speed).  The network is trained with Adam on shuffled minibatches.  A new
problem is then seeded at equilibrium with the predicted fields (mass renormalised) and
solved as usual: the solver decides convergence, the network only moves the start.

Marshalling only: solves, sample extraction, forward, backward and Adam run in the
library's kernels; numpy draws the shuffling permutations.
"""
from __future__ import annotations

import math
import time
from typing import Iterable, Optional

import numpy as np

from . import Batch, Mlp, Problem, _lib


def cavity_desc(n: int, kn: float, u_w: float = 0.01, order: int = 4, precision: str = "mixed",
                cfl: float = 0.9) -> _lib.ProblemDesc:
    """Lid-driven square cavity: lid (top wall) moving at +u_w, the other walls at rest."""
    return _lib.make_desc(n, n, False, False, (0.0, u_w, 0.0, 0.0), kn, ("half", order), ("half", order), cfl,
                          precision)


def generate(kns: Iterable[float], n: int = 64, order: int = 4, u_w: float = 0.01, tol: float = 1e-8,
             precision: str = "mixed", check_every: int = 200, max_steps: int = 400000, device="cuda:0",
             autotune: bool = True, pseudo: bool = True):
    """Solve one cavity per Kn (as one batch) and return (inputs, targets, reports): device
    float32 tensors of shape (len(kns) n^2, 3) and the per-instance solve reports.  autotune:
    time the compiled tile shapes on the batch first (a few steps each; the built-in choice is
    made for single problems).  pseudo: iterate with velocity-local pseudo-time steps (the same
    steady states in fewer steps)."""
    import torch
    kns = [float(k) for k in kns]
    descs = [cavity_desc(n, kn, u_w, order, precision) for kn in kns]
    b = Batch(None, descs=descs, device=device)
    b.set_pseudo_time(pseudo)
    t0 = time.perf_counter()
    if autotune:
        b.autotune(steps=3)  # leaves every member at rest
    tune_s = time.perf_counter() - t0
    if not autotune:
        for i in range(len(kns)):
            b.init_equilibrium(i)
    t0 = time.perf_counter()
    status, reps = b.solve(tol, max_steps, check_every=check_every)
    wall = time.perf_counter() - t0
    cells = n * n
    X = torch.empty((len(kns) * cells, 3), dtype=torch.float32, device=device)
    T = torch.empty_like(X)
    for i in range(len(kns)):
        b.field_samples(i, X[i * cells:(i + 1) * cells], T[i * cells:(i + 1) * cells])
    torch.cuda.synchronize(device)
    b.close()
    return X, T, {"status": status, "wall_s": wall, "autotune_s": tune_s, "reports": reps}


def train(net: Mlp, X, T, epochs: int, batch: int, lr: float = 3e-3, lr_final: float = 1e-5, seed: int = 0,
          log=None):
    """Adam on shuffled minibatches with a cosine decay of the learning rate from lr to lr_final.
    Returns the last minibatch loss of every epoch."""
    import torch
    N = X.shape[0]
    if batch > net.max_batch:
        raise ValueError("batch exceeds the network's max_batch")
    # minibatch order: a permutation per epoch drawn on the device (a host permutation of millions
    # of samples, and its copy, would cost more than the epoch's training steps)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(int(seed))
    steps = epochs * math.ceil(N / batch)
    s = 0
    losses = []
    per_epoch = math.ceil(N / batch)
    for e in range(epochs):
        perm = torch.randperm(N, generator=gen, device=X.device).to(torch.int32)
        # one call per epoch: the minibatch loop (backward, Adam) runs behind the C ABI
        fracs = (s + np.arange(per_epoch)) / max(1, steps - 1)
        net.train_steps(X, T, perm, batch, lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * fracs)))
        s += per_epoch
        losses.append(net.last_loss())
        if log and (e % max(1, epochs // 10) == 0 or e == epochs - 1):
            log(f"epoch {e}: minibatch loss {losses[-1]:.3e}")
    return losses


def evaluate(net: Mlp, X, T) -> float:
    """Mean squared error over all samples (in chunks of the network's max_batch)."""
    N = X.shape[0]
    tot = 0.0
    for k in range(0, N, net.max_batch):
        m = min(net.max_batch, N - k)
        net.backward(X[k:k + m], T[k:k + m])
        tot += net.last_loss() * m
    return tot / N


def seed(p: Problem, net: Mlp, kn: float, u_w: float):
    """Seed problem p at equilibrium with the predicted fields (mass renormalised)."""
    rho, ux, uy = net.predict_fields(kn, p.nx, p.ny, u_w)
    p.init_equilibrium_dev(rho, ux, uy, renormalize=True)


def seed_batch(b: Batch, i: int, net: Mlp, kn: float, u_w: float):
    nx, ny = b.shapes[i]
    rho, ux, uy = net.predict_fields(kn, nx, ny, u_w)
    b.init_equilibrium_dev(i, rho, ux, uy, renormalize=True)


def _eps(a, b):
    """(eps_u, eps_rho) of fields a = (rho, ux, uy) against b."""
    eu = float(np.hypot(a[1] - b[1], a[2] - b[2]).max() / np.hypot(b[1], b[2]).max())
    return eu, float(np.abs(a[0] - b[0]).max())


def experiment(train_kn, heldout_kn, train_n: int = 64, order: int = 4, u_w: float = 0.01, grids=(128, 256),
               epochs: int = 20, batch: int = 8192, lr: float = 3e-3, tol: float = 1e-8, precision: str = "mixed",
               ref_tol: float = 1e-11, seed_value: int = 0, log=print):
    """Train on solver-generated cavities, then compare warm and uniform starts on held-out Kn.

    For every held-out Kn and grid: steps and wall time to `tol` from the uniform start and
    from the network's seed (prediction and seeding included in the warm wall time), and the
    error of both final states against an FP64 solve of the same problem to `ref_tol`."""
    import torch
    out = {"train_count": len(train_kn), "train_n": train_n, "order": order, "epochs": epochs, "batch": batch}
    t0 = time.perf_counter()
    X, T, info = generate(train_kn, n=train_n, order=order, u_w=u_w, tol=tol, precision=precision)
    out["generate_s"] = round(time.perf_counter() - t0, 3)
    out["generate_solve_s"] = round(info["wall_s"], 3)
    out["generate_autotune_s"] = round(info["autotune_s"], 3)
    out["generate_pseudo_time"] = True
    out["generate_steps_max"] = int(max(r["steps"] for r in info["reports"]))
    out["samples"] = int(X.shape[0])
    log(f"  generated {X.shape[0]} samples from {len(train_kn)} solves in {out['generate_s']:.1f} s "
        f"(tile autotune {info['autotune_s']:.1f} s, solve {info['wall_s']:.1f} s)")
    net = Mlp(hidden=4, max_batch=batch, seed=seed_value)
    t0 = time.perf_counter()
    losses = train(net, X, T, epochs=epochs, batch=batch, lr=lr, seed=seed_value, log=log)
    torch.cuda.synchronize()
    out["train_s"] = round(time.perf_counter() - t0, 3)
    out["train_steps"] = epochs * math.ceil(X.shape[0] / batch)
    out["final_loss"] = evaluate(net, X, T)
    log(f"  trained {out['train_steps']} Adam steps in {out['train_s']:.1f} s; loss {out['final_loss']:.3e}")
    del X, T
    rows = []
    for n in grids:
        for kn in heldout_kn:
            kn = float(kn)
            p = Problem(desc=cavity_desc(n, kn, u_w, order, precision))
            p.init_equilibrium()
            p.solve(tol, 400, check_every=200)  # graph capture outside the timing
            p.init_equilibrium()
            cold = p.solve(tol, 2000000, check_every=200)
            cold_f = p.moments()[:3]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            seed(p, net, kn, u_w)
            warm = p.solve(tol, 2000000, check_every=200)
            warm_wall = time.perf_counter() - t0
            warm_f = p.moments()[:3]
            p.close()
            r = Problem(desc=cavity_desc(n, kn, u_w, order, "fp64"))
            r.init_equilibrium()
            ref = r.solve(ref_tol, 4000000, check_every=500)
            ref_f = r.moments()[:3]
            r.close()
            ec, ew = _eps(cold_f, ref_f), _eps(warm_f, ref_f)
            row = {"n": n, "kn": kn, "cold_steps": cold["steps"], "warm_steps": warm["steps"],
                   "cold_s": round(cold["wall_s"], 4), "warm_s": round(warm_wall, 4),
                   "cold_eps_u": ec[0], "warm_eps_u": ew[0], "cold_eps_rho": ec[1], "warm_eps_rho": ew[1],
                   "ref_status": ref["status"], "status": [cold["status"], warm["status"]]}
            rows.append(row)
            log(f"  {n}^2 Kn {kn:.4f}: uniform {cold['steps']} steps {cold['wall_s']:.3f} s, warm {warm['steps']} "
                f"steps {warm_wall:.3f} s; eps_u vs FP64 {ec[0]:.1e} / {ew[0]:.1e}")
    out["heldout"] = rows
    for n in grids:
        sel = [r for r in rows if r["n"] == n]
        out[f"grid{n}"] = {"cold_steps": sum(r["cold_steps"] for r in sel), "warm_steps": sum(r["warm_steps"] for r in sel),
                           "cold_s": round(sum(r["cold_s"] for r in sel), 3),
                           "warm_s": round(sum(r["warm_s"] for r in sel), 3),
                           "max_warm_eps_u": max(r["warm_eps_u"] for r in sel),
                           "max_cold_eps_u": max(r["cold_eps_u"] for r in sel)}
    out["net"] = net
    return out
