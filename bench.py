#!/usr/bin/env python3
"""Benchmark of the finite-difference lattice Boltzmann hot path on one MI355X.

One benchmark step is one full time step of the method on the large cavity
(1024 x 1024 cells, 16 x 16 = 256 half-range velocities, Kn = 1, lid 0.01,
FP32 deviation storage with FP64 wall and residual sums): relaxation, wall
emission, upwind transport, moments, wall fluxes and the residual reduction.
The state is resident in HBM before timing starts.

Output: one JSON line on stdout (progress on stderr).  `value` is cell-velocity
updates per second.  `roofline` prices the fused step kernel against the HBM
peak using its algorithmic bytes (every population read once and written once,
plus the per-cell moments) and its own average duration from HIP events on the
library's stream.  Extra fields: the time to residual 1e-8 of the 128 x 128
cavity in FP32, mixed precision and plain FP64; the Couette time to 1e-10 in
FP64; the learned warm start (trained on 2000 solver-generated 64^2 cavities,
then warm versus uniform starts on held-out Kn at 128^2 and 256^2); the
64-cavity sweep (Kn log-uniform in [0.01, 10], N in {64..192}, 8^2 or 12^2
velocities) solved to 1e-8 as one mixed-precision batch, from uniform and from
warm starts, versus plain FP64 single-instance solves of the same cases; and
the measured copy bandwidth.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "cell·velocity updates/s (GB/s vs HBM peak); time to residual 1e-8 vs plain FP64"
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "step_kernel_cavity1024_q256_fp32_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1308_0692_amd", "csrc", "kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(per_launch_bytes_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; otherwise None."""
    try:
        d = json.load(open(PROFILE_TRAFFIC))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def eps_u(ux, uy, uxr, uyr):
    import numpy as np
    return float(np.hypot(ux - uxr, uy - uyr).max() / np.hypot(uxr, uyr).max())


def time_to_residual(F, W):
    """FP32, mixed and plain FP64 solves of the 128^2 cavity to R < 1e-8 and the Couette case
    to 1e-10.  The error of each cavity result is stated against the FP64 one."""
    out = {}
    c2 = W.C2
    ref = None
    for prec, graph, pseudo in (("fp64", True, False), ("fp64", False, False), ("fp32", True, False),
                                ("mixed", True, False), ("mixed", True, True), ("fp64", True, True)):
        p = F.Problem(c2, precision=prec)
        p.set_pseudo_time(pseudo)
        p.init_equilibrium()
        p.solve(1e-8, 400, check_every=200, use_graph=graph)  # warm-up (graph capture)
        p.init_equilibrium()
        rep = p.solve(1e-8, 200000, check_every=200, use_graph=graph)
        key = f"cavity128_q64_{prec}{'_pseudo' if pseudo else ''}{'_graph' if graph else ''}"
        rho, ux, uy, _ = p.moments()
        if ref is None:
            ref = (rho, ux, uy)
        out[key] = {"wall_s": round(rep["wall_s"], 4), "steps": rep["steps"], "steps_fp32": rep["steps_fp32"],
                    "first_below": rep["first_below"], "updates_per_s": rep["updates_per_s"],
                    "eps_u_vs_fp64": eps_u(ux, uy, ref[1], ref[2]),
                    "eps_rho_vs_fp64": float(abs(rho - ref[0]).max())}
        log(f"  {key}: {rep['wall_s']:.3f} s, {rep['steps']} steps ({rep['steps_fp32']} in float)")
        p.close()
    p = F.Problem(W.C1, precision="fp64")
    p.init_equilibrium()
    p.solve(1e-10, 200, check_every=100)
    p.init_equilibrium()
    rep = p.solve(1e-10, 200000, check_every=100)
    out["couette200_q24_fp64_graph"] = {"wall_s": round(rep["wall_s"], 4), "steps": rep["steps"],
                                        "first_below": rep["first_below"]}
    log(f"  couette: {rep['wall_s']:.3f} s, {rep['steps']} steps")
    p.close()
    return out


SOLO_STEPS = {}  # plain FP64 steps of every sweep instance, for the CPU extrapolation


def sweep_c3(F, W, torch, net=None):
    """The 64-cavity sweep to R < 1e-8: one mixed-precision batch (autotuned float tile,
    graph-captured chunks) against plain FP64 single-instance solves of the same cases, timed
    twice: with every instance's graph captured beforehand (outside the timing) and launched
    step by step without graphs.  Every result's error is stated against the instance's FP64
    solution continued to R < 1e-11 (untimed; the FP64 path equals the oracle to 1e-12 at equal
    step counts): per instance for the batch (and the warm-started batch), and for the plain
    FP64 solves stopped at 1e-8, whose own stopping error is of the same size.  With a trained
    warm-start network the batch is solved a second time from the network's seeds (seeding
    inside the timing).  Each is also solved with velocity-local pseudo-time steps (the same fixed
    point, reached in fewer iterations)."""
    cases = W.c3_instances()
    solo_wall, solo_steps, ref, solo_eps = 0.0, [], [], []
    for c in cases:
        p = F.Problem(c, precision="fp64")
        p.init_equilibrium()
        p.solve(1e-8, 400, check_every=200)  # graph capture
        p.init_equilibrium()
        rep = p.solve(1e-8, 200000, check_every=200)
        solo_wall += rep["wall_s"]
        solo_steps.append(rep["steps"])
        if rep["status"] != 0:
            raise RuntimeError(f"{c.name}: plain FP64 solve did not converge")
        at8 = p.moments()[:3]
        r11 = p.solve(1e-11, 2000000, check_every=500)
        if r11["status"] != 0:
            raise RuntimeError(f"{c.name}: FP64 reference did not reach 1e-11")
        ref.append(p.moments()[:3])
        solo_eps.append((eps_u(at8[1], at8[2], ref[-1][1], ref[-1][2]), float(abs(at8[0] - ref[-1][0]).max())))
        p.close()
    SOLO_STEPS["c3"] = solo_steps
    log(f"  plain FP64, one instance at a time: {solo_wall:.2f} s, {sum(solo_steps)} steps")
    nograph_wall = 0.0
    for c in cases:
        p = F.Problem(c, precision="fp64")
        p.init_equilibrium()
        rep = p.solve(1e-8, 200000, check_every=200, use_graph=False)
        nograph_wall += rep["wall_s"]
        p.close()
    log(f"  plain FP64 without graph capture: {nograph_wall:.2f} s")
    b = F.Batch(cases, precision="mixed")
    t0 = time.perf_counter()
    ms = b.autotune(steps=3)
    tune_s = time.perf_counter() - t0
    out = {"instances": len(cases), "tol": 1e-8, "reference": "each instance in FP64 continued to R < 1e-11",
           "plain_fp64_solo": {"wall_s": round(solo_wall, 3), "steps": sum(solo_steps),
                               "max_eps_u_vs_ref": max(e[0] for e in solo_eps),
                               "max_eps_rho_vs_ref": max(e[1] for e in solo_eps)},
           "plain_fp64_solo_no_graph": {"wall_s": round(nograph_wall, 3)}, "autotune_s": round(tune_s, 3)}
    for key in ("mixed_batch", "mixed_batch_pseudo", "mixed_batch_warm", "mixed_batch_warm_pseudo"):
        if "warm" in key and net is None:
            continue
        from paper_1308_0692_amd import warmstart
        b.set_pseudo_time("pseudo" in key)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, c in enumerate(cases):
            if "warm" not in key:
                b.init_equilibrium(i)
            else:
                warmstart.seed_batch(b, i, net, c.kn, c.wall_u[1])
        status, reps = b.solve(1e-8, 200000, check_every=200)
        wall = time.perf_counter() - t0
        eu, er = [], []
        for i in range(len(cases)):
            rho, ux, uy, _ = b.moments(i)
            eu.append(eps_u(ux, uy, ref[i][1], ref[i][2]))
            er.append(float(abs(rho - ref[i][0]).max()))
        steps = [r["steps"] for r in reps]
        f32 = [r["steps_fp32"] for r in reps]
        log(f"  {key}: {wall:.2f} s (status {status}), {sum(steps)} steps of which {sum(f32)} in float; "
            f"max eps_u vs the 1e-11 reference {max(eu):.2e}")
        out[key] = {"wall_s": round(wall, 3), "status": status, "steps": sum(steps),
                    "steps_fp32": sum(f32), "converged": sum(r["status"] == 0 for r in reps),
                    "tile": F.tile_describe("fp32", b.tile), "autotune_ms_per_step": round(ms, 4),
                    "max_eps_u_vs_ref": max(eu), "max_eps_rho_vs_ref": max(er),
                    "eps_u_vs_ref": [float(f"{v:.3e}") for v in eu],
                    "eps_rho_vs_ref": [float(f"{v:.3e}") for v in er],
                    "speedup_vs_plain_fp64": round(solo_wall / wall, 3),
                    "speedup_vs_plain_fp64_no_graph": round(nograph_wall / wall, 3)}
    b.close()
    return out


def kn_sweeps():
    """Model columns of the paper's Couette figures and cavity table from this solver: slip and
    p_xy / p_fm of Couette flow over Kn, and lid drag D and flow rate G of the cavity, for the
    half-range lattice D2Q^h_16 and the standard lattice D2Q_16 (definitions in
    paper_1308_0692_amd/sweeps.py; Kn of Eq. (1), the paper's is sqrt(2) times larger)."""
    from paper_1308_0692_amd import sweeps
    out = {"kn_convention": "Eq. (1); kn_printed = sqrt(2) kn", "couette": {}, "cavity": {}}
    kns = [0.01, 0.03, 0.1, 0.3, 1.0, 3.0, 10.0]
    t0 = time.perf_counter()
    for lat in ("D2Qh16", "D2Q16"):
        rows = sweeps.couette_sweep(kns, lattice=lat, ny=100, refine=True)
        out["couette"][lat] = [{"kn": r["kn"], "slip": round(r["slip"], 6),
                                "pxy_over_pfm": round(r["pxy_over_pfm"], 6)} for r in rows]
    for lat in ("D2Qh16", "D2Q16"):
        rows = sweeps.cavity_sweep([0.05, 0.1, 0.2, 0.4], lattice=lat, n=64, refine=True)
        out["cavity"][lat] = [{"kn": r["kn"], "D": round(r["D"], 5), "G": round(r["G"], 5),
                               "D_64": round(r["D_N"], 5), "G_64": round(r["G_N"], 5)} for r in rows]
    out["wall_s"] = round(time.perf_counter() - t0, 2)
    for lat in ("D2Qh16", "D2Q16"):
        c = {r["kn"]: r for r in out["couette"][lat]}
        log(f"  {lat}: Kn 0.1 slip {c[0.1]['slip']:.4f} p/p_fm {c[0.1]['pxy_over_pfm']:.4f}; "
            f"Kn 1 slip {c[1.0]['slip']:.4f} p/p_fm {c[1.0]['pxy_over_pfm']:.4f}")
    return out


def hybrid_channel(F):
    """The half-range / full-range hybrid (one workgroup per channel, state in LDS for a whole
    launch) on the Couette channel of 200 cells, 4 nodes per half in the layers x GH3 in x,
    Kn 0.1, plates at -+0.01, FP64, to R < 1e-10: with the layers filling the channel (the plain
    half-range scheme of the 24-velocity Couette workload), and with layers of 40 and 20 cells
    around a bulk on 4 or 3 full-range nodes (12 or 9 velocities instead of 24).  Then Kn sweeps
    of 1,024 channels (Kn log-spaced over [0.01, 10]) solved by one launch each.  Slip and
    stress are compared with the layers-filling solution of the same Kn."""
    import numpy as np
    out = {}
    base = dict(ny=200, kn=0.1, u_w=(-0.01, 0.01), n_half=4, qx=("full", 3))
    ref = None
    for name, layer, nf in (("layers_fill", 100, 4), ("layer40_bulk4", 40, 4), ("layer40_bulk3", 40, 3),
                            ("layer20_bulk4", 20, 4)):
        h = F.Hybrid([dict(base, layer=layer, n_full=nf)])
        h.init_all()
        h.solve(1e-10, 50)  # first launch (module load)
        h.init_all()
        code, reps = h.solve(1e-10, 400000)
        r = reps[0]
        f = h.faces(0)
        slip, pxy = 1.0 - f[2] / 0.01, f[3]
        if ref is None:
            ref = (slip, pxy)
        out[name] = {"wall_s": round(r["wall_s"], 5), "steps": r["steps"],
                     "us_per_step": round(r["wall_s"] / max(r["steps"], 1) * 1e6, 3),
                     "updates_per_step": h.info[0]["state_doubles"], "status": r["status"],
                     "slip": round(slip, 8), "pxy": pxy,
                     "slip_rel_vs_layers_fill": abs(slip / ref[0] - 1), "pxy_rel_vs_layers_fill": abs(pxy / ref[1] - 1)}
        log(f"  {name}: {r['steps']} steps in {r['wall_s'] * 1e3:.2f} ms "
            f"({out[name]['us_per_step']} us/step, {out[name]['updates_per_step']} updates/step), "
            f"slip {slip:.6f}, p_xy rel. to layers-fill {out[name]['pxy_rel_vs_layers_fill']:.1e}")
        h.close()
    kns = np.logspace(-2, 1, 1024)
    sweep_ref = None
    for name, layer in (("sweep1024_layers_fill", 100), ("sweep1024_layer40_bulk4", 40)):
        h = F.Hybrid([dict(base, kn=float(k), layer=layer, n_full=4) for k in kns])
        h.init_all()
        code, reps = h.solve(1e-10, 1_000_000)
        wall = reps[0]["wall_s"]
        upd = sum(h.info[i]["state_doubles"] * reps[i]["steps"] for i in range(h.n))
        pxy = np.array([h.faces(i)[3] for i in range(h.n)])
        if sweep_ref is None:
            sweep_ref = pxy
        out[name] = {"channels": h.n, "wall_s": round(wall, 4), "converged": int(sum(r["status"] == 0 for r in reps)),
                     "steps_max": int(max(r["steps"] for r in reps)), "updates": int(upd),
                     "updates_per_s": upd / wall, "pxy_rel_vs_layers_fill_max": float(np.abs(pxy / sweep_ref - 1).max())}
        log(f"  {name}: {h.n} channels in {wall:.3f} s ({upd / wall:.3e} updates/s), "
            f"max steps {out[name]['steps_max']}, p_xy rel. max {out[name]['pxy_rel_vs_layers_fill_max']:.1e}")
        h.close()
    return out


def copy_ceiling(F, torch, nbytes=4 << 30, reps=10):
    """Achievable streaming bandwidth on this device: the library's probes over 4 GiB, copies with
    each mix of plain / non-temporal loads and stores (the step kernels load plainly and store
    non-temporally), a pure read and a pure write.  GB/s counts the bytes moved (2 x nbytes for a
    copy)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    out = {}
    for mode in ("nt", "plain", "nt_load", "nt_store", "read", "write"):
        F.stream_probe(dst, src, nbytes, mode, s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            F.stream_probe(dst, src, nbytes, mode, s)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        moved = nbytes * (1 if mode in ("read", "write") else 2)
        out[mode] = round(moved / (ms * 1e-3) / 1e9, 1)
    del src, dst
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, W, target_s: float = 15.0):
    """The FP64 oracle as it stands, on the host cores: a bounded number of steps of the same
    workload on every core and on one core, the small cases solved to their tolerance, and the
    64-cavity sweep as the sum of its single-instance solves, extrapolated from a few timed
    steps per instance and the step counts of the library's plain FP64 solves."""
    from oracle import scheme
    P = scheme.Problem.from_case(case)
    f = P.equilibrium()
    t0 = time.perf_counter()
    f = P.step(f, 1)
    t1 = time.perf_counter() - t0
    n = max(1, min(50, int(target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    f = P.step(f, n)
    dt = time.perf_counter() - t0
    ups = case.nx * case.ny * P.q * n / dt
    cores = scheme.threads()
    out = {"value": ups, "unit": "cell-velocity updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} FP64 steps of the {case.nx}x{case.ny} cavity with {P.q} velocities "
                     f"(after 1 untimed step), {dt:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    try:
        scheme.set_threads(1)
        t0 = time.perf_counter()
        f = P.step(f, 1)
        dt1 = time.perf_counter() - t0
        out["value_1core"] = case.nx * case.ny * P.q / dt1
        out["ns_per_update_1core"] = round(dt1 / (case.nx * case.ny * P.q) * 1e9, 3)
    finally:
        scheme.set_threads(cores)
    del f
    ttr = {}
    for c, tol in ((W.C1, 1e-10), (W.C2, 1e-8)):
        Pc = scheme.Problem.from_case(c)
        t0 = time.perf_counter()
        _, steps, hist = Pc.solve(Pc.equilibrium(), tol, 400000)
        ttr[c.name] = {"tol": tol, "wall_s": round(time.perf_counter() - t0, 3), "steps": steps}
    out["time_to_residual"] = ttr
    solo = SOLO_STEPS.get("c3")
    if solo:
        total, sampled = 0.0, 0.0
        for c, steps in zip(W.c3_instances(), solo):
            Pc = scheme.Problem.from_case(c)
            f0 = Pc.equilibrium()
            k = max(2, int(2e8 // (c.nx * c.ny * Pc.q)))  # ~0.2 s of work per instance
            t0 = time.perf_counter()
            Pc.step(f0, k)
            d = time.perf_counter() - t0
            sampled += d
            total += d / k * steps
        out["sweep64_solo_extrapolated"] = {"wall_s": round(total, 1), "extrapolated": True,
                                            "timed_s": round(sampled, 2),
                                            "how": "oracle s/step of each instance x its plain FP64 step count"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--tile", type=int, default=-2, help="-2 autotune, -1 heuristic, >=0 a tile index")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-residual runs")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 64-cavity batch versus plain FP64 runs")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip training the warm-start network on 2000 solver-generated 64^2 cavities, the warm "
                         "versus uniform starts on held-out Kn at 128^2 and 256^2, and the warm-started sweep")
    ap.add_argument("--no-kn-sweeps", action="store_true", help="skip the Couette and cavity Kn sweeps")
    ap.add_argument("--no-hybrid", action="store_true", help="skip the hybrid half/full-range channel runs")
    ap.add_argument("--heldout", type=int, default=16)
    ap.add_argument("--tune-cache", default=None,
                    help="file caching autotuned tiles (default: the library's user cache file; '' disables)")
    ap.add_argument("--epochs", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the step is measured on one GPU's "
              "share of the work, and no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1308_0692_amd as F
    import workloads as W

    tune_cache = F.default_tune_cache() if args.tune_cache is None else args.tune_cache
    F.set_tune_cache(tune_cache)
    case = W.C4
    log(f"[bench] workload {case.name}: {case.nx}x{case.ny} cells, Q={case.q}, Kn={case.kn}")
    p = F.Problem(case, precision="fp32")
    tune_s = None
    if args.tile == -2:
        t0 = time.perf_counter()
        ms = p.autotune(steps=5)
        tune_s = time.perf_counter() - t0
        log(f"[bench] autotuned tile {p.tile} ({F.tile_describe('fp32', p.tile)}): {ms:.3f} ms/step "
            f"({tune_s:.2f} s of tuning; cache {tune_cache or 'off'})")
    elif args.tile >= 0:
        p.set_tile(args.tile)
    tile_index = p.tile
    tile_desc = F.tile_describe("fp32", tile_index)
    p.init_equilibrium()
    p.step(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warm-up {args.warmup} steps done; timing {args.steps}")

    s = p.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    ms_step_k, ms_red_k = p.step_timed(args.steps)
    e1.record(s)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    R, nsteps = p.last_residual()
    log(f"[bench] {args.steps} steps: {ms_total:.2f} ms events, {wall*1e3:.2f} ms wall; "
        f"step kernels {ms_step_k:.2f} ms, reductions {ms_red_k:.2f} ms; R={R:.3e}")

    cells = case.nx * case.ny
    q = p.q
    updates_per_step = cells * q
    ms_per_step = ms_total / args.steps
    value = updates_per_step * args.steps / (ms_total * 1e-3)
    # Algorithmic bytes of one step-kernel launch, in the measurement plan's convention: every
    # population read once and written once (4 B each) and the three moments of every cell read
    # and written once at 4 B; wall fluxes and partial sums (O(perimeter)) are left out.  The
    # kernel carries its moments in double (24 B more per cell, 0.1 B per update here): that
    # figure is reported beside it.
    alg_bytes = updates_per_step * 8 + cells * 6 * 4
    alg_bytes_fp64m = updates_per_step * 8 + cells * 6 * 8 + 2 * 4 * max(case.nx, case.ny) * 8
    avg_kernel_s = ms_step_k * 1e-3 / args.steps
    achieved = alg_bytes / avg_kernel_s / 1e9
    traffic = measured_traffic(alg_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "step_kernel", "alg_bytes_per_launch": alg_bytes,
                "bytes_convention": "8 B per update (FP32 population read + write) + 24 B per cell "
                                    "(three moments read + written at 4 B)",
                "alg_bytes_fp64_moments": alg_bytes_fp64m,
                "frac_fp64_moments": round(alg_bytes_fp64m / avg_kernel_s / 1e9 / HBM_PEAK_GBPS, 4),
                "avg_kernel_ms": round(avg_kernel_s * 1e3, 5)}
    log(f"[bench] {value:.4e} updates/s; step kernel {achieved:.0f} GB/s = {achieved/HBM_PEAK_GBPS:.3f} of peak")

    extra = {}

    def part(name, fn):
        """Run one extra measurement; a failure is reported in the line instead of ending the run."""
        try:
            return fn()
        except Exception as e:  # noqa: BLE001 - the headline must still print
            log(f"[bench] {name} failed: {e!r}")
            extra[name] = {"error": repr(e)}
            return None

    def large_cavity_fp64():
        # the same cavity with populations stored in double (twice the bytes per update)
        p64 = F.Problem(case, precision="fp64")
        p64.autotune(steps=3)
        p64.init_equilibrium()
        p64.step(5)
        k64, _ = p64.step_timed(50)
        b64 = updates_per_step * 16 + cells * 6 * 8 + 2 * 4 * max(case.nx, case.ny) * 8
        extra["large_cavity_fp64"] = {"updates_per_s": updates_per_step * 50 / (k64 * 1e-3),
                                      "step_kernel_ms": round(k64 / 50, 5),
                                      "alg_GBps": round(b64 / (k64 / 50 * 1e-3) / 1e9, 1),
                                      "tile": F.tile_describe("fp64", p64.tile)}
        log(f"[bench] same cavity in FP64: step kernel {k64 / 50:.3f} ms "
            f"({extra['large_cavity_fp64']['alg_GBps']} GB/s)")
        p64.close()

    part("large_cavity_fp64", large_cavity_fp64)
    if not args.no_copy:
        def copy():
            probes = copy_ceiling(F, torch)
            extra["copy_GBps"] = probes["nt"]
            extra["stream_probes_GBps"] = probes
            roofline["ceiling_streaming_GBps"] = max(probes.values())
            roofline["frac_of_ceiling"] = round(achieved / max(probes.values()), 4)
            log(f"[bench] streaming probes (GB/s): {probes}")
        part("copy_GBps", copy)
    if not args.no_ttr:
        log("[bench] time to residual:")
        r = part("time_to_residual", lambda: time_to_residual(F, W))
        if r is not None:
            extra["time_to_residual"] = r
    p.close()
    net = None
    if not args.no_warm_start:
        def warm():
            from paper_1308_0692_amd import warmstart
            log("[bench] learned warm start:")
            train_kn = W.c5_training_kn()
            res = warmstart.experiment(train_kn, W.c5_heldout_kn(args.heldout, training=train_kn),
                                       epochs=args.epochs, log=lambda m: log(m))
            trained = res.pop("net")
            extra["warm_start"] = res
            return trained
        net = part("warm_start", warm)
    if not args.no_sweep:
        log("[bench] 64-cavity sweep to 1e-8:")
        r = part("sweep64", lambda: sweep_c3(F, W, torch, net))
        if r is not None:
            extra["sweep64"] = r
    if not args.no_kn_sweeps:
        log("[bench] Kn sweeps (Couette slip and stress, cavity D and G):")
        r = part("kn_sweeps", kn_sweeps)
        if r is not None:
            extra["kn_sweeps"] = r

    if not args.no_hybrid:
        log("[bench] hybrid half-range / full-range channel:")
        r = part("hybrid_channel", lambda: hybrid_channel(F))
        if r is not None:
            extra["hybrid_channel"] = r

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu = part("cpu_baseline", lambda: cpu_baseline(case, W))
        failed = extra.pop("cpu_baseline", None)
        if cpu is None:
            cpu = failed
        else:
            log(f"[bench] oracle: {cpu['value']:.3e} updates/s on {cpu['cores']} threads")

    line = {"metric": METRIC, "value": value, "unit": "cell-velocity updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": case.name, "nx": case.nx, "ny": case.ny, "q": q, "kn": case.kn,
                       "lid_u": case.wall_u[1], "velocities": "half-range Gauss-Hermite 8 per half, tensor",
                       "tile": tile_desc, "tile_index": tile_index,
                       "autotune_s": None if tune_s is None else round(tune_s, 3), "tune_cache": bool(tune_cache)},
            "roofline": roofline, "cpu_baseline": cpu, **extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
