#!/usr/bin/env python3
"""Benchmark: implicit VET radiation step, cell-updates/s at 256^3, mixed precision vs FP64.

Workload: the mixed-depth medium at 256^3 (lognormal density sigma 1.5, cell optical depth
log-uniform over 1e-3..1e3 and spatially correlated, random SPD unit-trace Eddington tensor,
central Gaussian source in E, T = 0.1, dt = 50 light-crossing times, open (characteristic outflow)
faces, FP32-exact inputs), 5 implicit steps.  The default run adds two legs as extra keys: the 512^3
scale recipe (mixed path, 1 warm-up + 3 steps) and the batched path (1024 blocks, 1 warm-up + 1 step).  A "step" is one rad_step call (the whole hot path: coefficient
setup, Picard iterations of FP64 residual, Krylov solve, exchange solve, commit).

The timed region starts with every input resident in HBM.  Both paths start from the same
initial state.  Printed: one JSON line with the mixed-path throughput as `value`, the FP64
path's throughput and the speedup, the error between the two and the oracle's residual of
the mixed result, the roofline of the dominant kernel measured live with HIP events, and the
FP64 CPU oracle timed on a bounded sample of the same recipe.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "implicit VET rad-step cell-updates/s at 256^3; mixed vs FP64 speedup"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_code_objects(torch, rad, p, state, coefs, dt, dx, bc, n=16):
    """One untimed rad_step on an n^3 corner of the workload.  The runtime loads a source file's kernels on
    the first launch of one of them; without this the load lands inside the event-timed warm-up step (about
    15 ms, in the class launched first: the coefficient setup)."""
    cut = lambda t: t[..., :n, :n, :n].contiguous()
    E, F, T = (cut(t) for t in state)
    ws = rad.alloc_workspace(rad.workspace_bytes(E.shape, p))
    w0 = time.perf_counter()
    rad.rad_step(E, F, T, *(cut(t) for t in coefs), dt, dx, bc, p, workspace=ws, check=False)
    torch.cuda.synchronize()
    log(f"  code objects loaded by a {n}^3 step ({1000 * (time.perf_counter() - w0):.0f} ms)")


def run_path(torch, rad, d, state0, coefs, prec, steps, warmup, tol, profile, m=30, autotune=None, eps_R=1e-2,
             poly=1):
    """Warm up, restore the initial state, then time `steps` consecutive rad_step calls.  autotune:
    None, "tiles" (tune the stencil z-ranges) or "all" (also the restart length), outside the timing."""
    E, F, T = (t.clone() for t in state0)
    rho, kP, kR, f = coefs
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], prec=prec, tol=tol, gmres_m=m, eps_R=eps_R, krylov_poly=poly)
    p.coef_dtype = 1 if rho.dtype == torch.float32 else 0
    ws = rad.alloc_workspace(rad.workspace_bytes(E.shape, p))
    tuned = None
    if autotune:
        tuned = rad.autotune_step(E, F, T, rho, kP, kR, f, d["dt"], d["dx"], d["bc"], p,
                                  tune_restart=autotune == "all", workspace=ws)
        log(f"  [{prec}] autotune: {tuned}")
        p.gmres_m = tuned["gmres_m"]
        p.krylov_poly = tuned["krylov_poly"]
    share = None
    if profile and warmup > 0:
        load_code_objects(torch, rad, p, (E, F, T), coefs, d["dt"], d["dx"], d["bc"])
    for s in range(warmup):
        # the last warm-up step (from the same initial state as timed step 0) times every kernel class
        full = profile and s == warmup - 1
        if full:
            rad.profile(True)
            rad.profile_reset()
            torch.cuda.synchronize()
            w0 = time.perf_counter()
        st = rad.rad_step(E, F, T, rho, kP, kR, f, d["dt"], d["dx"], d["bc"], p, workspace=ws, check=False)
        if full:
            torch.cuda.synchronize()
            share = dict(seconds=time.perf_counter() - w0, profile=rad.profile_read())
            rad.profile(False)
        log(f"  [{prec}] warmup step {s}: {st['picard_iters']} Picard, {st['krylov_iters']} Krylov, "
            f"{st['t_total_ms']:.0f} ms, res {st['scaled_residual']:.2e}")
    for dst, src in zip((E, F, T), state0):
        dst.copy_(src)
    prev = None
    stats = []
    # timed steps: events around the operator applies only (the roofline's kernel)
    rad.profile(2 if profile else False)
    rad.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        if s == steps - 1:
            prev = (E.clone(), F.clone(), T.clone())
        st = rad.rad_step(E, F, T, rho, kP, kR, f, d["dt"], d["dx"], d["bc"], p, workspace=ws, check=False)
        stats.append(st)
        log(f"  [{prec}] step {s}: rc {st['rc']}, {st['picard_iters']} Picard, {st['krylov_iters']} Krylov, "
            f"{st['refine_sweeps']} FP64 residuals, {st['t_total_ms']:.0f} ms, res {st['scaled_residual']:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = rad.profile_read() if profile else {}
    rad.profile(False)
    del ws
    return dict(seconds=t1 - t0, stats=stats, state=(E, F, T), prev=prev, profile=prof, tuned=tuned, share=share)


def measured_traffic(kernel_class, n):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy) of one library kernel
    class, from the committed rocprofv3 counter summary of the n^3 mixed step, or None when there is none or
    the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_mixed_{n}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = b"".join(open(os.path.join(ROOT, "paper_2202_08778_amd", "csrc", f), "rb").read()
                   for f in ("rad_single.hip", "rad_device.h", "rad_apply_tiled.h", "rad_amr.h"))
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    k = rec.get("classes", {}).get(kernel_class)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def relerr(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cpu_baseline(n_sample, tol, n_full):
    """FP64 oracle on the same recipe at n_sample^3, one step, timed on the host cores; with the time the
    oracle would take for one n_full^3 step at the sample's per-cell rate (a lower bound: its Krylov count
    grows with the grid)."""
    import oracle
    from paper_2202_08778_amd import workloads as W
    d = W.mixed_depth(n=n_sample, seed=3, steps=1, fp32_exact=True)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                       cv=d["cv"])
    t0 = time.perf_counter()
    _, _, _, st = P.step(d["E"], d["F"], d["T"], tol=tol, allow_unconverged=True)
    sec = time.perf_counter() - t0
    cells = n_sample ** 3
    return {"value": cells / sec, "unit": "cell-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"mixed-depth recipe at {n_sample}^3 (same generator, {d['bc']} faces, FP32-exact), 1 step, "
                      f"tol {tol:g}: {sec:.1f} s, {st['picard_iters']} Picard / {st['krylov_iters']} Krylov "
                      f"iterations, converged={st['converged']}",
            "extrapolated_seconds_per_step": {f"{n_full}^3": n_full ** 3 / (cells / sec),
                                              "note": "sample rate per cell; a lower bound (Krylov counts grow "
                                                      "with the grid)"}}


def bench_batched(args, torch, np, rad, W, steps=None, warmup=None, emit=True):
    """The batched path: 1024 independent Dirichlet blocks (edges 8..32, per-block dt and kappa), mixed
    precision, one persistent launch per step replayed from a HIP graph, inputs restored before each step.
    emit: print the JSON line (a run of its own); else return the result (a leg of the default run)."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    batch = W.batched_blocks(nblocks=1024, seed=4)
    descs, ar = rad.pack_blocks(batch["blocks"])
    cells = sum(b["n"] ** 3 for b in batch["blocks"])
    p = rad.params(prec="mixed", tol=args.tol, coef_dtype=1, krylov_poly=1 if args.krylov_poly == 2 else args.krylov_poly,
                   eps_R=args.eps_r)
    # GMRES(48): the stiff blocks that GMRES(12) leaves unconverged although the oracle solves them converge
    p.gmres_m = args.gmres_m if (args.gmres_m is not None and args.batched) else 48
    g = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt).cuda()
    dev = [g(ar["E"]), g(ar["F"]), g(ar["T"])] + [g(ar[k], torch.float32) for k in ("rho", "kP", "kR", "f")]
    init = [t.clone() for t in dev[:3]]
    plan = rad.Plan(descs, p)
    if args.autotune:
        log("autotuning the batched launch shape ...")
        plan.autotune(*dev)
    stats = None
    times = []
    for s in range(warmup + steps):
        for t, t0 in zip(dev[:3], init):
            t.copy_(t0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = plan.step(*dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if s >= warmup:
            times.append(dt)
        log(f"  [batched] {'warmup ' if s < warmup else ''}step {s}: {1000 * dt:.0f} ms")
        if s == warmup - 1 and args.reorder:
            plan.reorder(stats)   # queue the timed steps by the warm-up step's block solve times
            log("  [batched] queue reordered by measured block solve times")
    st = rad.Plan.read_stats(stats)
    sec = sum(times)
    conv = int((st["status"] == 0).sum())
    res = {"metric": "batched implicit VET rad-step cell-updates/s (1024 AMR-like blocks, mixed precision)",
           "value": cells * steps / sec, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": 1000.0 * sec / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "1024 Dirichlet blocks, edges uniform on {8,12,16,24,32}, dt 1..1000 crossings, "
                                  "kappa 1e-2..1e3 per block, one persistent graph-replayed launch per step",
                      "cells": cells, "gmres_m": p.gmres_m, "krylov_poly": p.krylov_poly, "eps_R": p.eps_R,
                      "queue": ("longest measured solve first (warm-up step's block times)"
                                if warmup > 0 and args.reorder else "largest block first"),
                      "launch": dict(zip(("threads", "per_cu", "largest_first"), plan.launch_shape()))},
           "blocks_converged": conv, "blocks": len(batch["blocks"]),
           "krylov_iters_max_block": int(st["krylov_iters"].max()),
           "krylov_iters_total": int(st["krylov_iters"].sum()),
           "block_solve_ms_max": float(st["t_total_ms"].max()),
           "block_solve_ms_sum": float(st["t_total_ms"].sum())}
    # chip busy fraction: the blocks' summed workgroup time over (workgroups x step time)
    shape = plan.launch_shape()
    wgs = shape[1] * torch.cuda.get_device_properties(0).multi_processor_count
    res["chip_busy_fraction"] = float(st["t_total_ms"].sum()) / (wgs * res["ms_per_step"])
    del plan, dev, init
    if not emit:
        return res
    print(json.dumps(res), flush=True)


def amr_cpu_baseline(tol):
    """The composite oracle on a bounded two-level sample of the same recipe, one step, on the host cores."""
    from oracle.amr import TwoLevel
    from paper_2202_08778_amd import workloads as W
    d = W.two_level((10, 10, 10), (3, 3, 3), (7, 7, 7), seed=6, fp32_exact=True)
    pb = TwoLevel(d["nc"], d["lo"], d["hi"], d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"])
    t0 = time.perf_counter()
    _, _, _, st = pb.step(d["E"], d["F"], d["T"], tol=tol)
    sec = time.perf_counter() - t0
    leaf = pb.N - int(pb.covered.sum())
    return {"value": leaf / sec, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"two-level recipe, coarse 10^3 with the box 3..7 refined (fine 8^3, {leaf} leaf cells), 1 step, "
                      f"tol {tol:g}: {sec:.1f} s, {st['picard_iters']} Newton iterations with sparse direct solves "
                      f"(numpy/scipy, one thread for the solves)"}


def bench_amr(args, torch, np, rad, W):
    """The two-level AMR grid: coarse n^3 with the central box [n/4, 3n/4)^3 refined by 2 (fine n^3), the
    two-level recipe (lognormal density, optical depth 1e-2..1e2 per coarse cell, dt = 20 coarse crossings),
    mixed precision, consecutive steps from the same initial state after the warm-up."""
    from oracle.amr import TwoLevel
    n = args.n or 256
    q = n // 4
    log(f"generating the two-level workload: coarse {n}^3, box [{q},{3 * q})^3 refined ...")
    d = W.two_level((n, n, n), (q, q, q), (3 * q, 3 * q, 3 * q), seed=6, fp32_exact=True)
    geom = rad.amr_geometry(d["nc"], d["lo"], d["hi"])
    dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt).cuda()
    pk = lambda k, dt=torch.float64: rad.amr_pack(dev(d[k][0], dt), dev(d[k][1], dt))
    state0 = [pk("E"), pk("F"), pk("T")]
    coefs = [pk(k, torch.float32) for k in ("rho", "kP", "kR", "f")]
    Nc, Nf = n ** 3, (2 * q) ** 3 * 8
    leaf = Nc - (2 * q) ** 3 + Nf
    p = rad.params(prec="mixed", tol=args.tol, gmres_m=args.gmres_m, coef_dtype=1, krylov_poly=args.krylov_poly)
    ws = rad.alloc_workspace(rad.workspace_bytes_amr2(geom, p))
    E, F, T = (t.clone() for t in state0)
    share = None
    if not args.no_profile and args.warmup > 0:   # a uniform corner of the coarse level
        lv0 = lambda k, dt=torch.float64: dev(d[k][0], dt)
        load_code_objects(torch, rad, p, [lv0(k) for k in ("E", "F", "T")],
                          [lv0(k, torch.float32) for k in ("rho", "kP", "kR", "f")], d["dt"], d["dx"], d["bc"])
    for s in range(args.warmup):
        # the last warm-up step (from the same initial state as timed step 0) times every kernel class
        full = not args.no_profile and s == args.warmup - 1
        if full:
            rad.profile(True)
            rad.profile_reset()
            torch.cuda.synchronize()
            w0 = time.perf_counter()
        st = rad.rad_step_amr2(geom, E, F, T, *coefs, d["dt"], d["dx"], d["bc"], p, workspace=ws, check=False)
        if full:
            torch.cuda.synchronize()
            share = (time.perf_counter() - w0, rad.profile_read())
            rad.profile(False)
        log(f"  [amr] warmup step {s}: {st['picard_iters']} Picard, {st['krylov_iters']} Krylov, "
            f"{st['t_total_ms']:.0f} ms, res {st['scaled_residual']:.2e}")
    for dst, src in zip((E, F, T), state0):
        dst.copy_(src)
    # timed steps: events around the operator applies only (the roofline's kernel)
    rad.profile(2 if not args.no_profile else False)
    rad.profile_reset()
    stats, prev = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        if s == args.steps - 1:
            prev = [t.cpu().numpy() for t in (E, F, T)]
        st = rad.rad_step_amr2(geom, E, F, T, *coefs, d["dt"], d["dx"], d["bc"], p, workspace=ws, check=False)
        stats.append(st)
        log(f"  [amr] step {s}: rc {st['rc']}, {st['picard_iters']} Picard, {st['krylov_iters']} Krylov, "
            f"{st['t_total_ms']:.0f} ms, res {st['scaled_residual']:.2e}")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    prof = rad.profile_read() if not args.no_profile else {}
    rad.profile(False)
    res = {"metric": "two-level AMR implicit VET rad-step cell-updates/s (leaf cells, mixed precision)",
           "value": leaf * args.steps / sec, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1000.0 * sec / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"two-level grid: coarse {n}^3 periodic with the box [{q},{3 * q})^3 refined by 2 "
                                  f"(fine {2 * q * 2}^3), lognormal sigma 1, optical depth 1e-2..1e2 per coarse cell, "
                                  f"dt = 20 coarse crossings, FP32-exact inputs, {args.steps} steps, tol {args.tol:g}",
                      "leaf_cells": leaf, "stored_cells": Nc + Nf, "gmres_m": p.gmres_m,
                      "krylov_poly": p.krylov_poly},
           "krylov_iters_per_step": sum(s_["krylov_iters"] for s_ in stats) / args.steps,
           "picard_iters_per_step": sum(s_["picard_iters"] for s_ in stats) / args.steps,
           "converged_steps": sum(1 for s_ in stats if s_["rc"] == 0),
           "final_scaled_residual": stats[-1]["scaled_residual"]}
    if prof:
        dom = max(prof, key=lambda k: prof[k]["ms"])
        e = prof[dom]
        gbs = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                           "algorithmic_bytes_per_launch": e["bytes"] / e["launches"],
                           "avg_launch_us": 1000.0 * e["ms"] / e["launches"], "launches": e["launches"]}
        tot_b = sum(v["bytes"] for v in prof.values())
        res["step_roofline"] = {"achieved": tot_b / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": tot_b / sec / 1e9 / HBM_PEAK_GBS}
    if share:
        # from the fully profiled warm-up step (events around every launch), not the timed steps
        wsec, sp = share
        res["kernel_time_share"] = {k: v["ms"] / (wsec * 1e3) for k, v in sorted(sp.items(), key=lambda kv: -kv[1]["ms"])}
        res["kernel_gbs"] = {k: v["bytes"] / (v["ms"] * 1e-3) / 1e9 for k, v in sp.items() if v["ms"] > 0}
        res["kernel_share_note"] = (f"one warm-up step with HIP events around every launch ({wsec * 1e3:.0f} ms); "
                                    "the timed steps carry events around the operator applies only")
    if not args.no_oracle_check:
        log("composite oracle: residual of the last step on sampled leaf cells (jump cells included) ...")
        pb = TwoLevel(d["nc"], d["lo"], d["hi"], d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"])
        out = [t.cpu().numpy() for t in (E, F, T)]
        rng = np.random.default_rng(0)
        N = pb.N
        # covered coarse cells are no part of the composite system: on output they hold the mean of their children
        leaves = np.nonzero(~pb.covered)[0]
        jumps = np.unique(np.concatenate([pb.fL[pb.fJ], pb.fR[pb.fJ]]))
        cells = np.unique(np.concatenate([rng.choice(leaves, 4096, replace=False),
                                          rng.choice(jumps, min(1024, jumps.size), replace=False)]))
        Fp = np.concatenate([prev[1][:3 * Nc].reshape(3, Nc), prev[1][3 * Nc:].reshape(3, Nf)], axis=1) / d["c"]
        Fo = np.concatenate([out[1][:3 * Nc].reshape(3, Nc), out[1][3 * Nc:].reshape(3, Nf)], axis=1) / d["c"]
        R, Wt = pb.residual_at(cells, prev[0], Fp, prev[2], out[0], Fo, out[2])
        c = cells
        RT = np.where((out[2][c] == 0) & (R[4] > 0), 0.0, R[4])
        WT = pb.alpha[c] + 4 * pb.sP[c] * pb.aR * out[2][c] ** 3
        nE, nF, nT = np.linalg.norm(out[0][c]), np.linalg.norm(Fo[:, c]), np.linalg.norm(out[2][c])
        res["oracle_scaled_residual_sampled"] = {
            "E": float(np.linalg.norm(R[0] / Wt[0]) / nE), "F": float(np.linalg.norm(R[1:4] / Wt[1:4]) / (nF + nE)),
            "T": float(np.linalg.norm(RT / WT) / nT), "cells": int(c.size), "jump_cells": int(np.isin(c, jumps).sum())}
        del pb
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (two-level sample) ...")
        res["cpu_baseline"] = amr_cpu_baseline(args.tol)
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="grid edge (default 256; 512 for --workload scale)")
    ap.add_argument("--workload", choices=("precision", "scale", "amr"), default="precision",
                    help="precision: mixed-depth 256^3 recipe (the metric's workload); scale: lognormal sigma 2, "
                         "optical depth 1e-4..1e4, dt = 200 crossings (512^3, 3 steps); amr: two-level grid, "
                         "coarse 256^3 with the central half-box refined")
    ap.add_argument("--batched", action="store_true",
                    help="instead: the batched path on 1024 AMR-like Dirichlet blocks (one graph replay per step)")
    ap.add_argument("--reorder", action="store_true",
                    help="with --batched: queue the timed steps by the warm-up step's measured block solve times "
                         "(longest first) instead of largest block first")
    ap.add_argument("--autotune", nargs="?", const="tiles", choices=("tiles", "all"), default=None,
                    help="autotune before timing: the stencil z-ranges (tiles) or also the restart length (all); "
                         "with --batched: the launch shape")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--eps-r", type=float, default=3e-2,
                    help="relative tolerance of each linear solve, single-grid and batched legs (default 3e-2, "
                         "the fastest of 0.005..0.1 on the 256^3, 512^3 and 1024-block workloads; the library's "
                         "default 1e-2)")
    ap.add_argument("--krylov-poly", type=int, choices=(0, 1, 2), default=None,
                    help="Krylov operator: the Jacobi-scaled B times 1: the Neumann polynomial 2I - B (the library's "
                         "default), 0: nothing, 2: a multigrid V-cycle (default here on the uniform grids; the "
                         "two-level and batched runs default to 1)")
    ap.add_argument("--gmres-m", type=int, default=None,
                    help="GMRES restart length (default 8 on the grids, where orthogonalisation grows with m "
                         "while the iteration count barely changes; the library's 12 for --batched)")
    ap.add_argument("--bc", choices=("open", "outflow", "periodic"), default=None,
                    help="faces of the uniform-grid workloads (default: open, the characteristic outflow)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-scale-leg", action="store_true",
                    help="skip the 512^3 scale leg (mixed path, 1 warm-up + 3 steps) of the default run")
    ap.add_argument("--no-batched-leg", action="store_true",
                    help="skip the batched leg (1024 blocks, 1 warm-up + 1 step) of the default run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=24)
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel HIP events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 4 plain device copies of 256 MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gmres_m is None and not args.batched:
        args.gmres_m = 8
    if args.krylov_poly is None:
        # the multigrid operator on the uniform grids (it falls back to the Neumann one by itself where a
        # cycle stalls); the two-level and batched paths have only the Neumann operator
        args.krylov_poly = 1 if (args.batched or args.workload == "amr") else 2
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; a sharded step would give "
              "each GPU a slab of the grid at this shape, with a one-plane halo exchange per operator apply",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2202_08778_amd import rad
    from paper_2202_08778_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batched:
        return bench_batched(args, torch, np, rad, W)
    if args.workload == "amr":
        return bench_amr(args, torch, np, rad, W)
    scale = args.workload == "scale"
    n = args.n or (512 if scale else 256)
    res = bench_grid(args, torch, np, rad, W, scale, n, args.steps, args.warmup, with_fp64=not args.no_fp64,
                     with_closure=True)
    if not scale and not args.no_scale_leg:
        # the 512^3 scale recipe, mixed path only: one warm-up and three timed steps
        torch.cuda.empty_cache()
        log("scale leg: 512^3 mixed-depth recipe (sigma 2, optical depth 1e-4..1e4, 200 crossings), mixed path ...")
        res["scale_512"] = bench_grid(args, torch, np, rad, W, True, 512, 3, 1, with_fp64=False, with_closure=False)
    if not args.no_batched_leg:
        torch.cuda.empty_cache()
        log("batched leg: 1024 Dirichlet blocks, one warm-up and one timed graph replay ...")
        res["batched_1024"] = bench_batched(args, torch, np, rad, W, steps=1, warmup=1, emit=False)
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline at {args.cpu_sample_n}^3 ...")
        res["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.tol, n)
    print(json.dumps(res), flush=True)


def bench_grid(args, torch, np, rad, W, scale, n, steps, warmup, with_fp64, with_closure):
    """One uniform-grid workload: the mixed path timed over `steps` steps after `warmup`, optionally the
    FP64 path from the same state, the oracle's residual of the last mixed step and the roofline."""
    log(f"generating the {'scale' if scale else 'precision'} workload at {n}^3 ...")
    d = W.mixed_depth_512(n=n, steps=steps) if scale else W.mixed_depth_256(n=n, steps=steps)
    if args.bc:
        d["bc"] = args.bc
    recipe = ("lognormal sigma 2, optical depth 1e-4..1e4, dt = 200 light-crossing times" if scale else
              "lognormal sigma 1.5, optical depth 1e-3..1e3, dt = 50 light-crossing times")
    faces = d["bc"] if isinstance(d["bc"], str) else "/".join(d["bc"])
    dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt).cuda()
    state0 = (dev(d["E"]), dev(d["F"]), dev(d["T"]))
    c32 = tuple(dev(d[k], torch.float32) for k in ("rho", "kP", "kR", "f"))
    N = n ** 3

    log("mixed path (FP32 Krylov + FP64 residual/refinement/exchange, FP32 coefficient storage):")
    mixed = run_path(torch, rad, d, state0, c32, "mixed", steps, warmup, args.tol, not args.no_profile,
                     args.gmres_m, args.autotune, args.eps_r, args.krylov_poly)
    value = N * steps / mixed["seconds"]
    out_m = [t.cpu().numpy() for t in mixed["state"]]

    closure = None
    if with_closure:
        # local M1 closure (Sec. 4.1) from the final state, FP32 output as the mixed path consumes it
        rad.profile_reset()
        rad.profile(True)
        fcl = torch.empty((6, n, n, n), dtype=torch.float32, device="cuda")
        for _ in range(10):
            rad.rad_closure(mixed["state"][0], mixed["state"][1], "m1", d["c"], f=fcl)
        torch.cuda.synchronize()
        cl = rad.profile_read().get("closure")
        rad.profile(False)
        del fcl
        closure = None if not cl else {"kernel": "k_closure (M1, FP32 out)",
                                       "us_per_launch": 1000 * cl["ms"] / cl["launches"],
                                       "algorithmic_bytes_per_launch": cl["bytes"] / cl["launches"],
                                       "achieved_GBps": cl["bytes"] / (cl["ms"] * 1e-3) / 1e9}

    fp64 = None
    if with_fp64:
        log("FP64 path (FP64 Krylov, FP64 coefficient storage):")
        c64 = tuple(dev(d[k]) for k in ("rho", "kP", "kR", "f"))
        fp64 = run_path(torch, rad, d, state0, c64, "fp64", steps, warmup, args.tol, False, args.gmres_m,
                        args.autotune, args.eps_r, args.krylov_poly)
        del c64

    res = {
        "metric": METRIC if not scale else "implicit VET rad-step cell-updates/s at 512^3 (scale recipe), mixed path",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1000.0 * mixed["seconds"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"mixed-depth medium {n}^3 ({recipe}), {faces} faces, "
                               f"FP32-exact inputs, {steps} implicit steps, tol {args.tol:g}",
                   "cells": N, "gmres_m": (mixed["tuned"] or {}).get("gmres_m", args.gmres_m), "eps_R": args.eps_r,
                   "krylov_poly": (mixed["tuned"] or {}).get("krylov_poly", args.krylov_poly),
                   "autotune": mixed["tuned"],
                   "precision": "FP32 Krylov/apply, FP64 residual, refinement and exchange"},
        "krylov_iters_per_step": sum(s["krylov_iters"] for s in mixed["stats"]) / steps,
        "krylov_iters_per_s": sum(s["krylov_iters"] for s in mixed["stats"]) / mixed["seconds"],
        "operator_applies_per_step": (1, 2, 3)[(mixed["tuned"] or {}).get("krylov_poly", args.krylov_poly)]
                                     * sum(s["krylov_iters"] for s in mixed["stats"]) / steps,
        "picard_iters_per_step": sum(s["picard_iters"] for s in mixed["stats"]) / steps,
        "converged_steps": sum(1 for s in mixed["stats"] if s["rc"] == 0),
        "final_scaled_residual": mixed["stats"][-1]["scaled_residual"],
        "energy_defect_last_step": mixed["stats"][-1]["energy_defect"],
        "algorithmic_bytes_per_step": sum(s["bytes_moved"] for s in mixed["stats"]) / steps,
    }
    if fp64 is not None:
        v64 = N * steps / fp64["seconds"]
        out_d = [t.cpu().numpy() for t in fp64["state"]]
        res["fp64_value"] = v64
        res["fp64_ms_per_step"] = 1000.0 * fp64["seconds"] / steps
        res["speedup_mixed_vs_fp64"] = value / v64
        res["fp64_krylov_iters_per_step"] = sum(s["krylov_iters"] for s in fp64["stats"]) / steps
        res["fp64_converged_steps"] = sum(1 for s in fp64["stats"] if s["rc"] == 0)
        res["relerr_mixed_vs_fp64"] = {k: relerr(a, b) for k, a, b in zip(("E", "F", "T"), out_m, out_d)}
        del out_d

    if not args.no_oracle_check:
        import oracle
        log("oracle residual of the mixed result (last step) ...")
        P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                           cv=d["cv"])
        prev = [t.cpu().numpy() for t in mixed["prev"]]
        r = P.scaled_residual(*prev, *out_m)
        res["oracle_scaled_residual_last_step"] = r[3]
        del P, prev

    if closure:
        res["closure_m1"] = closure
    prof = mixed["profile"]
    if prof:
        dom = max(prof, key=lambda k: prof[k]["ms"])
        e = prof[dom]
        gbs = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS,
                           "traffic": measured_traffic(dom, n),
                           "algorithmic_bytes_per_launch": e["bytes"] / e["launches"],
                           "avg_launch_us": 1000.0 * e["ms"] / e["launches"], "launches": e["launches"]}
        # the whole step: every kernel's algorithmic bytes over the step's wall time
        tot_b = sum(v["bytes"] for v in prof.values())
        res["step_roofline"] = {"achieved": tot_b / mixed["seconds"] / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": tot_b / mixed["seconds"] / 1e9 / HBM_PEAK_GBS,
                                "note": "sum of algorithmic bytes of all kernels / wall time of the timed steps"}
    sh = mixed["share"]
    if sh:
        # from the fully profiled warm-up step (events around every launch), not the timed steps
        sp = sh["profile"]
        res["kernel_time_share"] = {k: v["ms"] / (sh["seconds"] * 1e3) for k, v in
                                    sorted(sp.items(), key=lambda kv: -kv[1]["ms"])}
        res["kernel_gbs"] = {k: v["bytes"] / (v["ms"] * 1e-3) / 1e9 for k, v in sp.items() if v["ms"] > 0}
        res["kernel_share_note"] = ("one warm-up step with HIP events around every launch "
                                    f"({sh['seconds'] * 1e3:.0f} ms); the timed steps carry events "
                                    "around the operator applies only")

    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = {"read": x.numel() * 4, "write": y.numel() * 4}
        del x, y
    del mixed, state0, c32, d, out_m
    return res


if __name__ == "__main__":
    main()
