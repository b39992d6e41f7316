#!/usr/bin/env python3
"""Throughput benchmark of the adaptive finite-volume hot path on one MI355X.

Headline workload: 2D four-quadrant Riemann problem (seeded states), adaptive
MR hierarchy with 5 levels (32^2 .. 512^2), eps = 1e-3 on density details,
global time step at CFL 0.45, run towards t = 0.25, FP32 state and flux with
FP64 CFL / totals / threshold.  One bench step = one full time step of the
hot path (CFL reduction, two finite-volume stages on every leaf with
projection and ghost fill, MR analysis, flags, tiling, prediction of new
cells).  value = leaf cell-updates per second over the timed steps, inputs
resident in HBM.

Prints ONE JSON line.  --gpus N > 1 is not supported: this build runs on one
GPU.
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

# algorithmic floating-point operations of one finite-volume stage per leaf
# cell (count of the adds, multiplies, divides and square roots of the
# expression tree: one primitive conversion per cell, one flux per face, the
# update), see the design notes for the breakdown
FLOPS_PER_CELL_STAGE = {2: 325, 3: 568}
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_adaptive(precision, seed=0):
    from paper_1603_05211_amd import EU_FP32, EU_FP64, Solver, inputs
    s = Solver(2, n0=32, levels=5, precision=EU_FP32 if precision == "fp32" else EU_FP64,
               cfl=0.45, t_end=0.25, eps=1e-3, eta=0.8, patch_min=8, patch_max=32)
    s.init_quadrant(inputs.quadrant_states(seed))
    return s


def timed_advance(s, steps, use_graph=True):
    import torch
    u0, st0 = s.leaf_updates()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = s.advance(steps, use_graph=use_graph)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u1, st1 = s.leaf_updates()
    return done, u1 - u0, t1 - t0


def kernel_profile(s, steps):
    """Average duration of the finite-volume stage kernel, from HIP events
    recorded around each launch on the context's stream."""
    u0, st0 = s.leaf_updates()
    s.profile(True)
    s.advance(steps, use_graph=False)
    ms, n = s.kernel_time()
    s.profile(False)
    u1, st1 = s.leaf_updates()
    cells_per_launch = (u1 - u0) / max(st1 - st0, 1)
    return ms / max(n, 1), n, cells_per_launch


def cpu_baseline(budget_s=15.0, seed=0):
    """The FP64 oracle on the same workload, from initialisation, for as many
    steps as fit in about budget_s seconds of host time."""
    import oracle as orc
    from paper_1603_05211_amd import inputs
    prim = inputs.quadrant_states(seed)
    h = orc.Hierarchy(2, 5, 32, eps=1e-3, eta=0.8, pmin=8, pmax=32)
    h.init_finest(orc.init_quadrant(512, 1.4, prim))
    t0 = time.perf_counter()
    updates, steps = 0, 0
    while time.perf_counter() - t0 < budget_s and h.t < 0.25:
        leaves, _ = h.counts()
        h.step(0.45, 0.25)
        updates += int(leaves.sum())
        steps += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": updates / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, same workload (seed 0), first {steps} time steps from "
                      f"initialisation ({updates} leaf updates in {dt:.1f} s)"}


def extra_uniform(dim, n, precision, steps, seed=0):
    from paper_1603_05211_amd import EU_FP32, EU_FP64, Solver, inputs
    prec = EU_FP32 if precision == "fp32" else EU_FP64
    if dim == 2:
        s = Solver(2, n0=n, levels=1, precision=prec, cfl=0.45)
        s.init_quadrant(inputs.quadrant_states(seed))
    else:
        e = inputs.ellipsoid(seed)
        s = Solver(3, n0=n, levels=1, precision=prec, cfl=0.4, lo=-1.0, hi=1.0)
        s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    s.advance(3, use_graph=True)
    variant, _ = s.autotune(reps=5)
    done, upd, dt = timed_advance(s, steps)
    ms, nl, cells = kernel_profile(s, 4)
    out = {"value": upd / dt, "steps": done, "fv_stage_ms": ms, "stage_schedule": variant}
    s.close()
    return out


def extra_adaptive3d_lts(precision, steps, seed=0):
    """3D ellipsoid, 4 levels 32^3..256^3, eps 1e-3, local time stepping."""
    from paper_1603_05211_amd import EU_DT_LTS, EU_FP32, EU_FP64, Solver, inputs
    e = inputs.ellipsoid(seed)
    s = Solver(3, n0=32, levels=4, precision=EU_FP32 if precision == "fp32" else EU_FP64, cfl=0.4,
               t_end=0.2, eps=1e-3, eta=0.8, patch_min=8, patch_max=32, lo=-1.0, hi=1.0,
               time_mode=EU_DT_LTS)
    s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    s.advance(2, use_graph=True)
    variant, _ = s.autotune(reps=3)
    done, upd, dt = timed_advance(s, steps)
    leaves, active = s.counters()
    out = {"value": upd / dt, "steps": done, "ms_per_level0_step": 1e3 * dt / max(done, 1),
           "stage_schedule": variant,
           "leaves": [int(x) for x in leaves], "patch_cells": [int(x) for x in active]}
    s.close()
    return out


def extra_batch(precision, steps, seed=0):
    from paper_1603_05211_amd import EU_FP32, EU_FP64, Solver, inputs
    b = inputs.batch(seed)
    s = Solver(2, sides=list(b.sides), precision=EU_FP32 if precision == "fp32" else EU_FP64, cfl=0.45)
    s.init_quadrant_batch(b.states)
    s.advance(3, use_graph=True)
    variant, _ = s.autotune(reps=3)
    done, upd, dt = timed_advance(s, steps)
    ms, nl, cells = kernel_profile(s, 4)
    out = {"value": upd / dt, "steps": done, "cells_per_step": int(b.sides.astype(float).__pow__(2).sum()),
           "fv_stage_ms": ms, "stage_schedule": variant}
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-extra", action="store_true", help="skip the context configurations")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-steps", type=int, default=40)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    s = make_adaptive(args.precision)
    variant, variant_ms = s.autotune(reps=10)
    log(f"autotuned stage schedule {variant} ({variant_ms})")
    log(f"warmup {args.warmup} steps")
    s.advance(args.warmup, use_graph=True)
    log(f"timing {args.steps} steps")
    done, upd, wall = timed_advance(s, args.steps)
    if done != args.steps:
        log(f"warning: only {done} of {args.steps} steps before t_end")
    value = upd / wall
    leaves, active = s.counters()
    log(f"profiling {args.profile_steps} steps with events")
    fv_ms, nlaunch, cells_per_launch = kernel_profile(s, args.profile_steps)
    flops = FLOPS_PER_CELL_STAGE[2] * cells_per_launch
    achieved = flops / (fv_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    es = 4 if args.precision == "fp32" else 8
    s.close()

    result = {
        "metric": "cell-updates/s (FP32 batched vs FP64 plain) at stated L1 err; % HBM roofline",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": done,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(done, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic: seeded four-quadrant Riemann states (seed 0)",
        "config": {"workload": "quad2d_adaptive5: 2D four-quadrant Riemann, adaptive MR 5 levels "
                               "32^2..512^2, eps 1e-3, eta 0.8, patches 8..32, global dt, CFL 0.45, "
                               "t_end 0.25",
                   "precision": args.precision, "leaf_updates": upd,
                   "stage_schedule": variant, "stage_schedule_ms": variant_ms,
                   "leaves_per_step_mean": upd / max(done, 1)},
        "roofline": {"bound": "alu", "kernel": "k_fv_stage", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "avg_launch_ms": fv_ms, "launches": nlaunch,
                     "cells_per_launch": cells_per_launch,
                     "flops_per_cell": FLOPS_PER_CELL_STAGE[2],
                     "hbm_algorithmic_GBs": 3 * 4 * es * cells_per_launch / (fv_ms * 1e-3) / 1e9},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline()
    if not args.no_extra:
        log("context configurations")
        ex = {}
        s64 = make_adaptive("fp64")
        s64.advance(args.warmup, use_graph=True)
        d, u, w = timed_advance(s64, args.steps)
        ex["quad2d_adaptive5_fp64"] = {"value": u / w, "steps": d}
        s64.close()
        ex["quad2d_uniform512_fp64"] = extra_uniform(2, 512, "fp64", 100)
        ex["quad2d_uniform512_fp32"] = extra_uniform(2, 512, "fp32", 100)
        ex["ellip3d_uniform256_fp32"] = extra_uniform(3, 256, "fp32", 40)
        ex["ellip3d_uniform256_fp64"] = extra_uniform(3, 256, "fp64", 20)
        ex["quad2d_batch512_fp32"] = extra_batch("fp32", 20)
        ex["ellip3d_adaptive4_lts_fp32"] = extra_adaptive3d_lts("fp32", 10)
        result["extra"] = ex
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
