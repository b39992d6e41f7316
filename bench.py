#!/usr/bin/env python3
"""Throughput benchmark of the adaptive finite-volume hot path on one MI355X.

A bench step is one whole run of a workload from its initial state over its
defined extent (the 2D adaptive workload to t = 0.25, 936 time steps for
seed 0): initialisation (untimed), then every time step of the run replayed
from captured HIP graphs (runs of sixteen steps per graph).  A time step is the whole hot path: CFL
reduction, two finite-volume stages on every leaf with projection and ghost
fill, MR analysis, flags, tiling, lists, prediction of new cells.  value =
leaf cell-updates per second over the timed runs, with the state resident in
HBM.  The result does not depend on --steps (the number of runs timed).

Default workload (quad2d_adaptive5): 2D four-quadrant Riemann problem (seeded
states), adaptive MR hierarchy with 5 levels (32^2 .. 512^2), eps = 1e-3 on
density details, eta_tol = 0.8, patches 8..32, global time step at CFL 0.45,
run to t = 0.25, FP32 state and flux with FP64 CFL / totals / threshold.
Every result carries its error against the FP64 oracle (or the FP64 path,
where the oracle cannot run the workload in minutes).

Context lines also time the AMR method (AMR scheme with the scaled-gradient
criterion, eps_rho = 0.05, Berger-Rigoutsos clustering) on the same
five-level hierarchy and the AMR scheme on the batch and the 128^2 grid.

Other workloads (--workload): ellip3d_adaptive4_lts (3D, 4 levels, local time
stepping, to t = 0.2), ellip3d_uniform256 (200 steps), quad2d_batch512 (512
instances, 100 steps, one launch per stage for all), quad2d_uniform128 (100
steps).

Prints ONE JSON line.  --gpus N > 1 is not supported: the benchmark runs on one
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic floating-point operations of one finite-volume stage per leaf
# cell: adds, multiplies, divides and square roots of the expression tree
# (one primitive conversion per cell, one flux per face, the update).  MR
# scheme: a midpoint-rule stage; AMR scheme (2D): the whole MUSCL-Hancock
# step (predictor of the face values and the AUSMDV corrector).
FLOPS_PER_CELL_STAGE = {2: 325, 3: 568}
FLOPS_PER_CELL_AMR = {2: 445}
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}      # MI355X vector peaks
HBM_PEAK_GBS = 8000.0
FV_SOURCES = ["paper_1603_05211_amd/csrc/eu_kernels.hpp", "paper_1603_05211_amd/csrc/eu_kset_impl.hpp",
              "paper_1603_05211_amd/csrc/eu_internal.hpp", "paper_1603_05211_amd/csrc/eu_strip.hpp",
              "paper_1603_05211_amd/csrc/eu_strip3.hpp", "paper_1603_05211_amd/csrc/eu_hancock.hpp"]
SCHEME_NAMES = ["MR (MUSCL, van Albada, AUSM+, RK2)", "AMR (MUSCL-Hancock, Minmod, AUSMDV)"]
# workloads set up with the AMR scheme when asked for (Run below)
AMR_WORKLOADS = {"quad2d_adaptive5", "quad2d_batch512", "quad2d_uniform128"}
METRIC = "cell-updates/s (FP32 batched vs FP64 plain) at stated L1 err; % HBM roofline"

WORKLOADS = {
    "quad2d_adaptive5": "2D four-quadrant Riemann, adaptive MR 5 levels 32^2..512^2, eps 1e-3, "
                        "eta 0.8, patches 8..32, global dt, CFL 0.45, run to t = 0.25",
    "ellip3d_adaptive4_lts": "3D ellipsoidal blast on [-1,1]^3, adaptive MR 4 levels 32^3..256^3, "
                             "eps 1e-3, eta 0.8, patches 8..32, local time steps, CFL 0.4, run to t = 0.2",
    "ellip3d_uniform256": "3D ellipsoidal blast on [-1,1]^3, uniform 256^3, CFL 0.4, 200 steps",
    "quad2d_batch512": "512 independent 2D four-quadrant Riemann instances, sides 32..512, CFL 0.45, "
                       "100 steps",
    "quad2d_uniform128": "2D four-quadrant Riemann, uniform 128^2, CFL 0.45, 100 steps",
}
FIXED_STEPS = {"ellip3d_uniform256": 200, "quad2d_batch512": 100, "quad2d_uniform128": 100}
T_END = {"quad2d_adaptive5": 0.25, "ellip3d_adaptive4_lts": 0.2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# workloads on the GPU
# ---------------------------------------------------------------------------

class Run:
    """A workload on the library: the solver and how to (re)initialise it."""

    def __init__(self, workload, precision, seed=0, scheme=0):
        from paper_1603_05211_amd import EU_CRIT_GRADIENT, EU_DT_LTS, EU_FP32, EU_FP64, EU_TILER_BR, Solver, inputs
        self.workload, self.precision, self.scheme = workload, precision, scheme
        prec = EU_FP32 if precision == "fp32" else EU_FP64
        if workload == "quad2d_adaptive5" and scheme == 1:
            # the AMR method on the same hierarchy: AMR scheme, the
            # scaled-gradient criterion on density (the paper's 2D eps_rho)
            # and Berger-Rigoutsos clustering
            s = Solver(2, n0=32, levels=5, precision=prec, cfl=0.45, t_end=0.25, eps=0.05, eta=0.8,
                       patch_min=8, patch_max=32, scheme=1, criterion=EU_CRIT_GRADIENT, tiler=EU_TILER_BR)
            prim = inputs.quadrant_states(seed)
            self.init = lambda: s.init_quadrant(prim)
            self.dim = 2
        elif workload == "quad2d_adaptive5":
            s = Solver(2, n0=32, levels=5, precision=prec, cfl=0.45, t_end=0.25, eps=1e-3, eta=0.8,
                       patch_min=8, patch_max=32)
            prim = inputs.quadrant_states(seed)
            self.init = lambda: s.init_quadrant(prim)
            self.dim = 2
        elif workload == "ellip3d_adaptive4_lts":
            e = inputs.ellipsoid(seed)
            s = Solver(3, n0=32, levels=4, precision=prec, cfl=0.4, t_end=0.2, eps=1e-3, eta=0.8,
                       patch_min=8, patch_max=32, lo=-1.0, hi=1.0, time_mode=EU_DT_LTS)
            self.init = lambda: s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
            self.dim = 3
        elif workload == "ellip3d_uniform256":
            e = inputs.ellipsoid(seed)
            s = Solver(3, n0=256, levels=1, precision=prec, cfl=0.4, lo=-1.0, hi=1.0)
            self.init = lambda: s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
            self.dim = 3
        elif workload == "quad2d_batch512":
            b = inputs.batch(seed)
            s = Solver(2, sides=list(b.sides), precision=prec, cfl=0.45, scheme=scheme)
            self.init = lambda: s.init_quadrant_batch(b.states)
            self.dim = 2
        elif workload == "quad2d_uniform128":
            s = Solver(2, n0=128, levels=1, precision=prec, cfl=0.45, scheme=scheme)
            prim = inputs.quadrant_states(seed)
            self.init = lambda: s.init_quadrant(prim)
            self.dim = 2
        else:
            raise ValueError(workload)
        self.s = s
        self.init()
        self.nsteps = None
        self.variant = None
        self.tuning = None

    def close(self):
        self.s.close()

    def kernel(self):
        """The finite-volume kernel the chosen schedule launches."""
        if self.scheme == 1:
            return "k_hancock_tile" if self.variant is None or self.variant < 6 else "k_hancock_strip"
        if self.variant is None or self.variant < 6:
            return "k_fv_stage"
        return "k_fv_strip3" if self.dim == 3 else "k_fv_strip"

    def flops_per_cell_stage(self):
        return FLOPS_PER_CELL_AMR[self.dim] if self.scheme == 1 else FLOPS_PER_CELL_STAGE[self.dim]

    def extent(self, tune_every=0, reps=5):
        """One untimed run over the workload's extent from the initial state;
        with tune_every > 0 every stage schedule is timed on the live state
        every tune_every steps and the schedule with the least summed time
        over the run is kept.  Sets the steps of a run."""
        s = self.s
        self.init()
        fixed = FIXED_STEPS.get(self.workload)
        t_end = T_END.get(self.workload, math.inf)
        chunk = tune_every if tune_every > 0 else (fixed or 64)
        tot, samples, done = None, 0, 0
        while True:
            if tune_every > 0:
                _, ms = s.autotune(reps=reps)
                tot = ms if tot is None else [a + b for a, b in zip(tot, ms)]
                samples += 1
            want = chunk if fixed is None else min(chunk, fixed - done)
            k = s.advance(want, use_graph=True)
            done += k
            if fixed is not None and done >= fixed:
                break
            if fixed is None and (k < want or s.time()[0] >= t_end):
                break
        self.nsteps = done
        if tot is not None:
            best = min(range(len(tot)), key=lambda i: tot[i])
            s.set_variant(best)
            self.variant = best
            self.tuning = {"samples": samples, "every_steps": tune_every,
                           "ms_summed_per_schedule": [round(x, 5) if math.isfinite(x) else None for x in tot]}
        return done

    def timed(self, k):
        """k runs over the extent, each from the initial state (untimed
        initialisation), each timed between two device synchronisations.
        Returns (leaf updates, seconds, runs)."""
        import torch
        s = self.s
        upd, sec = 0, 0.0
        for _ in range(k):
            self.init()
            u0, _ = s.leaf_updates()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = s.advance(self.nsteps, use_graph=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            u1, _ = s.leaf_updates()
            if n != self.nsteps:
                raise RuntimeError(f"run took {n} steps, expected {self.nsteps}")
            upd += u1 - u0
            sec += t1 - t0
        return upd, sec, k

    def stage_samples(self, samples=64, reps=20):
        """Average duration of the finite-volume stage kernel over the run:
        at `samples` evenly spaced steps, reps first-stage passes on the live
        state (in the configuration the step launches them) replayed from one
        HIP graph between two HIP events on the library's stream.  Returns
        (ms per launch, launches timed, cells per launch, launches per pass,
        flops-weighted TFLOP/s)."""
        s = self.s
        self.init()
        every = max(1, self.nsteps // samples)
        ms_sum, cells_sum, launches, lpp, done, nsamp = 0.0, 0.0, 0, 1, 0, 0
        while done + every < self.nsteps:
            done += s.advance(every, use_graph=True)
            ms, cells, lpp = s.stage_time(reps)
            ms_sum += ms * reps
            cells_sum += cells * reps
            launches += lpp * reps
            nsamp += 1
        n = max(launches, 1)
        flops = self.flops_per_cell_stage() * cells_sum
        # finite-volume launches of this phase: the steps between samples
        # (launches per pass each) and each sample's untimed and timed replay
        self.phase_launches = nsamp * lpp * (every + 2 * reps)
        return ms_sum / n, launches, cells_sum / n, lpp, flops / (ms_sum * 1e-3) / 1e12 if ms_sum else 0.0


def source_hash():
    h = hashlib.sha256()
    for p in FV_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, precision, kernel, cells_per_launch, schedule=None):
    """HBM bytes per launch of the finite-volume kernel: the committed counter
    summary of this workload, kernel and stage schedule (FETCH_SIZE and
    WRITE_SIZE per launch, scaled by the readings of a plain 256 MiB device
    copy) gives bytes per cell-stage, which is scaled to this run's
    cell-stages per launch.  None when the summary is missing or the kernel
    sources changed since the counters were taken."""
    d = path = None
    for name in ([f"{kernel}_{workload}_{precision}_s{schedule}_traffic.json"] if schedule is not None else []) + \
            [f"{kernel}_{workload}_{precision}_traffic.json"]:
        path = os.path.join(ROOT, "profiles", name)
        try:
            with open(path) as f:
                d = json.load(f)
            break
        except (OSError, ValueError):
            d = None
    if d is None:
        return None, "no counter summary"
    if d.get("source_hash") != source_hash():
        return None, "kernel changed since the counters were taken"
    src = os.path.relpath(path, ROOT)
    if "schedule" in d:
        src += f" (counters taken with stage schedule {d['schedule']})"
    return d["traffic_bytes_per_cell_stage"] * cells_per_launch, src


STAGE_REPS = 20   # passes per timed graph replay (the replay's own launch cost spread over them)


def roofline(r, precision, samples=64):
    ms, nl, cells, lpp, tflops = r.stage_samples(samples, STAGE_REPS)
    peak = PEAK_TFLOPS[precision]
    kern = r.kernel()
    traffic, src = traffic_from_profile(r.workload, precision, kern, cells, r.variant)
    return {"bound": "alu", "kernel": kern, "achieved": tflops, "peak": peak, "unit": "TFLOP/s",
            "frac": tflops / peak, "traffic": traffic, "traffic_source": src, "avg_launch_ms": ms,
            "launches": nl, "launches_per_pass": lpp, "cell_stages_per_launch": cells,
            "phase_launches": getattr(r, "phase_launches", None),
            "flops_per_cell_stage": r.flops_per_cell_stage(),
            "timing": f"HIP events on the library's stream around graphs of {STAGE_REPS} passes of one step's "
                      f"finite-volume work at {samples} evenly spaced steps of the run (the tracer's "
                      "kernel durations are in profiles/)"}


# ---------------------------------------------------------------------------
# accuracy (the error assessment of Sec. 3)
# ---------------------------------------------------------------------------

def field_errors(g, o, dim, dx):
    """Per field: L1 = dx^d sum |g - o| and normwise L-inf relative
    max |g - o| / max |o|, on arrays (nv, n, ..)."""
    import numpy as np
    vol = dx ** dim
    l1 = [float(np.abs(g[f] - o[f]).sum() * vol) for f in range(g.shape[0])]
    linf = [float(np.abs(g[f] - o[f]).max() / max(np.abs(o[f]).max(), 1e-300)) for f in range(g.shape[0])]
    return l1, linf


def adaptive_oracle_run(workload, seed=0):
    """The FP64 oracle over the whole 2D adaptive run (test infrastructure:
    the error reference of the bench line and its multi-threaded CPU
    baseline)."""
    import oracle as orc
    from paper_1603_05211_amd import inputs
    h = orc.Hierarchy(2, 5, 32, eps=1e-3, eta=0.8, pmin=8, pmax=32)
    h.init_finest(orc.init_quadrant(512, 1.4, inputs.quadrant_states(seed)))
    t0 = time.perf_counter()
    upd, steps = 0, 0
    while h.t < 0.25:
        leaves, _ = h.counts()
        h.step(0.45, 0.25)
        upd += int(leaves.sum())
        steps += 1
    return h, upd, steps, time.perf_counter() - t0


def hierarchy_error(snap, h):
    """Composite (finest-grid) errors of a GPU hierarchy (a snapshot of its
    final state) against the oracle, flag disagreements per level and
    patch-table differences."""
    import numpy as np
    g, o = snap["composite"], h.composite()
    l1, linf = field_errors(g, o, 2, h.dx(h.L - 1))
    flags = [int((snap["flags"][l] != h.flags(l)).sum()) for l in range(h.L - 1)]
    Pg = {tuple(r) for r in snap["patches"].tolist()}
    Po = {tuple(r) for r in h.patches().tolist()}
    return {"l1": l1, "linf_rel": linf, "flag_disagreements_per_level": flags,
            "patch_rows_differing": len(Pg ^ Po), "bit_exact": bool(np.array_equal(g, o)),
            "reference": "FP64 oracle, the same run (composite on the finest grid, Sec. 3)"}


def uniform_error(a, b, dim, dx, ref):
    l1, linf = field_errors(a, b, dim, dx)
    return {"l1": l1, "linf_rel": linf, "reference": ref}


# ---------------------------------------------------------------------------
# CPU baseline (the oracle, as it stands)
# ---------------------------------------------------------------------------

def cpu_sample(workload, budget_s, seed=0):
    """The FP64 oracle on the first steps of the workload for about budget_s
    seconds of host time; returns (cell updates, seconds, steps)."""
    import oracle as orc
    from paper_1603_05211_amd import inputs
    if workload == "quad2d_adaptive5":
        h = orc.Hierarchy(2, 5, 32, eps=1e-3, eta=0.8, pmin=8, pmax=32)
        h.init_finest(orc.init_quadrant(512, 1.4, inputs.quadrant_states(seed)))
        step = lambda: (int(h.counts()[0].sum()), h.step(0.45, 0.25))[0]
    elif workload == "quad2d_uniform128":
        h = orc.Hierarchy(2, 1, 128)
        h.init_finest(orc.init_quadrant(128, 1.4, inputs.quadrant_states(seed)))
        step = lambda: (128 * 128, h.step(0.45))[0]
    elif workload == "ellip3d_uniform256":
        e = inputs.ellipsoid(seed)
        h = orc.Hierarchy(3, 1, 256, lo=-1.0, hi=1.0)
        h.init_finest(orc.init_ellipsoid(256, 1.4, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0, e.rc))
        step = lambda: (256 ** 3, h.step(0.4))[0]
    elif workload == "ellip3d_adaptive4_lts":
        e = inputs.ellipsoid(seed)
        h = orc.Hierarchy(3, 4, 32, lo=-1.0, hi=1.0, eps=1e-3, eta=0.8, pmin=8, pmax=32)
        h.init_finest(orc.init_ellipsoid(256, 1.4, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0, e.rc))
        step = lambda: h.step_lts(0.4, 0.2)[1]
    else:  # batch: whole instances in order, 10 steps each
        b = inputs.batch(seed)
        state = {"i": 0}

        def step():
            i = state["i"]
            n = int(b.sides[i])
            hh = orc.Hierarchy(2, 1, n)
            hh.init_finest(orc.init_quadrant(n, 1.4, b.states[i]))
            for _ in range(10):
                hh.step(0.45)
            state["i"] = i + 1
            return 10 * n * n
    t0 = time.perf_counter()
    upd, steps = 0, 0
    while steps < 1 or time.perf_counter() - t0 < budget_s:
        upd += step()
        steps += 1
    return upd, time.perf_counter() - t0, steps


def cpu_sample_1thread(workload, budget_s):
    """The same sample in a child process with one OpenMP thread."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample", workload,
                        "--cpu-budget", str(budget_s)], capture_output=True, text=True, env=env)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": d["updates"] / d["seconds"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle, one thread: first {d['steps']} steps of the same run "
                      f"({d['updates']} cell updates in {d['seconds']:.1f} s)"}


# ---------------------------------------------------------------------------

def extra_line(workload, precision, runs, tune=True, after=None, scheme=0):
    """A context line: the workload timed over its extent (runs runs),
    `after(run)` called on the final state of the last timed run (its
    result, when a dict, is the line's accuracy), then the finite-volume
    kernel's rate over the run."""
    r = Run(workload, precision, scheme=scheme)
    r.extent(tune_every=max(1, (FIXED_STEPS.get(workload) or 200) // 4) if tune else 0, reps=3)
    upd, sec, k = r.timed(runs)
    out = {"value": upd / sec, "runs": k, "steps_per_run": r.nsteps, "ms_per_run": 1e3 * sec / k,
           "stage_schedule": r.variant, "tuning": r.tuning, "precision": precision,
           "scheme": SCHEME_NAMES[scheme]}
    if after is not None:
        acc = after(r)
        if isinstance(acc, dict):
            out["accuracy"] = acc
    out["roofline"] = roofline(r, precision, samples=16)
    es, nv = (4 if precision == "fp32" else 8), r.dim + 2
    out["roofline"]["hbm_algorithmic_GBs"] = out["value"] * 2 * nv * es / 1e9
    out["roofline"]["hbm_algorithmic_frac"] = out["value"] * 2 * nv * es / 1e9 / HBM_PEAK_GBS
    r.close()
    return out


def hierarchy_snapshot(s):
    return {"composite": s.composite(), "flags": [s.flags(l) for l in range(s.levels - 1)],
            "patches": s.patches()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="runs over the workload's extent to time")
    ap.add_argument("--warmup", type=int, default=1, help="untimed runs before the timed ones")
    ap.add_argument("--workload", default="quad2d_adaptive5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-extra", action="store_true", help="skip the context configurations")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and error report")
    ap.add_argument("--schedule", type=int, default=-1, choices=list(range(-1, 10)),
                    help="force a stage-kernel schedule instead of autotuning over the run")
    ap.add_argument("--scheme", default="mr", choices=["mr", "amr"],
                    help="amr: time the AMR method (MUSCL-Hancock scheme; on the five-level hierarchy also "
                         "the gradient criterion and clustering) instead of the MR scheme; needs --no-cpu")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (counter calibration)")
    ap.add_argument("--cpu-sample", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_sample:   # child process of the single-thread CPU baseline
        upd, sec, steps = cpu_sample(args.cpu_sample, args.cpu_budget)
        print(json.dumps({"updates": upd, "seconds": sec, "steps": steps}))
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)

    if args.scheme == "amr" and not args.no_cpu:
        print("bench.py: --scheme amr needs --no-cpu (the CPU baseline and error report run the MR scheme)",
              file=sys.stderr)
        sys.exit(2)
    if args.scheme == "amr" and args.workload not in AMR_WORKLOADS:
        print(f"bench.py: --scheme amr runs on {', '.join(sorted(AMR_WORKLOADS))}, not {args.workload}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        del a, c

    wl = args.workload
    scheme = 1 if args.scheme == "amr" else 0
    r = Run(wl, args.precision, scheme=scheme)
    if args.schedule >= 0:
        r.s.set_variant(args.schedule)
        r.variant = args.schedule
        r.extent()
        log(f"stage schedule {r.variant} (forced); {r.nsteps} steps per run")
    else:
        every = max(1, (FIXED_STEPS.get(wl) or 400) // 8)
        r.extent(tune_every=every, reps=10 if r.dim == 2 else 3)
        log(f"schedule {r.variant} best over the run {r.tuning}; {r.nsteps} steps per run")
    for _ in range(args.warmup):
        r.timed(1)
    log(f"timing {args.steps} runs of {r.nsteps} steps")
    upd, sec, k = r.timed(args.steps)
    value = upd / sec
    ms_run = 1e3 * sec / k
    log(f"value {value:.4g} cell-updates/s, {ms_run:.3f} ms per run")
    # final state of the last timed run, for the error report
    snap = hierarchy_snapshot(r.s) if wl == "quad2d_adaptive5" and not args.no_cpu else None
    log("stage kernel timed with events over the run")
    roof = roofline(r, args.precision)
    es = 4 if args.precision == "fp32" else 8
    nv = r.dim + 2
    roof["hbm_algorithmic_GBs"] = value * 2 * nv * es / 1e9
    roof["hbm_algorithmic_frac"] = value * 2 * nv * es / 1e9 / HBM_PEAK_GBS
    roof["hbm_algorithmic_note"] = ("whole job, 2 nv s bytes per cell update (read Q^n, write Q^{n+1}); "
                                    "an algorithmic lower bound, not a counter reading")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": k,
        "warmup": args.warmup,
        "ms_per_step": ms_run,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic: seeded inputs (seed 0) shaped like the paper's test problems",
        "config": {"workload": f"{wl}: {WORKLOADS[wl]}" + (
                       "; run with the AMR method: scaled-gradient criterion on density (eps 0.05), "
                       "Berger-Rigoutsos clustering" if scheme and wl == "quad2d_adaptive5" else ""),
                   "precision": args.precision,
                   "step": "one whole run over the workload's extent from the initial state "
                           "(initialisation untimed)",
                   "time_steps_per_run": r.nsteps, "leaf_updates_per_run": upd // k,
                   "stage_schedule": r.variant, "stage_tuning": r.tuning,
                   "scheme": SCHEME_NAMES[scheme]},
        "roofline": roof,
    }
    oracle_h = None
    if not args.no_cpu:
        if wl == "quad2d_adaptive5":
            log("FP64 oracle over the same run (error reference and CPU baseline)")
            oracle_h, o_upd, o_steps, o_sec = adaptive_oracle_run(wl)
            threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
            result["cpu_baseline"] = {
                "value": o_upd / o_sec, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
                "sample": f"FP64 oracle, the whole run ({o_steps} steps, {o_upd} cell updates in {o_sec:.1f} s, "
                          f"OpenMP over cells with {threads} threads)"}
            result["accuracy"] = hierarchy_error(snap, oracle_h)
            result["accuracy"]["oracle_steps"] = o_steps
        else:
            upd1, sec1, steps1 = cpu_sample(wl, 15.0)
            threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
            result["cpu_baseline"] = {"value": upd1 / sec1, "unit": "cell-updates/s", "cores": threads,
                                      "kind": "oracle",
                                      "sample": f"FP64 oracle: first {steps1} steps ({upd1} cell updates in "
                                                f"{sec1:.1f} s, {threads} threads)"}
        log("single-thread CPU baseline")
        result["cpu_baseline_1thread"] = cpu_sample_1thread(wl, 15.0)
    r.close()

    if not args.no_extra:
        log("context configurations")
        ex = {}
        if wl == "quad2d_adaptive5":
            other = "fp64" if args.precision == "fp32" else "fp32"
            err = (lambda rr: hierarchy_error(hierarchy_snapshot(rr.s), oracle_h)) if oracle_h is not None else None
            ex[f"quad2d_adaptive5_{other}"] = extra_line("quad2d_adaptive5", other, 2, after=err)
        ex["quad2d_batch512_fp32"] = extra_line("quad2d_batch512", "fp32", 2, after=batch_error)
        keep = {}
        ex["ellip3d_uniform256_fp32"] = extra_line("ellip3d_uniform256", "fp32", 1,
                                                   after=lambda rr: keep.update(q32=rr.s.level(0)))
        ex["ellip3d_uniform256_fp64"] = extra_line("ellip3d_uniform256", "fp64", 1,
                                                   after=lambda rr: keep.update(q64=rr.s.level(0)))
        ex["ellip3d_uniform256_fp32"]["accuracy"] = uniform_error(
            keep["q32"], keep["q64"], 3, 2.0 / 256,
            "the FP64 GPU path after the same 200 steps (it matches the oracle to 1e-12 at full size, "
            "tests/test_gpu_parity.py)")
        keep.clear()
        ex["ellip3d_uniform256_fp64"]["accuracy"] = {
            "reference": "FP64 oracle: normwise L-inf <= 1e-12 on the first steps at full size "
                         "(tests/test_gpu_parity.py)"}
        ex["ellip3d_adaptive4_lts_fp32"] = extra_line("ellip3d_adaptive4_lts", "fp32", 1)
        ex["quad2d_uniform128_fp64"] = extra_line("quad2d_uniform128", "fp64", 3, after=uniform128_error)
        ex["quad2d_adaptive5_amr_fp32"] = extra_line("quad2d_adaptive5", "fp32", 2, scheme=1)
        ex["quad2d_adaptive5_amr_fp32"]["accuracy"] = {
            "reference": "FP64 oracle on the same method: FP64 bit for bit on 4-level 2D and 3-level 3D runs, "
                         "FP32 L1 <= 1e-5, L-inf <= 2e-3 and flag disagreements <= 2 % per level over 60 steps "
                         "of this hierarchy (tests/test_gpu_clustering.py)"}
        ex["quad2d_batch512_amr_fp32"] = extra_line("quad2d_batch512", "fp32", 2, scheme=1,
                                                    after=lambda rr: batch_error(rr, scheme=1))
        ex["quad2d_uniform128_amr_fp64"] = extra_line("quad2d_uniform128", "fp64", 3, scheme=1,
                                                      after=lambda rr: uniform128_error(rr, scheme=1))
        result["extra"] = ex
    print(json.dumps(result), flush=True)


def batch_error(r, ninst=4, scheme=0):
    """The batch's first instances of the two smallest sides against the
    FP64 oracle over the same 100 steps."""
    import numpy as np
    import oracle as orc
    from paper_1603_05211_amd import inputs
    b = inputs.batch(0)
    order = [i for i in np.argsort(b.sides, kind="stable")][:ninst]
    out = []
    for i in order:
        n = int(b.sides[i])
        h = orc.Hierarchy(2, 1, n, scheme=scheme)
        h.init_finest(orc.init_quadrant(n, 1.4, b.states[i]))
        for _ in range(r.nsteps):
            h.step(0.45)
        g = r.s.level(0, inst=int(i))
        l1, linf = field_errors(g, h.level(0), 2, 1.0 / n)
        out.append({"instance": int(i), "side": n, "l1": l1, "linf_rel": linf})
    return {"sampled_instances": out, "reference": "FP64 oracle, the same 100 steps of those instances"}


def uniform128_error(r, scheme=0):
    import oracle as orc
    from paper_1603_05211_amd import inputs
    h = orc.Hierarchy(2, 1, 128, scheme=scheme)
    h.init_finest(orc.init_quadrant(128, 1.4, inputs.quadrant_states(0)))
    for _ in range(r.nsteps):
        h.step(0.45)
    e = uniform_error(r.s.level(0), h.level(0), 2, 1.0 / 128, "FP64 oracle, the same 100 steps")
    import numpy as np
    e["bit_exact"] = bool(np.array_equal(r.s.level(0), h.level(0)))
    return e


if __name__ == "__main__":
    main()
