"""Error assessment of the adaptive computations (Sec. 3) on one GPU.

The paper measures its adaptive runs against a fine reference solution of
its own: the L1 error of the density on the finest grid of a run (the
reference projected onto it by cell means), the accuracy perturbation
against the uniform finest-grid FV run, memory and mesh compression (the
average number of cells of the whole hierarchy, and of leaves, over the
time steps, per cell of the finest uniform grid), CPU-time compression and
the overhead per leaf, Gamma^a / Gamma^FV - 1.  This module computes the same
measures with the library: the reference is a uniform FP64 run of the AMR
scheme on a fine grid, as in Sec. 4.1; the runs are the discretizations of
Sec. 2 (MR-FV, MR, MRLT, AMR-FV, AMR, AMRLT); "CPU time" is the GPU time of
the run.

    python -m paper_1603_05211_amd.study [--levels 4 5 6] [--ref 4096]
    python -m paper_1603_05211_amd.study --3d [--levels 3 4 5] [--ref 1024]

prints one JSON object (and a markdown table on stderr).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import (EU_CRIT_GRADIENT, EU_CRIT_MR, EU_DT_GLOBAL, EU_DT_LTS, EU_FP64, EU_SCHEME_AMR, EU_SCHEME_MR,
               EU_TILER_BLOCKS, EU_TILER_BR, Solver, inputs)

# ----------------------------------------------------------------------------
# the measures of Sec. 3
# ----------------------------------------------------------------------------


def project(Q: np.ndarray, n: int) -> np.ndarray:
    """Cell means of an (nv, N, N[, N]) array on the coarser n-grid (N a
    power-of-two multiple of n): the reference projected onto a run's grid."""
    dim = Q.ndim - 1
    k = Q.shape[-1] // n
    if k == 1:
        return Q.copy()
    shape = (Q.shape[0],) + sum(((n, k) for _ in range(dim)), ())
    axes = tuple(range(2, 2 + 2 * dim, 2))
    return Q.reshape(shape).mean(axis=axes)


def l1_error(rho: np.ndarray, rho_ref: np.ndarray, lo: float = 0.0, hi: float = 1.0) -> float:
    """L1 norm of the density error on the domain: sum |rho - rho_ref| dx^d."""
    dx = (hi - lo) / rho.shape[-1]
    return float(np.abs(rho - rho_ref).sum() * dx ** rho.ndim)


def memory_compression(cells_per_step, n_finest_cells: int) -> float:
    """Average number of cells of the whole hierarchy over the time steps,
    per cell of the finest uniform grid."""
    return float(np.mean(cells_per_step)) / n_finest_cells


def mesh_compression(leaves_per_step, n_finest_cells: int) -> float:
    """Average number of leaves over the time steps, per cell of the finest
    uniform grid."""
    return float(np.mean(leaves_per_step)) / n_finest_cells


def time_compression(t_adaptive: float, t_fv: float) -> float:
    return t_adaptive / t_fv


def accuracy_perturbation(e_fv: float, e_adaptive: float) -> float:
    """|L1^FV - L1^a| / L1^FV."""
    return abs(e_fv - e_adaptive) / e_fv


def overhead(t_adaptive: float, leaf_steps_adaptive: float, t_fv: float, leaf_steps_fv: float) -> float:
    """Gamma^a / Gamma^FV - 1, Gamma = time / sum over time steps of the leaves."""
    return (t_adaptive / leaf_steps_adaptive) / (t_fv / leaf_steps_fv) - 1.0


# ----------------------------------------------------------------------------
# runs
# ----------------------------------------------------------------------------


def _timed_run(make, init, t_end: float, log=None, once=False):
    """A run to t_end replayed from the step graph, timed between two device
    synchronisations: one untimed run first (in chunks of 64 steps, until a
    chunk ends early: steps past t_end do nothing but still launch) counts
    the steps, then the timed run replays exactly that many.  log: called
    with the step count after every chunk of the untimed run.  once: the
    chunked run alone, its time taken around it (references)."""
    import torch
    s = make()
    init(s)
    s.autotune(reps=3)
    if once:
        init(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while True:
        k = s.advance(64, use_graph=True)
        steps += k
        if log is not None:
            log(f"    {steps} steps, t = {s.time()[0]:.4f}")
        if k < 64:
            break
    if once:
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0, steps
    init(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = s.advance(steps, use_graph=True)
    torch.cuda.synchronize()
    if done != steps:
        raise RuntimeError(f"timed run took {done} steps, the first {steps}")
    return s, time.perf_counter() - t0, steps


def _history(s, init, t_end: float, lts_substeps: int):
    """Leaves and cells of the whole hierarchy at every time step (eager
    steps; untimed); finest-level time steps are counted for local time
    stepping (each level-0 step holds lts_substeps of them)."""
    init(s)
    leaves, cells = [], []
    while s.time()[0] < t_end:
        lv, ac = s.counters()
        leaves += [int(lv.sum())] * lts_substeps
        cells += [int(ac.sum())] * lts_substeps
        s.step(True)
    return leaves, cells


ADAPTIVE = ("MR", "MRLT", "AMR", "AMRLT")


def run_study(levels=(4, 5, 6), n0: int = 32, n_ref: int = 4096, t_end: float = 0.25, cfl: float = 0.45,
              eps: float = 0.0023, eps_grad: float = 0.05, prim=None, log=None) -> dict:
    """Lax-Liu configuration #6 (Table 1, the default) on [0,1]^2 with
    outflow boundaries to t_end: a uniform FP64 reference of the AMR scheme
    on n_ref^2, then for every number of levels L (finest grid N = n0
    2^(L-1)) the six discretizations of Sec. 2, all FP64: MR-FV and AMR-FV
    (the MR and AMR schemes on the uniform N^2 grid), MR (MR scheme, MR
    criterion eps, global step), MRLT (the same with local time steps), AMR
    (AMR scheme, scaled-gradient criterion on density eps_grad,
    Berger-Rigoutsos clustering, global step) and AMRLT (the same with local
    time steps); the MR runs tile with the block tiler.  Accuracy
    perturbation and time compression of an adaptive run are taken against
    the uniform run of its scheme."""
    log = log or (lambda *a: None)
    prim = inputs.lax_liu_6() if prim is None else prim
    init = lambda s: s.init_quadrant(prim)
    log(f"reference: AMR scheme, uniform {n_ref}^2, FP64")
    ref, t_ref, steps_ref = _timed_run(
        lambda: Solver(2, n0=n_ref, levels=1, precision=EU_FP64, cfl=cfl, t_end=t_end, scheme=EU_SCHEME_AMR),
        init, t_end, log, once=True)
    rho_ref = ref.level(0)[0].copy()   # drops the other fields
    ref.close()
    out = {"problem": "Lax-Liu configuration #6 (Table 1), [0,1]^2, outflow, t_end %g" % t_end,
           "reference": {"scheme": "AMR (MUSCL-Hancock, Minmod, AUSMDV)", "n": n_ref, "steps": steps_ref,
                         "gpu_s": t_ref},
           "cfl": cfl, "runs": []}
    for L in levels:
        N = n0 << (L - 1)
        NC = N * N
        rr = project(rho_ref[None], N)[0]
        row = {"levels": L, "N": N}
        for name, sch in (("MR-FV", EU_SCHEME_MR), ("AMR-FV", EU_SCHEME_AMR)):
            log(f"L = {L}: {name} {N}^2")
            fv, t_fv, steps_fv = _timed_run(
                lambda: Solver(2, n0=N, levels=1, precision=EU_FP64, cfl=cfl, t_end=t_end, scheme=sch), init, t_end)
            row[name] = {"l1": l1_error(fv.level(0)[0], rr), "gpu_s": t_fv, "steps": steps_fv}
            fv.close()
        variants = (("MR", EU_SCHEME_MR, EU_CRIT_MR, eps, EU_DT_GLOBAL, "MR-FV", EU_TILER_BLOCKS),
                    ("MRLT", EU_SCHEME_MR, EU_CRIT_MR, eps, EU_DT_LTS, "MR-FV", EU_TILER_BLOCKS),
                    ("AMR", EU_SCHEME_AMR, EU_CRIT_GRADIENT, eps_grad, EU_DT_GLOBAL, "AMR-FV", EU_TILER_BR),
                    ("AMRLT", EU_SCHEME_AMR, EU_CRIT_GRADIENT, eps_grad, EU_DT_LTS, "AMR-FV", EU_TILER_BR))
        for name, sch, crit, e, tm, base, tiler in variants:
            log(f"  {name}")
            mk = lambda: Solver(2, n0=n0, levels=L, precision=EU_FP64, cfl=cfl, t_end=t_end, eps=e, eta=0.8,
                                patch_max=32, time_mode=tm, scheme=sch, criterion=crit, tiler=tiler)
            s, t_a, steps_a = _timed_run(mk, init, t_end)
            e_a = l1_error(s.composite()[0], rr)
            sub = 2 ** (L - 1) if tm == EU_DT_LTS else 1
            leaves, cells = _history(s, init, t_end, sub)
            s.close()
            leaf_steps = float(np.sum(leaves))
            fv = row[base]
            row[name] = {"threshold": e, "l1": e_a, "gpu_s": t_a, "steps": steps_a,
                         "finest_steps": len(leaves),
                         "accuracy_perturbation": accuracy_perturbation(fv["l1"], e_a),
                         "memory_compression": memory_compression(cells, NC),
                         "mesh_compression": mesh_compression(leaves, NC),
                         "time_compression": time_compression(t_a, fv["gpu_s"]),
                         "overhead": overhead(t_a, leaf_steps, fv["gpu_s"], float(NC) * fv["steps"])}
        out["runs"].append(row)
    for k in range(1, len(out["runs"])):
        a, b = out["runs"][k - 1], out["runs"][k]
        for name in ("MR-FV", "AMR-FV") + ADAPTIVE:
            b[name]["rate"] = math.log2(a[name]["l1"] / b[name]["l1"])
    return out


ADAPTIVE_3D = ("MR", "MRLT", "AMR", "AMRLT")


def run_study_3d(levels=(3, 4, 5), n0: int = 32, n_ref: int = 1024, t_end: float = 0.28, cfl: float = 0.4,
                 eps: float = 0.013, eps_grad: float = 0.05, log=None) -> dict:
    """The 3D ellipsoidal shock of Sec. 4.2 as printed (inputs.paper_ellipsoid:
    Omega = [-2,2]^3, outflow, t_e = 0.28, r_c = 3/5, a = 1/3, b = 1, c = 3,
    the printed densities and energy densities): a uniform FP64 reference of
    the MR scheme on n_ref^3, then for every number of levels L (finest grid
    N = n0 2^(L-1)) the six discretizations, all FP64: MR-FV and AMR-FV on
    the uniform N^3 grid, MR and MRLT (MR criterion eps = 0.013, the paper's
    3D threshold), AMR and AMRLT (scaled gradients of density and pressure,
    eps_grad = 0.05 each, the paper's 3D thresholds; Berger-Rigoutsos
    clustering)."""
    log = log or (lambda *a: None)
    e = inputs.paper_ellipsoid()
    lo, hi = -2.0, 2.0
    init = lambda s: s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    log(f"reference: MR scheme, uniform {n_ref}^3, FP64")
    ref, t_ref, steps_ref = _timed_run(
        lambda: Solver(3, n0=n_ref, levels=1, precision=EU_FP64, cfl=cfl, t_end=t_end, lo=lo, hi=hi), init, t_end,
        log, once=True)
    log(f"  {steps_ref} steps in {t_ref:.1f} s")
    rho_ref = ref.level(0)[0].copy()   # drops the other fields
    ref.close()
    out = {"problem": "3D ellipsoidal shock (Sec. 4.2, initial data as printed), [-2,2]^3, outflow, t_end %g"
                      % t_end,
           "reference": {"scheme": "MR (MUSCL, van Albada, AUSM+, RK2)", "n": n_ref, "steps": steps_ref,
                         "gpu_s": t_ref},
           "cfl": cfl, "runs": []}
    for L in levels:
        N = n0 << (L - 1)
        NC = N ** 3
        rr = project(rho_ref[None], N)[0]
        row = {"levels": L, "N": N}
        for name, sch in (("MR-FV", EU_SCHEME_MR), ("AMR-FV", EU_SCHEME_AMR)):
            log(f"L = {L}: {name} {N}^3")
            fv, t_fv, steps_fv = _timed_run(
                lambda: Solver(3, n0=N, levels=1, precision=EU_FP64, cfl=cfl, t_end=t_end, lo=lo, hi=hi, scheme=sch),
                init, t_end, log)
            row[name] = {"l1": l1_error(fv.level(0)[0], rr, lo, hi), "gpu_s": t_fv, "steps": steps_fv}
            fv.close()
        variants = (("MR", EU_SCHEME_MR, EU_CRIT_MR, eps, 0.0, EU_DT_GLOBAL, "MR-FV", EU_TILER_BLOCKS),
                    ("MRLT", EU_SCHEME_MR, EU_CRIT_MR, eps, 0.0, EU_DT_LTS, "MR-FV", EU_TILER_BLOCKS),
                    ("AMR", EU_SCHEME_AMR, EU_CRIT_GRADIENT, eps_grad, eps_grad, EU_DT_GLOBAL, "AMR-FV", EU_TILER_BR),
                    ("AMRLT", EU_SCHEME_AMR, EU_CRIT_GRADIENT, eps_grad, eps_grad, EU_DT_LTS, "AMR-FV", EU_TILER_BR))
        for name, sch, crit, e_r, e_p, tm, base, tiler in variants:
            log(f"  {name}")
            mk = lambda: Solver(3, n0=n0, levels=L, precision=EU_FP64, cfl=cfl, t_end=t_end, eps=e_r, eta=0.8,
                                patch_max=32, time_mode=tm, lo=lo, hi=hi, scheme=sch, criterion=crit, eps_p=e_p,
                                tiler=tiler)
            s, t_a, steps_a = _timed_run(mk, init, t_end, log)
            e_a = l1_error(s.composite()[0], rr, lo, hi)
            sub = 2 ** (L - 1) if tm == EU_DT_LTS else 1
            leaves, cells = _history(s, init, t_end, sub)
            s.close()
            f = row[base]
            row[name] = {"threshold": e_r, "l1": e_a, "gpu_s": t_a, "steps": steps_a, "finest_steps": len(leaves),
                         "accuracy_perturbation": accuracy_perturbation(f["l1"], e_a),
                         "memory_compression": memory_compression(cells, NC),
                         "mesh_compression": mesh_compression(leaves, NC),
                         "time_compression": time_compression(t_a, f["gpu_s"]),
                         "overhead": overhead(t_a, float(np.sum(leaves)), f["gpu_s"], float(NC) * f["steps"])}
        out["runs"].append(row)
    for k in range(1, len(out["runs"])):
        a, b = out["runs"][k - 1], out["runs"][k]
        for name in ("MR-FV", "AMR-FV") + ADAPTIVE_3D:
            b[name]["rate"] = math.log2(a[name]["l1"] / b[name]["l1"])
    return out


def markdown(res: dict) -> str:
    rows = ["| L | N | run | L1(rho) | rate | accuracy perturbation | memory | mesh | GPU-time compression | "
            "overhead | GPU s |", "|---:|---:|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in res["runs"]:
        first = True
        for name in ("MR-FV", "AMR-FV") + ADAPTIVE:
            if name not in r:
                continue
            a = r[name]
            lead = f"| {r['levels']} | {r['N']} |" if first else "| | |"
            first = False
            rate = f"{a['rate']:.2f}" if "rate" in a else ""
            if name.endswith("FV"):
                rows.append(f"{lead} {name} | {a['l1']:.6f} | {rate} | | | | | | {a['gpu_s']:.3f} |")
            else:
                rows.append(f"{lead} {name} | {a['l1']:.6f} | {rate} | {a['accuracy_perturbation']:.3f} | "
                            f"{a['memory_compression']:.3f} | {a['mesh_compression']:.3f} | "
                            f"{a['time_compression']:.3f} | {a['overhead']:.2f} | {a['gpu_s']:.3f} |")
    return "\n".join(rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--levels", type=int, nargs="+", default=[4, 5, 6])
    ap.add_argument("--n0", type=int, default=32)
    ap.add_argument("--ref", type=int, default=4096)
    ap.add_argument("--t-end", type=float, default=0.25)
    ap.add_argument("--eps", type=float, default=0.0023)
    ap.add_argument("--eps-grad", type=float, default=0.05)
    ap.add_argument("--3d", dest="three", action="store_true",
                    help="the 3D ellipsoidal shock instead (defaults --levels 3 4 5 --ref 1024 --t-end 0.28 "
                         "--eps 0.013)")
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    if a.three:
        given = lambda name: any(x == name or x.startswith(name + "=") for x in (argv or sys.argv[1:]))
        res = run_study_3d(tuple(a.levels) if given("--levels") else (3, 4, 5), a.n0,
                           a.ref if given("--ref") else 1024, a.t_end if given("--t-end") else 0.28,
                           eps=a.eps if given("--eps") else 0.013, eps_grad=a.eps_grad, log=log)
        log(markdown(res))
        print(json.dumps(res), flush=True)
        return
    res = run_study(tuple(a.levels), a.n0, a.ref, a.t_end, eps=a.eps, eps_grad=a.eps_grad, log=log)
    log(markdown(res))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
