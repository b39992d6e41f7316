"""Shared helpers of the GPU parity tests: build matching oracle / library
runs on identical seeded inputs and compare them."""
import math
import sys

import numpy as np

import oracle as orc
from paper_1603_05211_amd import EU_DT_GLOBAL, EU_DT_LTS, EU_FP32, EU_FP64, Solver, inputs

G = 1.4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dilate(m, r, periodic):
    out = m.copy()
    n = m.shape[0]
    idx = np.arange(n)
    for ax in range(m.ndim):
        acc = np.zeros_like(out)
        for s in range(-r, r + 1):
            j = (idx + s) % n if periodic else np.clip(idx + s, 0, n - 1)
            acc |= np.take(out, j, axis=ax)
        out = acc
    return out


def compare_masks(h, s):
    """Patch membership, flags and the patch table must agree bit for bit."""
    for l in range(h.L):
        a_o, a_g = h.active(l), s.active(l)
        assert np.array_equal(a_o, a_g), f"active mask differs on level {l}: {(a_o != a_g).sum()} cells"
    for l in range(h.L - 1):
        f_o, f_g = h.flags(l), s.flags(l)
        assert np.array_equal(f_o, f_g), f"flags differ on level {l}: {(f_o != f_g).sum()} cells"
    P_o, P_g = h.patches(), s.patches()
    assert np.array_equal(P_o, P_g), f"patch tables differ: {len(P_o)} vs {len(P_g)} rows"


def state_errors(h, s, which=0):
    """Per-level, per-field normwise relative L-inf error over active and ghost
    cells, and the L1 error (cell volume weighted) of each field."""
    periodic = h.bc == orc.BC_PERIODIC
    linf = np.zeros(h.nv)
    l1 = np.zeros(h.nv)
    for l in range(h.L):
        act = h.active(l).astype(bool)
        if not act.any():   # a level with no patch holds no cell to compare
            continue
        mask = act | (dilate(act, 2, periodic) if l > 0 else act)
        Qo = h.level(l) if which == 0 else h.level_stage(l)
        Qg = s.level(l, which)
        vol = h.dx(l) ** h.dim
        for f in range(h.nv):
            o, g = Qo[f][mask], Qg[f][mask]
            scale = max(np.abs(o).max(), 1e-300)
            linf[f] = max(linf[f], np.abs(g - o).max() / scale)
            leaf = h.leaf_mask(l)
            l1[f] += np.abs(Qg[f][leaf] - Qo[f][leaf]).sum() * vol
    return linf, l1


def make_pair(dim, levels, n0, precision=EU_FP64, bc=0, eps=1e-3, lo=None, hi=None, cfl=0.45,
              t_end=math.inf, pmax=32, lts=False, scheme=0, criterion=0, eps_p=0.0):
    lo = (0.0 if dim == 2 else -1.0) if lo is None else lo
    hi = 1.0 if hi is None else hi
    h = orc.Hierarchy(dim, levels, n0, bc=bc, lo=lo, hi=hi, eps=eps, pmax=pmax, scheme=scheme,
                      criterion=criterion, eps_p=eps_p)
    s = Solver(dim, n0=n0, levels=levels, precision=precision, bc=bc, cfl=cfl, t_end=t_end, eps=eps,
               lo=lo, hi=hi, patch_max=pmax, time_mode=EU_DT_LTS if lts else EU_DT_GLOBAL, scheme=scheme,
               criterion=criterion, eps_p=eps_p)
    h.cfl_number = cfl
    h.lts = lts
    return h, s


def init_pair(h, s, kind, seed):
    nf = h.n(h.L - 1)
    if kind == "quadrant":
        prim = inputs.quadrant_states(seed)
        h.init_finest(orc.init_quadrant(nf, G, prim, h.lo, h.hi))
        s.init_quadrant(prim)
    elif kind == "ellipsoid":
        e = inputs.ellipsoid(seed)
        h.init_finest(orc.init_ellipsoid(nf, G, e.a, e.b, e.c, e.theta, e.phi, e.states, h.lo, h.hi, e.rc))
        s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    else:
        raise ValueError(kind)


def run_pair(h, s, steps, t_end=math.inf, regrid=True):
    """Advance both sides step by step (the CFL number the pair was made
    with); return the dt sequences."""
    cfl = h.cfl_number
    dts_o, dts_g = [], []
    for _ in range(steps):
        if h.t >= t_end:
            break
        if getattr(h, "lts", False):
            dts_o.append(h.step_lts(cfl, t_end, regrid=regrid)[0])
        else:
            dts_o.append(h.step(cfl, t_end, regrid=regrid))
        s.step(regrid)
        dts_g.append(s.time()[1])
    return np.array(dts_o), np.array(dts_g)
