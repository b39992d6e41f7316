"""Berger-Rigoutsos clustering (the AMR method's patch generation, Sec. 2.2,
as a variant tiler) on the GPU against the FP64 oracle: masks, flags and the
patch table of rectangles bit for bit, states bit for bit over adaptive runs,
in 2D and 3D, with one and with several patch_max blocks per wave word, with
the MR and the AMR scheme, global and local time steps."""
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_DT_GLOBAL, EU_DT_LTS, EU_FP32, EU_FP64, EU_TILER_BR, Solver, inputs

from gpu_helpers import G, compare_masks, say, state_errors

pytestmark = pytest.mark.gpu


def pair(dim, L, n0, pmax, eta=0.8, bc=0, scheme=0, criterion=0, eps=1e-3, eps_p=0.0, lts=False, seed=3):
    lo = 0.0 if dim == 2 else -1.0
    cfl = 0.45 if dim == 2 else 0.4
    h = orc.Hierarchy(dim, L, n0, lo=lo, eps=eps, eta=eta, bc=bc, pmax=pmax, scheme=scheme, criterion=criterion,
                      eps_p=eps_p, tiler=orc.TILER_BR)
    s = Solver(dim, n0=n0, levels=L, precision=EU_FP64, cfl=cfl, eps=eps, eta=eta, bc=bc, lo=lo, patch_max=pmax,
               scheme=scheme, criterion=criterion, eps_p=eps_p, time_mode=EU_DT_LTS if lts else EU_DT_GLOBAL,
               tiler=EU_TILER_BR)
    h.cfl_number = cfl
    h.lts = lts
    if dim == 2:
        prim = inputs.quadrant_states(seed)
        h.init_finest(orc.init_quadrant(n0 << (L - 1), G, prim))
        s.init_quadrant(prim)
    else:
        e = inputs.ellipsoid(seed)
        h.init_finest(orc.init_ellipsoid(n0 << (L - 1), G, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0,
                                         e.rc))
        s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    return h, s, cfl


def rectangles(P):
    return int(((P[:, 4] != P[:, 5]) | ((P[:, 6] != 1) & (P[:, 6] != P[:, 4]))).sum())


def run(h, s, cfl, steps, lts=False):
    for _ in range(steps):
        if lts:
            h.step_lts(cfl)
            s.step(True)
        else:
            assert h.step(cfl) == (s.step(True), s.time()[1])[1]
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    return linf


@pytest.mark.parametrize("dim,L,n0,pmax,eta,bc", [
    (2, 4, 32, 32, 0.8, 0),     # 4 x 4 blocks per wave, chained flagging
    (2, 4, 32, 64, 0.5, 0),     # 8 x 8 blocks per wave
    (2, 4, 32, 16, 0.9, 1),     # 2 x 2 blocks, periodic
    (3, 3, 16, 16, 0.8, 0),     # 2^3 blocks, chained flagging
    (3, 3, 16, 32, 0.6, 0),     # 4^3 blocks per wave
])
def test_clustering_mr_fp64(dim, L, n0, pmax, eta, bc):
    say("clustering MR fp64", dim, L, n0, pmax, eta, bc)
    h, s, cfl = pair(dim, L, n0, pmax, eta=eta, bc=bc)
    compare_masks(h, s)
    say("  patches", len(h.patches()), "rectangles", rectangles(h.patches()))
    linf = run(h, s, cfl, 6)
    say("  linf", linf, "patches", len(h.patches()), "rectangles", rectangles(h.patches()))
    assert linf.max() <= 1e-12
    if pmax > 16:
        assert rectangles(h.patches()) > 0


@pytest.mark.parametrize("dim,L,n0,pmax", [(2, 4, 32, 32), (3, 3, 16, 16)])
def test_clustering_amr_gradient_fp64(dim, L, n0, pmax):
    say("clustering AMR scheme, gradient criterion", dim, L, n0, pmax)
    h, s, cfl = pair(dim, L, n0, pmax, scheme=orc.SCHEME_AMR, criterion=orc.CRIT_GRADIENT, eps=0.05, eps_p=0.05,
                     seed=4)
    compare_masks(h, s)
    linf = run(h, s, cfl, 5)
    say("  linf", linf, "patches", len(h.patches()))
    assert linf.max() <= 1e-12


@pytest.mark.parametrize("scheme", [0, 1])
def test_clustering_lts_fp64(scheme):
    """MRLT, and AMRLT with the gradient criterion (the AMR method's own
    configuration), clustered."""
    say("clustering with local time steps, scheme", scheme)
    if scheme == 0:
        h, s, cfl = pair(2, 4, 32, 32, lts=True, seed=5)
    else:
        h, s, cfl = pair(2, 4, 32, 32, lts=True, seed=5, scheme=orc.SCHEME_AMR, criterion=orc.CRIT_GRADIENT,
                         eps=0.05, eps_p=0.05)
    linf = run(h, s, cfl, 2, lts=True)
    say("  linf", linf, "patches", len(h.patches()))
    assert linf.max() <= 1e-12


def test_amr_method_headline_hierarchy_fp32():
    """The AMR method as benchmarked on the five-level hierarchy (32^2 ..
    512^2): AMR scheme, scaled-gradient criterion on density (eps 0.05),
    Berger-Rigoutsos clustering, FP32, 60 steps against the FP64 oracle:
    every field's L1 (relative to the density's) within 1e-5 and normwise
    L-inf within 2e-3 on the composite, flag disagreements at most 2 % per
    level."""
    import numpy as np

    say("clustering: AMR method fp32, headline hierarchy, 60 steps")
    h = orc.Hierarchy(2, 5, 32, eps=0.05, eta=0.8, pmax=32, scheme=orc.SCHEME_AMR, criterion=orc.CRIT_GRADIENT,
                      tiler=orc.TILER_BR)
    s = Solver(2, n0=32, levels=5, precision=EU_FP32, cfl=0.45, eps=0.05, eta=0.8, patch_max=32,
               scheme=orc.SCHEME_AMR, criterion=orc.CRIT_GRADIENT, tiler=EU_TILER_BR)
    prim = inputs.quadrant_states(0)
    h.init_finest(orc.init_quadrant(512, G, prim))
    s.init_quadrant(prim)
    for _ in range(60):
        h.step(0.45)
    assert s.advance(60, use_graph=True) == 60
    g, o = s.composite(), h.composite()
    scale = np.abs(o[0]).sum()
    l1 = [float(np.abs(g[f] - o[f]).sum() / scale) for f in range(4)]
    linf = [float(np.abs(g[f] - o[f]).max() / np.abs(o[f]).max()) for f in range(4)]
    say("  L1 rel", l1, "Linf rel", linf, "patches", len(h.patches()), len(s.patches()))
    assert max(l1) <= 1e-5 and max(linf) <= 2e-3
    for l in range(h.L - 1):
        fo, fg = h.flags(l).astype(bool), s.flags(l).astype(bool)
        dis = int((fo != fg).sum())
        say(f"  level {l}: flagged {int(fo.sum())}, disagreements {dis}")
        assert dis <= max(2, 0.02 * fo.sum())


def test_amr_method_3d_fp32():
    """The AMR method in 3D (scaled gradients of density and pressure, eps
    0.05 each, clustering with 4^3 blocks per pmax block) in FP32 for 12
    steps against the FP64 oracle: every field's L1 (relative to the
    density's) within 1e-5, normwise L-inf within 2e-3 on the composite, flag
    disagreements at most 2 % per level."""
    import numpy as np

    say("clustering: AMR method fp32, 3D")
    e = inputs.ellipsoid(6)
    h = orc.Hierarchy(3, 3, 16, lo=-1.0, eps=0.05, eta=0.8, pmax=32, scheme=orc.SCHEME_AMR,
                      criterion=orc.CRIT_GRADIENT, eps_p=0.05, tiler=orc.TILER_BR)
    s = Solver(3, n0=16, levels=3, precision=EU_FP32, cfl=0.4, eps=0.05, eta=0.8, lo=-1.0, patch_max=32,
               scheme=orc.SCHEME_AMR, criterion=orc.CRIT_GRADIENT, eps_p=0.05, tiler=EU_TILER_BR)
    h.init_finest(orc.init_ellipsoid(64, G, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0, e.rc))
    s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    for _ in range(12):
        h.step(0.4)
    assert s.advance(12, use_graph=True) == 12
    g, o = s.composite(), h.composite()
    scale = np.abs(o[0]).sum()
    l1 = [float(np.abs(g[f] - o[f]).sum() / scale) for f in range(5)]
    linf = [float(np.abs(g[f] - o[f]).max() / np.abs(o[f]).max()) for f in range(5)]
    say("  L1 rel", l1, "Linf rel", linf, "patches", len(h.patches()), len(s.patches()))
    assert max(l1) <= 1e-5 and max(linf) <= 2e-3
    for l in range(h.L - 1):
        fo, fg = h.flags(l).astype(bool), s.flags(l).astype(bool)
        dis = int((fo != fg).sum())
        say(f"  level {l}: flagged {int(fo.sum())}, disagreements {dis}")
        assert dis <= max(2, 0.02 * fo.sum())
