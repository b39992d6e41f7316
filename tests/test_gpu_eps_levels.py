"""Level-dependent MR thresholds (a variant of the MR criterion) on the GPU
against the FP64 oracle: masks, flags and patch tables bit for bit, states
bit for bit over adaptive runs (2D and 3D), and a new threshold taken again
through eu_mr_flag (the significance kernel)."""
import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_FP64, Solver, inputs

from gpu_helpers import G, compare_masks, say, state_errors

pytestmark = pytest.mark.gpu


def pair(dim, L, n0, eps, **kw):
    lo = 0.0 if dim == 2 else -1.0
    h = orc.Hierarchy(dim, L, n0, lo=lo, eps=eps, eps_levels=True, pmax=32 if dim == 2 else 16)
    s = Solver(dim, n0=n0, levels=L, precision=EU_FP64, cfl=0.45 if dim == 2 else 0.4, eps=eps, lo=lo,
               patch_max=32 if dim == 2 else 16, eps_levels=1, **kw)
    if dim == 2:
        prim = inputs.quadrant_states(1)
        h.init_finest(orc.init_quadrant(n0 << (L - 1), G, prim))
        s.init_quadrant(prim)
    else:
        e = inputs.ellipsoid(2)
        h.init_finest(orc.init_ellipsoid(n0 << (L - 1), G, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0,
                                         e.rc))
        s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    return h, s


@pytest.mark.parametrize("dim,L,n0", [(2, 4, 32), (3, 3, 16)])
def test_level_thresholds_fp64(dim, L, n0):
    say("eps levels fp64", dim, L, n0)
    h, s = pair(dim, L, n0, 1e-3)
    compare_masks(h, s)
    cfl = 0.45 if dim == 2 else 0.4
    for _ in range(8):
        assert h.step(cfl) == (s.step(True), s.time()[1])[1]
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    say("  linf", linf)
    assert linf.max() <= 1e-12


def test_new_threshold_through_mr_flag():
    say("eps levels: eu_mr_flag with a new threshold")
    h, s = pair(2, 4, 32, 1e-3)
    for eps in (4e-3, 3e-4):
        h.step(0.45, regrid=False)
        s.step(False)
        h.set_eps(eps)
        h.regrid()
        s.mr_decompose()
        s.mr_flag(eps)
        compare_masks(h, s)
        linf, _ = state_errors(h, s)
        assert linf.max() <= 1e-12
