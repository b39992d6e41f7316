"""GPU against the FP64 oracle at the edges of the configuration space: every
patch_max (8 .. 64, the largest giving a flagging workgroup 128 cells per
thread in 3D), efficiency thresholds at both ends, eps = 0 (everything
refined), the smallest grids, periodic 3D hierarchies.  Same bar as the
parity tests: FP64 state within 1e-12, masks, flags, patch tables and time
steps bit-exact."""
import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_FP64, Solver

from gpu_helpers import G, compare_masks, init_pair, run_pair, say, state_errors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def pair(dim, levels, n0, pmax=32, eta=0.8, eps=1e-3, bc=orc.BC_TRANSMISSIVE, cfl=0.4):
    lo = 0.0 if dim == 2 else -1.0
    h = orc.Hierarchy(dim, levels, n0, bc=bc, lo=lo, hi=1.0, eps=eps, eta=eta, pmax=pmax)
    s = Solver(dim, n0=n0, levels=levels, precision=EU_FP64, bc=bc, cfl=cfl, eps=eps, eta=eta,
               lo=lo, hi=1.0, patch_max=pmax)
    h.cfl_number = cfl
    h.lts = False
    return h, s


def check(h, s, steps):
    compare_masks(h, s)
    do, dg = run_pair(h, s, steps)
    assert np.array_equal(do, dg)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    say("  linf", linf.max(), "patches", len(h.patches()))
    assert linf.max() <= FP64_TOL


@pytest.mark.parametrize("pmax", [8, 16, 64])
def test_patch_max_2d(pmax):
    say("2d pmax", pmax)
    h, s = pair(2, 3, 32, pmax=pmax)
    init_pair(h, s, "quadrant", 11)
    check(h, s, 4)


@pytest.mark.parametrize("pmax", [8, 16])
def test_patch_max_3d(pmax):
    say("3d pmax", pmax)
    h, s = pair(3, 3, 16, pmax=pmax)
    init_pair(h, s, "ellipsoid", 3)
    check(h, s, 2)


def test_patch_max_64_3d():
    """pmax 64 in 3D: a flagging workgroup covers a 32^3 footprint."""
    say("3d pmax 64")
    h, s = pair(3, 2, 32, pmax=64)
    init_pair(h, s, "ellipsoid", 4)
    check(h, s, 1)


@pytest.mark.parametrize("eta", [0.3, 1.0])
def test_efficiency_threshold(eta):
    say("eta", eta)
    h, s = pair(2, 4, 32, eta=eta)
    init_pair(h, s, "quadrant", 12)
    check(h, s, 3)


def test_eps_zero_refines_everything():
    """eps = 0: every detail is significant, every level is one patch cover."""
    h, s = pair(2, 3, 32, eps=0.0)
    init_pair(h, s, "quadrant", 13)
    for l in range(3):
        assert s.active(l).all()
    check(h, s, 2)


def test_smallest_hierarchy():
    """n0 = 8 (one block on level 0), two levels, patch_max 16."""
    h, s = pair(2, 2, 8, pmax=16)
    init_pair(h, s, "quadrant", 14)
    check(h, s, 5)


def test_per_level_flagging_matches(monkeypatch):
    """One flagging launch per level, forced on a 2D four-level run (by
    default every level is flagged in one launch there): masks, flags, patch
    tables, time steps and state as the oracle's."""
    monkeypatch.setenv("EU_FLAG_BUILD", "levels")
    say("per-level flagging")
    h, s = pair(2, 4, 16)
    init_pair(h, s, "quadrant", 13)
    check(h, s, 4)


def test_periodic_3d_adaptive_single_flag_launch():
    """Periodic 3D hierarchy with patch_max 16: all levels flagged in one
    launch, whose nesting masks wrap around the domain."""
    say("3d periodic pmax 16, four levels")
    h, s = pair(3, 4, 8, pmax=16, bc=orc.BC_PERIODIC)
    init_pair(h, s, "ellipsoid", 6)
    check(h, s, 2)


def test_periodic_3d_adaptive():
    h, s = pair(3, 3, 16, bc=orc.BC_PERIODIC)
    init_pair(h, s, "ellipsoid", 5)
    T0 = s.conserved_totals()
    check(h, s, 3)
    T1 = s.conserved_totals()
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0)))


def test_two_launch_list_build_matches(monkeypatch):
    """The two-launch list build (classification, then compaction), which
    only very large hierarchies reach by themselves, forced on a 2D adaptive
    run: masks, flags, patch tables, time steps and state as the oracle's."""
    monkeypatch.setenv("EU_LIST_BUILD", "2")
    say("two-launch list build")
    h, s = pair(2, 4, 16)
    init_pair(h, s, "quadrant", 13)
    check(h, s, 4)
