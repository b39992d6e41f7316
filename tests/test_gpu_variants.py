"""The MR-scheme variants on the GPU against the FP64 oracle on identical
seeded inputs: Heun's RK2 and AUSM+ with Liou's critical sound speed, on
adaptive hierarchies (2D, 3D), uniform grids, batches and (critical speed)
local time steps; FP64 bit for bit, every tile schedule; the strip
schedules refused."""
import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import (EU_AUSM_CRITICAL, EU_DT_LTS, EU_FP64, EU_RK_HEUN, EU_STAGE_SCHEDULES,
                                  EU_STRIP_SCHEDULE0, EuError, Solver, inputs)

from gpu_helpers import G, compare_masks, say, state_errors

pytestmark = pytest.mark.gpu

VARIANTS = [(1, 0), (0, 1), (1, 1)]


def hpair(dim, L, n0, rk, cs, lts=False, seed=2):
    lo = 0.0 if dim == 2 else -1.0
    cfl = 0.45 if dim == 2 else 0.4
    h = orc.Hierarchy(dim, L, n0, lo=lo, eps=1e-3, pmax=32 if dim == 2 else 16, rk=rk, ausm_speed=cs)
    s = Solver(dim, n0=n0, levels=L, precision=EU_FP64, cfl=cfl, eps=1e-3, lo=lo, patch_max=32 if dim == 2 else 16,
               rk=rk, ausm_speed=cs, time_mode=EU_DT_LTS if lts else 0)
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


@pytest.mark.parametrize("rk,cs", VARIANTS)
@pytest.mark.parametrize("dim,L,n0", [(2, 3, 32), (3, 3, 8)])
def test_hierarchy_fp64(rk, cs, dim, L, n0):
    say("variants hierarchy rk", rk, "cs", cs, "dim", dim)
    h, s, cfl = hpair(dim, L, n0, rk, cs)
    for _ in range(8):
        dt = h.step(cfl)
        s.step(True)
        assert s.time()[1] == dt
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    say("  linf", linf)
    assert linf.max() <= 1e-12


@pytest.mark.parametrize("var", range(EU_STRIP_SCHEDULE0))
def test_every_tile_schedule_heun_critical(var):
    say("variants schedule", var)
    h, s, cfl = hpair(2, 3, 32, 1, 1, seed=4)
    s.set_variant(var)
    for _ in range(5):
        h.step(cfl)
        s.step(True)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= 1e-12


def test_critical_speed_local_time_steps():
    say("variants: critical speed with local time steps")
    h, s, cfl = hpair(2, 3, 32, 0, 1, lts=True, seed=5)
    for _ in range(3):
        dt, _ = h.step_lts(cfl)
        s.step(True)
        assert s.time()[1] == dt
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= 1e-12


def test_batch_heun_critical_and_strips_refused():
    sides = [32, 64, 96]
    states = np.stack([inputs.quadrant_states(50 + i) for i in range(3)])
    s = Solver(2, sides=sides, precision=EU_FP64, cfl=0.45, rk=EU_RK_HEUN, ausm_speed=EU_AUSM_CRITICAL)
    s.init_quadrant_batch(states)
    for var in range(EU_STAGE_SCHEDULES):
        if var >= EU_STRIP_SCHEDULE0:
            with pytest.raises(EuError):
                s.set_variant(var)
    var, ms = s.autotune(reps=2)
    assert var < EU_STRIP_SCHEDULE0
    s.advance(12, use_graph=True)
    for i, n in enumerate(sides):
        h = orc.Hierarchy(2, 1, n, rk=1, ausm_speed=1)
        h.init_finest(orc.init_quadrant(n, G, states[i]))
        for _ in range(12):
            h.step(0.45)
        assert np.array_equal(s.level(0, inst=i), h.level(0)), i


def test_heun_refused_with_local_time_steps():
    with pytest.raises(EuError):
        Solver(2, n0=32, levels=3, time_mode=EU_DT_LTS, rk=EU_RK_HEUN)
