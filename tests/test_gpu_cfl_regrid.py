"""The CFL signal speed options and the regrid interval on the GPU against
the FP64 oracle: time steps, masks and states bit for bit, on hierarchies
(eager steps, graph runs and regrid cycles, both schemes, local time
steps), a uniform 3D grid on the strip kernels and a batch."""
import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_CFL_MAX, EU_DT_GLOBAL, EU_DT_LTS, EU_FP64, Solver, inputs

from gpu_helpers import G, compare_masks, say, state_errors

pytestmark = pytest.mark.gpu


def pair(L=4, n0=32, every=1, mode=0, scheme=0, lts=False, seed=3, cfl=0.4):
    h = orc.Hierarchy(2, L, n0, eps=1e-3, cfl_mode=mode, regrid_every=every, scheme=scheme)
    s = Solver(2, n0=n0, levels=L, precision=EU_FP64, cfl=cfl, eps=1e-3, cfl_mode=mode, regrid_every=every,
               scheme=scheme, time_mode=EU_DT_LTS if lts else EU_DT_GLOBAL)
    prim = inputs.quadrant_states(seed)
    h.init_finest(orc.init_quadrant(n0 << (L - 1), G, prim))
    s.init_quadrant(prim)
    return h, s


@pytest.mark.parametrize("scheme", [0, 1])
def test_cfl_max_hierarchy(scheme):
    say("cfl max, hierarchy, scheme", scheme)
    h, s = pair(mode=orc.CFL_MAX, scheme=scheme, cfl=0.25)
    for _ in range(6):
        assert h.step(0.25) == (s.step(True), s.time()[1])[1]
    assert s.advance(10, use_graph=True) == 10
    for _ in range(10):
        h.step(0.25)
    assert s.time()[0] == h.t
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= 1e-12


def test_cfl_max_uniform_3d_strips():
    """The strip kernels' CFL epilogue uses the same signal speed (CFL 0.15:
    in 3D the max form gives up to three times the sum form's step)."""
    from paper_1603_05211_amd import EU_STRIP_SCHEDULE0
    say("cfl max, 3D uniform strips")
    e = inputs.ellipsoid(2)
    n = 32
    h = orc.Hierarchy(3, 1, n, lo=-1.0, cfl_mode=orc.CFL_MAX)
    h.init_finest(orc.init_ellipsoid(n, G, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0, e.rc))
    s = Solver(3, n0=n, levels=1, precision=EU_FP64, cfl=0.15, lo=-1.0, cfl_mode=EU_CFL_MAX)
    s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    s.set_variant(EU_STRIP_SCHEDULE0)
    for _ in range(4):
        assert h.step(0.15) == (s.step(True), s.time()[1])[1]
    assert np.isfinite(h.level(0)).all()
    err = np.abs(s.level(0) - h.level(0)).max() / np.abs(h.level(0)).max()
    assert err <= 1e-12


def test_cfl_max_batch():
    say("cfl max, batch")
    sides = [32, 96, 64]
    s = Solver(2, sides=sides, precision=EU_FP64, cfl=0.25, cfl_mode=EU_CFL_MAX)
    states = [inputs.quadrant_states(200 + i) for i in range(len(sides))]
    s.init_quadrant_batch(np.stack(states))
    hs = []
    for i, n in enumerate(sides):
        h = orc.Hierarchy(2, 1, n, cfl_mode=orc.CFL_MAX)
        h.init_finest(orc.init_quadrant(n, G, states[i]))
        hs.append(h)
    for _ in range(3):
        s.step(True)
        for h in hs:
            h.step(0.25)
    for i, h in enumerate(hs):
        err = np.abs(s.level(0, inst=i) - h.level(0)).max() / np.abs(h.level(0)).max()
        assert err <= 1e-12, (i, err)


@pytest.mark.parametrize("every,scheme,graph", [(3, 0, True), (3, 0, False), (3, 1, True), (2, 1, True)])
def test_regrid_interval(every, scheme, graph):
    """Steps 1 .. 17 in calls of 2, 7 and 8 steps: eager steps up to a
    regrid, whole regrid cycles from one graph each, the rest eagerly; with
    the AMR scheme the state alternates between the arrays and an odd cycle
    changes the array."""
    say("regrid every", every, "scheme", scheme, "graph", graph)
    h, s = pair(every=every, scheme=scheme)
    for n in (2, 7, 8):
        assert s.advance(n, use_graph=graph) == n
        for _ in range(n):
            h.step(0.4, regrid=None)
        assert s.time()[0] == h.t
        compare_masks(h, s)
        linf, _ = state_errors(h, s)
        assert linf.max() <= 1e-12, (n, linf)


def test_regrid_interval_lts():
    say("regrid every 2, local time steps")
    h, s = pair(L=3, every=2, lts=True)
    for n in (1, 4):
        assert s.advance(n, use_graph=True) == n
        for _ in range(n):
            h.step_lts(0.4, regrid=None)
        compare_masks(h, s)
        linf, _ = state_errors(h, s)
        assert linf.max() <= 1e-12, (n, linf)
