"""The strip schedules of the finite-volume update (2D grids of one level:
uniform grids and batches), one stage per launch and both stages fused,
against the FP64 oracle on identical seeded inputs: FP64 bit for bit (the
expression trees are the oracle's), FP32 within the FP32 bound; strips
narrower and wider than the grid, ragged strip rows, outflow and periodic
boundaries, runs past t_end with the fused form's alternating arrays, graph
replay and eager steps."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import (EU_FP32, EU_FP64, EU_STAGE_SCHEDULES, EU_STRIP_SCHEDULE0, EuError,
                                  Solver, inputs)

from gpu_helpers import G, say

pytestmark = pytest.mark.gpu

STRIP = list(range(EU_STRIP_SCHEDULE0, EU_STAGE_SCHEDULES))
FUSED = [v for v in STRIP if v >= EU_STRIP_SCHEDULE0 + 2]


def oracle_uniform(n, prim, steps, bc=0, cfl=0.45, t_end=math.inf):
    h = orc.Hierarchy(2, 1, n, bc=bc)
    h.init_finest(orc.init_quadrant(n, G, prim))
    dts = []
    for _ in range(steps):
        if h.t >= t_end:
            break
        dts.append(h.step(cfl, t_end))
    return h, dts


@pytest.mark.parametrize("var", STRIP)
@pytest.mark.parametrize("seed", [0, 1])
def test_uniform128_fp64_bit_exact(var, seed):
    """128^2 four-quadrant data, 100 steps at CFL 0.45 (full size); step by
    step with the time steps compared, then the state."""
    say("strip uniform 128 fp64 schedule", var, "seed", seed)
    prim = inputs.quadrant_states(seed)
    h, dts = oracle_uniform(128, prim, 100)
    s = Solver(2, n0=128, levels=1, precision=EU_FP64, cfl=0.45)
    s.init_quadrant(prim)
    s.set_variant(var)
    got = []
    for k in range(100):
        s.step(False)
        got.append(s.time()[1])
    assert np.array_equal(np.array(dts), np.array(got))
    assert np.array_equal(s.level(0), h.level(0)), np.abs(s.level(0) - h.level(0)).max()
    assert np.allclose(s.conserved_totals(), h.totals(), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("var", STRIP)
def test_batch_fp64_ragged_sides(var):
    """Sides smaller than a strip, not multiples of the strip width or its
    rows, per-instance time steps; 20 steps replayed from the step graph."""
    sides = [8, 24, 32, 96, 64, 160, 40, 136]
    states = np.stack([inputs.quadrant_states(200 + i) for i in range(len(sides))])
    say("strip batch fp64 schedule", var, "sides", sides)
    s = Solver(2, sides=sides, precision=EU_FP64, cfl=0.45)
    s.init_quadrant_batch(states)
    s.set_variant(var)
    s.advance(20, use_graph=True)
    T = s.conserved_totals()
    for i, n in enumerate(sides):
        h, _ = oracle_uniform(n, states[i], 20)
        Qg = s.level(0, inst=i)
        assert np.array_equal(Qg, h.level(0)), (i, n, np.abs(Qg - h.level(0)).max())
        assert np.allclose(T[i], h.totals(), rtol=1e-13)


@pytest.mark.parametrize("var", STRIP)
def test_fused_alternation_past_t_end(var):
    """A run to t_end and beyond: eager steps, then graph replays of an odd
    number of steps (the fused form's state alternates arrays; steps past
    t_end change nothing)."""
    prim = inputs.quadrant_states(3)
    t_end = 0.05
    h, dts = oracle_uniform(64, prim, 10_000, t_end=t_end)
    say("strip t_end schedule", var, "oracle steps", len(dts))
    s = Solver(2, n0=64, levels=1, precision=EU_FP64, cfl=0.45, t_end=t_end)
    s.init_quadrant(prim)
    s.set_variant(var)
    for _ in range(3):
        s.step(False)
    s.advance(len(dts) - 3 + 5, use_graph=True)
    assert s.time()[0] == h.t
    assert np.array_equal(s.level(0), h.level(0))
    s.advance(3, use_graph=False)
    assert np.array_equal(s.level(0), h.level(0))


def test_periodic_stage_wise_strips_and_fused_rejected():
    """Periodic boundaries wrap across strips: the one-stage strip schedules
    take them (bit for bit); the fused ones do not apply (EU_EINVAL)."""
    prim = inputs.quadrant_states(4)
    h, _ = oracle_uniform(128, prim, 30, bc=orc.BC_PERIODIC, cfl=0.4)
    for var in STRIP:
        s = Solver(2, n0=128, levels=1, precision=EU_FP64, cfl=0.4, bc=1)
        s.init_quadrant(prim)
        if var in FUSED:
            with pytest.raises(EuError) as e:
                s.set_variant(var)
            assert e.value.code == 1
            s.close()
            continue
        say("strip periodic schedule", var)
        s.set_variant(var)
        s.advance(30, use_graph=True)
        assert np.array_equal(s.level(0), h.level(0))
        s.close()


def test_strip_schedules_rejected_on_hierarchies():
    s = Solver(2, n0=32, levels=3, precision=EU_FP64)
    for var in STRIP:
        with pytest.raises(EuError):
            s.set_variant(var)
    t = Solver(3, n0=16, levels=2, precision=EU_FP64, lo=-1.0)
    for var in STRIP:
        with pytest.raises(EuError):
            t.set_variant(var)


def oracle_ellipsoid(n, e, steps, bc=0, cfl=0.4, t_end=math.inf):
    h = orc.Hierarchy(3, 1, n, bc=bc, lo=-1.0, hi=1.0)
    h.init_finest(orc.init_ellipsoid(n, G, e.a, e.b, e.c, e.theta, e.phi, e.states, -1.0, 1.0, e.rc))
    dts = []
    for _ in range(steps):
        if h.t >= t_end:
            break
        dts.append(h.step(cfl, t_end))
    return h, dts


@pytest.mark.parametrize("var", STRIP)
@pytest.mark.parametrize("n", [32, 64])
def test_uniform3d_fp64_bit_exact(var, n):
    """3D strips (8 or 16 rows per workgroup, 32 or 64 planes per strip):
    the ellipsoid blast, step by step with the time steps compared; 64 is
    not a multiple of the strip's 60 columns or its 4 / 12 output rows."""
    e = inputs.ellipsoid(2)
    steps = 12 if n == 32 else 6
    h, dts = oracle_ellipsoid(n, e, steps)
    say("strip 3d fp64 schedule", var, "n", n)
    s = Solver(3, n0=n, levels=1, precision=EU_FP64, cfl=0.4, lo=-1.0, hi=1.0)
    s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    s.set_variant(var)
    got = []
    for _ in range(steps):
        s.step(False)
        got.append(s.time()[1])
    assert np.array_equal(np.array(dts), np.array(got))
    assert np.array_equal(s.level(0), h.level(0)), np.abs(s.level(0) - h.level(0)).max()


@pytest.mark.parametrize("var", [EU_STRIP_SCHEDULE0, EU_STRIP_SCHEDULE0 + 3])
def test_uniform3d_periodic_and_graph(var):
    e = inputs.ellipsoid(4)
    h, _ = oracle_ellipsoid(32, e, 10, bc=orc.BC_PERIODIC)
    s = Solver(3, n0=32, levels=1, precision=EU_FP64, cfl=0.4, lo=-1.0, hi=1.0, bc=1)
    s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    s.set_variant(var)
    s.advance(10, use_graph=True)
    assert np.array_equal(s.level(0), h.level(0))


@pytest.mark.parametrize("var", STRIP)
def test_uniform3d_fp32_within_bound(var):
    e = inputs.ellipsoid(0)
    h, _ = oracle_ellipsoid(32, e, 20)
    s = Solver(3, n0=32, levels=1, precision=EU_FP32, cfl=0.4, lo=-1.0, hi=1.0)
    s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    s.set_variant(var)
    s.advance(20, use_graph=True)
    g, o = s.level(0), h.level(0)
    scale = np.abs(o[0]).sum()
    for f in range(5):
        l1 = np.abs(g[f] - o[f]).sum() / scale
        linf = np.abs(g[f] - o[f]).max() / np.abs(o[f]).max()
        say(f"  3d fp32 schedule {var} field {f}: L1 rel {l1:.2e}, Linf rel {linf:.2e}")
        assert l1 <= 1e-5 and linf <= 1e-3


@pytest.mark.parametrize("var", STRIP)
def test_fp32_within_bound(var):
    """FP32 state and flux against the FP64 oracle: every field's L1 and
    normwise L-inf after 100 steps of the 128^2 workload."""
    prim = inputs.quadrant_states(0)
    h, _ = oracle_uniform(128, prim, 100)
    s = Solver(2, n0=128, levels=1, precision=EU_FP32, cfl=0.45)
    s.init_quadrant(prim)
    s.set_variant(var)
    s.advance(100, use_graph=True)
    g, o = s.level(0), h.level(0)
    vol = (1.0 / 128) ** 2
    for f in range(4):
        l1 = np.abs(g[f] - o[f]).sum() * vol
        l1_rel = l1 / (np.abs(o[f]).sum() * vol)
        linf = np.abs(g[f] - o[f]).max() / np.abs(o[f]).max()
        say(f"  fp32 schedule {var} field {f}: L1 rel {l1_rel:.2e}, Linf rel {linf:.2e}")
        # momenta pass through zero: their L1 is bounded against the density's scale
        assert (l1_rel if f in (0, 3) else l1 / (np.abs(o[0]).sum() * vol)) <= 1e-5
        assert linf <= 1e-3


def test_autotune_and_stage_time_batch_leave_state():
    b = inputs.batch(7, n_instances=12)
    s = Solver(2, sides=list(b.sides), precision=EU_FP32, cfl=0.45)
    s.init_quadrant_batch(b.states)
    s.advance(3)
    before = [s.level(0, inst=i) for i in range(12)]
    var, ms = s.autotune(reps=3)
    say("  batch autotune", var, ms)
    assert len(ms) == EU_STAGE_SCHEDULES and all(m > 0 and m < math.inf for m in ms)
    msp, cells, nl = s.stage_time(reps=3)
    assert cells == 2 * int(sum(int(n) ** 2 for n in b.sides))
    assert nl == (1 if var in FUSED else 2)
    for i in range(12):
        assert np.array_equal(s.level(0, inst=i), before[i])


@pytest.mark.parametrize("var", STRIP)
def test_cfl_partials_from_the_update(var):
    """The launch writing the new state leaves the next step's CFL partials:
    eager steps, fv_step twice without a CFL reduction between (the partials
    are cleared first), an external dt, and the count of cells advanced."""
    prim = inputs.quadrant_states(8)
    n = 64
    h = orc.Hierarchy(2, 1, n)
    h.init_finest(orc.init_quadrant(n, G, prim))
    s = Solver(2, n0=n, levels=1, precision=EU_FP64, cfl=0.45)
    s.init_quadrant(prim)
    s.set_variant(var)
    for k in range(4):
        dt_o = h.step(0.45)
        s.step(False)
        assert s.time()[1] == dt_o
    upd, steps = s.leaf_updates()
    assert steps == 4 and upd == 4 * n * n
    # two updates with the last dt, no reduction between, then the reduction
    dt = s.time()[1]
    import torch
    d = torch.tensor([dt], dtype=torch.float64, device=s.device)
    s.fv_step(dt=d)
    s.fv_step(dt=d)
    h.step_fixed(dt)
    h.step_fixed(dt)
    assert np.array_equal(s.level(0), h.level(0))
    assert s.cfl_dt() == h.cfl(0.45)[0]
