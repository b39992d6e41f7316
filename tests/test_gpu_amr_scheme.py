"""The AMR scheme of Sec. 2 (unsplit MUSCL-Hancock, Minmod, AUSMDV) on the
GPU strip and tile kernels against the FP64 oracle on identical seeded inputs: FP64 bit
for bit (uniform grids, ragged batches, periodic boundaries, runs past t_end
with the alternating state arrays), FP32 within the FP32 bound, and the
schedules that do not apply rejected."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import (EU_FP32, EU_FP64, EU_SCHEME_AMR, EU_STAGE_SCHEDULES, EU_STRIP_SCHEDULE0, EuError,
                                  Solver, inputs)

from gpu_helpers import G, say

pytestmark = pytest.mark.gpu

# Hancock tile kernel (0-2) and Hancock strips (6, 7) on uniform grids; the
# strips only on batches
AMR_SCHEDULES = [0, 1, 2, EU_STRIP_SCHEDULE0, EU_STRIP_SCHEDULE0 + 1]
BATCH_SCHEDULES = [EU_STRIP_SCHEDULE0, EU_STRIP_SCHEDULE0 + 1]


def oracle_amr(n, prim, steps, bc=0, cfl=0.45, t_end=math.inf):
    h = orc.Hierarchy(2, 1, n, bc=bc, scheme=orc.SCHEME_AMR)
    h.init_finest(orc.init_quadrant(n, G, prim))
    dts = []
    for _ in range(steps):
        if h.t >= t_end:
            break
        dts.append(h.step(cfl, t_end))
    return h, dts


@pytest.mark.parametrize("var", AMR_SCHEDULES)
@pytest.mark.parametrize("seed", [0, 1])
def test_uniform128_fp64_bit_exact(var, seed):
    say("amr scheme uniform 128 fp64 schedule", var, "seed", seed)
    prim = inputs.quadrant_states(seed)
    h, dts = oracle_amr(128, prim, 100)
    s = Solver(2, n0=128, levels=1, precision=EU_FP64, cfl=0.45, scheme=EU_SCHEME_AMR)
    s.init_quadrant(prim)
    s.set_variant(var)
    got = []
    for _ in range(100):
        s.step(False)
        got.append(s.time()[1])
    assert np.array_equal(np.array(dts), np.array(got))
    assert np.array_equal(s.level(0), h.level(0)), np.abs(s.level(0) - h.level(0)).max()
    assert np.allclose(s.conserved_totals(), h.totals(), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("var", BATCH_SCHEDULES)
def test_batch_fp64_ragged_sides(var):
    sides = [8, 24, 32, 96, 64, 160, 40, 136]
    states = np.stack([inputs.quadrant_states(300 + i) for i in range(len(sides))])
    say("amr scheme batch fp64 schedule", var)
    s = Solver(2, sides=sides, precision=EU_FP64, cfl=0.45, scheme=EU_SCHEME_AMR)
    s.init_quadrant_batch(states)
    s.set_variant(var)
    s.advance(21, use_graph=True)
    for i, n in enumerate(sides):
        h, _ = oracle_amr(n, states[i], 21)
        Qg = s.level(0, inst=i)
        assert np.array_equal(Qg, h.level(0)), (i, n, np.abs(Qg - h.level(0)).max())


@pytest.mark.parametrize("var", [0, EU_STRIP_SCHEDULE0])
def test_periodic_and_past_t_end(var):
    say("amr scheme periodic and past t_end, schedule", var)
    prim = inputs.quadrant_states(5)
    h, _ = oracle_amr(64, prim, 25, bc=orc.BC_PERIODIC, cfl=0.4)
    s = Solver(2, n0=64, levels=1, precision=EU_FP64, cfl=0.4, bc=1, scheme=EU_SCHEME_AMR)
    s.init_quadrant(prim)
    s.set_variant(var)
    s.advance(25, use_graph=True)
    assert np.array_equal(s.level(0), h.level(0))
    t_end = 0.04
    h, dts = oracle_amr(64, prim, 10_000, t_end=t_end)
    s = Solver(2, n0=64, levels=1, precision=EU_FP64, cfl=0.45, t_end=t_end, scheme=EU_SCHEME_AMR)
    s.init_quadrant(prim)
    s.set_variant(var)
    s.step(False)
    s.advance(len(dts) + 4, use_graph=True)
    assert s.time()[0] == h.t
    assert np.array_equal(s.level(0), h.level(0))


def test_fp32_within_bound():
    prim = inputs.quadrant_states(0)
    h, _ = oracle_amr(128, prim, 100)
    s = Solver(2, n0=128, levels=1, precision=EU_FP32, cfl=0.45, scheme=EU_SCHEME_AMR)
    s.init_quadrant(prim)
    s.advance(100, use_graph=True)
    g, o = s.level(0), h.level(0)
    scale = np.abs(o[0]).sum()
    for f in range(4):
        l1 = np.abs(g[f] - o[f]).sum()
        linf = np.abs(g[f] - o[f]).max() / np.abs(o[f]).max()
        say(f"  amr fp32 field {f}: L1 rel {l1 / scale:.2e}, Linf rel {linf:.2e}")
        assert l1 / scale <= 1e-5 and linf <= 1e-3


def test_schedules_that_do_not_apply():
    s = Solver(2, n0=64, levels=1, precision=EU_FP64, scheme=EU_SCHEME_AMR)
    s.init_quadrant(inputs.quadrant_states(0))
    for var in range(EU_STAGE_SCHEDULES):
        if var in AMR_SCHEDULES:
            s.set_variant(var)
        else:
            with pytest.raises(EuError):
                s.set_variant(var)
    var, ms = s.autotune(reps=3)
    assert var in AMR_SCHEDULES
    assert all((m < math.inf) == (i in AMR_SCHEDULES) for i, m in enumerate(ms))
    ms_, cells, nl = s.stage_time(reps=3)
    assert cells == 64 * 64 and nl == 1
    b = Solver(2, sides=[32, 64], precision=EU_FP64, scheme=EU_SCHEME_AMR)
    b.init_quadrant_batch(np.stack([inputs.quadrant_states(1), inputs.quadrant_states(2)]))
    for var in range(EU_STAGE_SCHEDULES):
        if var in BATCH_SCHEDULES:
            b.set_variant(var)
        else:
            with pytest.raises(EuError):
                b.set_variant(var)
