"""Every stage-kernel schedule gives bit-identical FP64 results (FP32 ones
agree to rounding), and the autotuner and the stage timer leave the state
untouched."""
import numpy as np
import pytest

from paper_1603_05211_amd import EU_DT_LTS, EU_FP32, EU_FP64, EU_STAGE_SCHEDULES, EU_STRIP_SCHEDULE0, Solver, inputs

from gpu_helpers import init_pair, make_pair, say

pytestmark = pytest.mark.gpu


def _run(dim, lts, variant, precision=EU_FP64, steps=4):
    h, s = make_pair(dim, 3, 16 if dim == 3 else 32, precision=precision, cfl=0.4, lts=lts)
    init_pair(h, s, "ellipsoid" if dim == 3 else "quadrant", 5)
    s.set_variant(variant)
    s.advance(steps, use_graph=True)
    return [s.level(l) for l in range(3)], [s.active(l) for l in range(3)]


@pytest.mark.parametrize("dim,lts", [(2, False), (3, False), (2, True), (3, True)])
def test_schedules_bit_identical(dim, lts):
    ref_q, ref_a = _run(dim, lts, 0)
    for var in range(1, EU_STRIP_SCHEDULE0):   # the tile schedules (the strip ones need one level)
        q, a = _run(dim, lts, var)
        for l in range(3):
            assert np.array_equal(a[l], ref_a[l]), (var, l)
            act = ref_a[l].astype(bool)
            assert np.array_equal(q[l][:, act], ref_q[l][:, act]), (dim, lts, var, l)


def test_fp32_schedules_agree():
    """FP32 kernels may contract multiply-adds differently per schedule, so
    schedules agree to FP32 rounding, not bit for bit."""
    ref_q, ref_a = _run(2, False, 0, precision=EU_FP32)
    for var in range(1, EU_STRIP_SCHEDULE0):
        q, a = _run(2, False, var, precision=EU_FP32)
        for l in range(3):
            act = ref_a[l].astype(bool) & a[l].astype(bool)
            rel = np.abs(q[l][0][act] - ref_q[l][0][act]).sum() / np.abs(ref_q[l][0][act]).sum()
            assert rel <= 1e-6, (var, l, rel)


def test_autotune_leaves_state_and_picks_a_schedule():
    s = Solver(2, n0=32, levels=4, precision=EU_FP32, cfl=0.45, t_end=0.25)
    s.init_quadrant(inputs.quadrant_states(0))
    s.advance(3)
    before = [s.level(l) for l in range(4)]
    var, ms = s.autotune(reps=5)
    say("  autotune", var, ms)
    assert 0 <= var < EU_STRIP_SCHEDULE0 and len(ms) == EU_STAGE_SCHEDULES
    assert all(0 < m < float("inf") for m in ms[:EU_STRIP_SCHEDULE0])
    assert all(m == float("inf") for m in ms[EU_STRIP_SCHEDULE0:])
    for l in range(4):
        assert np.array_equal(s.level(l), before[l])
    t = Solver(2, n0=32, levels=4, precision=EU_FP32, cfl=0.45, t_end=0.25)
    t.init_quadrant(inputs.quadrant_states(0))
    t.advance(3)
    t.set_variant(var)
    s.advance(5)
    t.advance(5)
    for l in range(4):
        assert np.array_equal(s.level(l), t.level(l))


@pytest.mark.parametrize("lts", [False, True])
def test_stage_time_leaves_state_and_counts_cells(lts):
    """The event-timed passes change nothing, and the cell-stages they report
    are both stages of the leaves (global step, two launches) or the first
    stage of the patch cells (local time stepping, one launch per level)."""
    if lts:
        s = Solver(3, n0=16, levels=3, precision=EU_FP32, cfl=0.4, lo=-1.0, hi=1.0, time_mode=EU_DT_LTS)
        e = inputs.ellipsoid(0)
        s.init_ellipsoid(e.a, e.b, e.c, e.theta, e.phi, e.states, e.rc)
    else:
        s = Solver(2, n0=32, levels=4, precision=EU_FP32, cfl=0.45, t_end=0.25)
        s.init_quadrant(inputs.quadrant_states(0))
    s.advance(2)
    before = [s.level(l) for l in range(s.levels)]
    ms, cells, nl = s.stage_time(reps=4)
    say("  stage_time", ms, cells, nl)
    assert ms > 0 and nl == (s.levels if lts else 2)
    leaves, active = s.counters()
    assert cells == (int(active.sum()) if lts else 2 * int(leaves.sum()))
    for l in range(s.levels):
        assert np.array_equal(s.level(l), before[l])
