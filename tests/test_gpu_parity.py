"""GPU (gfx950 HIP, through the C-ABI) against the FP64 oracle on identical
seeded inputs.

Bar: FP64 state within normwise relative L-inf 1e-12 (the expression trees are
the same, so agreement is expected to be bit for bit), time steps, patch
membership, refinement flags and patch tables bit-exact.  FP32 runs report
their error against the FP64 oracle and must keep the density's relative L1
error within 1e-5 after the run: FP32 unit roundoff is 6e-8, an update
accumulates O(10) roundings per stage and the error grows at most linearly
over the 20-100 steps of these runs, so 1e-5 leaves two decades of margin,
while a dropped term or a transposed operand exceeds it by far.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_FP32, EU_FP64, EuError, Solver, inputs

from gpu_helpers import G, compare_masks, dilate, init_pair, make_pair, run_pair, say, state_errors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_uniform2d_fp64_128_100steps(seed):
    """2D four-quadrant data, 128^2, 100 steps at CFL 0.45 (full size)."""
    say("uniform2d fp64 128^2 seed", seed)
    h, s = make_pair(2, 1, 128)
    init_pair(h, s, "quadrant", seed)
    do, dg = run_pair(h, s, 100)
    assert np.array_equal(do, dg)
    linf, _ = state_errors(h, s)
    say("  linf", linf)
    assert linf.max() <= FP64_TOL
    To, Tg = h.totals(), s.conserved_totals()
    assert np.allclose(Tg, To, rtol=1e-13, atol=1e-15)


def test_uniform3d_fp64_small():
    say("uniform3d fp64 32^3")
    h, s = make_pair(3, 1, 32, cfl=0.4)
    init_pair(h, s, "ellipsoid", 0)
    do, dg = run_pair(h, s, 12)
    assert np.array_equal(do, dg)
    linf, _ = state_errors(h, s)
    say("  linf", linf)
    assert linf.max() <= FP64_TOL


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adaptive2d_fp64(seed):
    """4 levels 32^2..256^2, eps 1e-3: hierarchy, flags, patches bit-exact."""
    say("adaptive2d fp64 seed", seed)
    h, s = make_pair(2, 4, 32)
    init_pair(h, s, "quadrant", seed)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL
    for k in range(3):
        do, dg = run_pair(h, s, 5)
        assert np.array_equal(do, dg)
        compare_masks(h, s)
        linf, _ = state_errors(h, s)
        say("  after", 5 * (k + 1), "steps linf", linf.max(), "patches", len(h.patches()))
        assert linf.max() <= FP64_TOL
    for l in range(h.L - 1):
        assert np.array_equal(h.details(l), s.details(l))
    lo_, ao = h.counts()
    lg, ag = s.counters()
    assert np.array_equal(lo_, lg) and np.array_equal(ao, ag)
    assert np.allclose(s.conserved_totals(), h.totals(), rtol=1e-13)


def test_adaptive2d_fp64_periodic_conservation():
    say("adaptive2d fp64 periodic")
    h, s = make_pair(2, 3, 32, bc=orc.BC_PERIODIC, cfl=0.4)
    init_pair(h, s, "quadrant", 6)
    T0 = s.conserved_totals()
    do, dg = run_pair(h, s, 12)
    assert np.array_equal(do, dg)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL
    T1 = s.conserved_totals()
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0)))


def test_adaptive3d_fp64():
    say("adaptive3d fp64 16^3..64^3")
    h, s = make_pair(3, 3, 16, cfl=0.4)
    init_pair(h, s, "ellipsoid", 1)
    compare_masks(h, s)
    do, dg = run_pair(h, s, 6)
    assert np.array_equal(do, dg)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    say("  linf", linf, "patches", len(h.patches()))
    assert linf.max() <= FP64_TOL


def test_stage_state_fp64():
    """The RK2 intermediate state Q* (after projection and ghost fill)."""
    h, s = make_pair(2, 3, 32)
    init_pair(h, s, "quadrant", 3)
    dt = h.cfl(0.45)[0]
    h.stage(1, dt)
    s.cfl_dt()
    s.fv_step()
    linf, _ = state_errors(h, s, which=1)
    assert linf.max() <= FP64_TOL


def test_graph_replay_equals_eager():
    a = Solver(2, n0=32, levels=3, precision=EU_FP64)
    b = Solver(2, n0=32, levels=3, precision=EU_FP64)
    prim = inputs.quadrant_states(9)
    a.init_quadrant(prim)
    b.init_quadrant(prim)
    assert a.advance(10, use_graph=True) == 10
    for _ in range(10):
        b.step(True)
    for l in range(3):
        assert np.array_equal(a.level(l), b.level(l))
        assert np.array_equal(a.active(l), b.active(l))
    # replays interleaved with eager host work keep agreeing
    a.conserved_totals()
    assert a.advance(5, use_graph=True) == 5
    for _ in range(5):
        b.step(True)
    for l in range(3):
        assert np.array_equal(a.level(l), b.level(l))


@pytest.mark.parametrize("kw", [dict(levels=3), dict(levels=3, scheme=1), dict(levels=1, n0=64, scheme=1)])
def test_graph_runs_equal_eager(kw):
    """Runs of sixteen steps replay one graph; the rest replays the graphs of
    one step.  Either way the state (patch cells and ghost cells) is that of
    eager steps, bit for bit, also where every step moves the state to the
    other array (the AMR scheme) and a run starts from the second array.
    Cells outside the patches and their ghost layers hold no state (with
    the AMR scheme they are whatever the other array held) and are not
    compared."""
    kw = dict(kw)
    n0 = kw.pop("n0", 32)
    a = Solver(2, n0=n0, precision=EU_FP64, **kw)
    b = Solver(2, n0=n0, precision=EU_FP64, **kw)
    prim = inputs.quadrant_states(4)
    a.init_quadrant(prim)
    b.init_quadrant(prim)
    for n in (3, 19, 8):
        assert a.advance(n, use_graph=True) == n
        for _ in range(n):
            b.step(True)
        for l in range(kw["levels"]):
            act = a.active(l).astype(bool)
            assert np.array_equal(act, b.active(l).astype(bool))
            m = act | (dilate(act, 2, False) if l > 0 else act)
            assert np.array_equal(a.level(l)[:, m], b.level(l)[:, m]), (n, l)
        assert a.time() == b.time()


def test_dt_across_entry_points():
    """The time step of a step after a regrid comes from CFL partials the
    regrid left; entry points between steps that change the state or reuse
    the partials' memory must not leave stale ones.  The dt sequence and the
    state stay those of the oracle through every such mix."""
    h, s = make_pair(2, 4, 16)
    init_pair(h, s, "quadrant", 5)
    dts_o, dts_g = [], []

    def both(regrid=True, graph=False):
        dts_o.append(h.step(h.cfl_number, regrid=regrid))
        if graph:
            assert s.advance(1, use_graph=True) == 1
        else:
            s.step(regrid)
        dts_g.append(s.time()[1])

    both()
    s.conserved_totals()          # reuses the partials' memory
    both()
    both(regrid=False)            # a step without regrid leaves no partials
    both()
    s.stage_time(2)               # stage passes leave the state as it was
    both(graph=True)
    s.conserved_totals()
    both(graph=True)
    both()
    s.mr_decompose()              # projection and details, leaves unchanged
    both(graph=True)
    assert np.array_equal(np.array(dts_o), np.array(dts_g))
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL


def test_t_end_reached_exactly():
    h, s = make_pair(2, 3, 32, t_end=0.01)
    init_pair(h, s, "quadrant", 2)
    n_o = 0
    while h.t < 0.01:
        h.step(0.45, 0.01)
        n_o += 1
    n_g = s.advance(n_o + 5, use_graph=True)
    assert n_g == n_o
    assert s.time()[0] == h.t
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_error_report(dim):
    if dim == 2:
        h, s = make_pair(2, 3, 32, precision=EU_FP32, cfl=0.4)
        init_pair(h, s, "quadrant", 0)
        steps = 30
    else:
        h, s = make_pair(3, 2, 16, precision=EU_FP32, cfl=0.4)
        init_pair(h, s, "ellipsoid", 0)
        steps = 10
    for _ in range(steps):
        dt = h.step(0.4)
    s.advance(steps, use_graph=False)
    # the hierarchies may differ where an FP32 detail sits at the threshold;
    # compare the projected finest-grid solutions (error assessment, Sec. 3)
    flag_dis = sum(int((h.flags(l) != s.flags(l)).sum()) for l in range(h.L - 1))
    Uo = h.composite()
    Ug = composite_gpu(s, h)
    vol = h.dx(h.L - 1) ** dim
    rel_l1 = np.abs(Ug[0] - Uo[0]).sum() * vol / (np.abs(Uo[0]).sum() * vol)
    say(f"  fp32 dim {dim}: rho L1 rel {rel_l1:.3e}, flag disagreements {flag_dis}")
    assert rel_l1 <= 1e-5


def composite_gpu(s, h):
    """The GPU's finest-grid projection (eu_copy_uniform)."""
    return s.composite()


def test_batch_fp64_instances():
    sides = [32, 96, 64, 128, 40, 72]
    states = np.stack([inputs.quadrant_states(100 + i) for i in range(len(sides))])
    s = Solver(2, sides=sides, precision=EU_FP64, cfl=0.45)
    s.init_quadrant_batch(states)
    s.advance(20, use_graph=True)
    T = s.conserved_totals()
    for i, n in enumerate(sides):
        h = orc.Hierarchy(2, 1, n)
        h.init_finest(orc.init_quadrant(n, G, states[i]))
        for _ in range(20):
            h.step(0.45)
        Qg = s.level(0, inst=i)
        err = np.abs(Qg - h.level(0)).max() / np.abs(h.level(0)).max()
        assert err <= FP64_TOL, (i, n, err)
        assert np.allclose(T[i], h.totals(), rtol=1e-13)


def test_nonphysical_state_reported():
    s = Solver(2, n0=16, levels=1, precision=EU_FP64)
    W = np.ones((4, 16, 16))
    W[1:3] = 0.0
    Q = orc.prim2cons(2, G, W)
    Q[0, 3, 4] = -1.0
    s.set_finest(Q)
    with pytest.raises(EuError) as ei:
        s.cfl_dt()
    assert ei.value.code == 4
    s.clear_status()
    assert s.status() == 0


def test_full_size_adaptive2d_quad_5levels():
    """The full 2D adaptive configuration (5 levels 32^2 .. 512^2, eps 1e-3)
    for its first steps, FP64."""
    say("full adaptive2d 5 levels")
    h, s = make_pair(2, 5, 32, t_end=0.25)
    init_pair(h, s, "quadrant", 0)
    compare_masks(h, s)
    do, dg = run_pair(h, s, 8, t_end=0.25)
    assert np.array_equal(do, dg)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    say("  linf", linf)
    assert linf.max() <= FP64_TOL


def test_full_size_uniform3d_256_fp64():
    """256^3 ellipsoid (full size), first 2 steps, FP64."""
    say("full uniform3d 256^3")
    h, s = make_pair(3, 1, 256, cfl=0.4)
    init_pair(h, s, "ellipsoid", 0)
    do, dg = run_pair(h, s, 2)
    assert np.array_equal(do, dg)
    Qo, Qg = h.level(0), s.level(0)
    err = np.abs(Qg - Qo).max(axis=(1, 2, 3)) / np.abs(Qo).max(axis=(1, 2, 3))
    say("  linf", err)
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("dim", [2, 3])
def test_composite_fp64_bit_exact(dim):
    """eu_copy_uniform against the oracle's projection onto the finest grid
    (Sec. 3 error assessment), FP64, after adaptive steps."""
    if dim == 2:
        h, s = make_pair(2, 4, 32)
        init_pair(h, s, "quadrant", 4)
        steps = 6
    else:
        h, s = make_pair(3, 3, 16, cfl=0.4)
        init_pair(h, s, "ellipsoid", 2)
        steps = 3
    run_pair(h, s, steps)
    Uo, Ug = h.composite(), s.composite()
    assert Ug.shape == Uo.shape
    assert np.array_equal(Ug, Uo)
    # the stage array it used as scratch is rebuilt by the next step
    do, dg = run_pair(h, s, 2)
    assert np.array_equal(do, dg)
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL
