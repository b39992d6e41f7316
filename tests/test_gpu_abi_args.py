"""The arguments of the C-ABI's method calls, each against the FP64 oracle
(through the library, on the GPU): the CFL number and the remaining-time clip
of eu_cfl_dt and its device output, an external device dt and the level of
eu_fv_step, the device output of eu_conserved_totals, the threshold of
eu_mr_flag; and the give-up path of the bounded waits between workgroups,
forced from the host."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_DT_LTS, EU_FP64, EuError, Solver, inputs
from paper_1603_05211_amd._abi import EU_EHIP, EU_EINVAL

from gpu_helpers import G, compare_masks, init_pair, make_pair, say, state_errors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def test_cfl_number_and_clip_and_device_output():
    import torch
    say("eu_cfl_dt: cfl, t_remaining, dt_dev")
    h, s = make_pair(2, 3, 32)
    init_pair(h, s, "quadrant", 4)
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_o = h.cfl(0.2)[0]
    dt_g = s.cfl_dt(cfl=0.2, dt_out=dt_dev)
    assert dt_g == dt_o                       # bit for bit, another CFL number
    s.stream.synchronize()
    assert dt_dev.item() == dt_g
    assert s.time() == (dt_g, dt_g)           # the step it sized is committed
    s.fv_step()
    h.step_fixed(dt_o)
    h.regrid()
    s.mr_decompose()
    s.mr_flag()
    # a clip below the CFL step: dt equals it exactly
    t0 = s.time()[0]
    dt_c = s.cfl_dt(t_remaining=1e-4)
    assert dt_c == 1e-4 and s.time()[0] == t0 + 1e-4
    s.fv_step()
    h.step_fixed(1e-4)
    h.regrid()
    s.mr_decompose()
    s.mr_flag()
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL
    with pytest.raises(EuError):
        s.cfl_dt(cfl=math.nan)


def test_external_device_dt_and_level():
    import torch
    say("eu_fv_step: dt_dev, level")
    h, s = make_pair(2, 3, 32)
    init_pair(h, s, "quadrant", 5)
    dt_cfl = s.cfl_dt()
    dt_ext = 0.6 * dt_cfl                      # e.g. a minimum over several subdomains
    s.fv_step(dt=torch.tensor([dt_ext], dtype=torch.float64, device="cuda"), level=-1)
    assert s.time() == (dt_ext, dt_ext)
    h.step_fixed(dt_ext)
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL
    with pytest.raises(EuError) as e:
        s.fv_step(level=0)                    # a global time step has no per-level call
    assert e.value.code == EU_EINVAL
    with pytest.raises(EuError):
        s.fv_step(level=3)


def test_lts_level_zero_equals_all_levels():
    say("eu_fv_step level 0 with local time steps")
    a = Solver(2, n0=32, levels=3, precision=EU_FP64, time_mode=EU_DT_LTS)
    b = Solver(2, n0=32, levels=3, precision=EU_FP64, time_mode=EU_DT_LTS)
    prim = inputs.quadrant_states(6)
    a.init_quadrant(prim)
    b.init_quadrant(prim)
    for _ in range(3):
        assert a.cfl_dt() == b.cfl_dt()
        a.fv_step(level=-1)
        b.fv_step(level=0)
    for l in range(3):
        assert np.array_equal(a.level(l), b.level(l))


def test_totals_device_output_batch():
    import torch
    say("eu_conserved_totals: totals_dev")
    b = inputs.batch(3, n_instances=4)
    s = Solver(2, sides=list(b.sides), precision=EU_FP64)
    s.init_quadrant_batch(b.states)
    s.advance(3)
    out = torch.full((4, 4), math.nan, dtype=torch.float64, device="cuda")
    assert s.conserved_totals(out_dev=out, host=False) is None
    s.stream.synchronize()
    host = s.conserved_totals()
    assert np.array_equal(out.cpu().numpy(), host)


def test_flag_threshold_argument():
    say("eu_mr_flag: eps")
    h, s = make_pair(2, 4, 32, eps=1e-3)
    init_pair(h, s, "quadrant", 7)
    for eps in (1e-2, 3e-4):
        dt = h.step(h.cfl_number, regrid=False)
        s.step(False)
        assert s.time()[1] == dt
        h.set_eps(eps)
        h.regrid()
        s.mr_decompose()
        s.mr_flag(eps)
        compare_masks(h, s)
        linf, _ = state_errors(h, s)
        assert linf.max() <= FP64_TOL
    # later steps keep the new threshold
    h.step(h.cfl_number)
    s.step(True)
    compare_masks(h, s)


def test_bounded_wait_gives_up(monkeypatch):
    """Host-forced: the list build waits for an epoch that no workgroup
    publishes (a short bound), so the waits of every list workgroup after
    the first give up; every kernel still ends and the next synchronising
    call reports EU_EHIP.  The hierarchy has more than 256 blocks, so the
    build has two workgroups and the second one waits."""
    say("bounded waits: give-up path")
    monkeypatch.setenv("EU_WAIT_TEST", "stale")
    s = Solver(2, n0=32, levels=3, precision=EU_FP64)
    monkeypatch.delenv("EU_WAIT_TEST")
    s.init_quadrant(inputs.quadrant_states(0))
    assert s.status() == EU_EHIP
    s.close()
    # a context made without the setting is unaffected
    t = Solver(2, n0=32, levels=3, precision=EU_FP64)
    t.init_quadrant(inputs.quadrant_states(0))
    assert t.status() == 0
    assert t.advance(2) == 2 and t.status() == 0
