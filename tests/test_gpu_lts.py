"""Local time stepping on the GPU against the oracle: the recursive level
cycle (time-interpolated ghost cells, flux correction), FP64 bit-level
agreement of time steps, hierarchy and state, and conservation."""
import numpy as np
import pytest

import oracle as orc
from paper_1603_05211_amd import EU_FP32, EU_FP64

from gpu_helpers import compare_masks, init_pair, make_pair, run_pair, say, state_errors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_lts_adaptive2d_fp64(seed):
    say("lts adaptive2d fp64 seed", seed)
    h, s = make_pair(2, 3, 32, cfl=0.4, lts=True)
    init_pair(h, s, "quadrant", seed)
    for k in range(3):
        do, dg = run_pair(h, s, 2)
        assert np.array_equal(do, dg), (do, dg)
        compare_masks(h, s)
        linf, _ = state_errors(h, s)
        say("  linf", linf.max())
        assert linf.max() <= FP64_TOL
    lo_, _ = h.counts()
    lg, _ = s.counters()
    assert np.array_equal(lo_, lg)


def test_lts_adaptive3d_fp64():
    say("lts adaptive3d fp64")
    h, s = make_pair(3, 3, 16, cfl=0.4, lts=True)
    init_pair(h, s, "ellipsoid", 2)
    do, dg = run_pair(h, s, 3)
    assert np.array_equal(do, dg)
    compare_masks(h, s)
    linf, _ = state_errors(h, s)
    say("  linf", linf)
    assert linf.max() <= FP64_TOL


def test_lts_periodic_conservation_gpu():
    h, s = make_pair(2, 3, 32, bc=orc.BC_PERIODIC, cfl=0.4, lts=True)
    init_pair(h, s, "quadrant", 6)
    T0 = s.conserved_totals()
    do, dg = run_pair(h, s, 5)
    assert np.array_equal(do, dg)
    T1 = s.conserved_totals()
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0)))
    linf, _ = state_errors(h, s)
    assert linf.max() <= FP64_TOL


def test_lts_graph_equals_eager_and_counts():
    a_o, a = make_pair(2, 3, 32, cfl=0.4, lts=True)
    b_o, b = make_pair(2, 3, 32, cfl=0.4, lts=True)
    init_pair(a_o, a, "quadrant", 3)
    init_pair(b_o, b, "quadrant", 3)
    a.advance(4, use_graph=True)
    for _ in range(4):
        b.step(True)
    for l in range(3):
        assert np.array_equal(a.level(l), b.level(l))
    upd_o = 0
    for _ in range(4):
        upd_o += a_o.step_lts(0.4)[1]
    assert a.leaf_updates() == (upd_o, 4)


def test_lts_fp32_error_report():
    h, s = make_pair(2, 3, 32, precision=EU_FP32, cfl=0.4, lts=True)
    init_pair(h, s, "quadrant", 0)
    for _ in range(6):
        h.step_lts(0.4)
    s.advance(6, use_graph=False)
    U_o = h.composite()
    U = s.level(0)
    for l in range(1, 3):
        P = orc.predict(2, U, 0)
        act = s.active(l).astype(bool)
        P[:, act] = s.level(l)[:, act]
        U = P
    rel = np.abs(U[0] - U_o[0]).sum() / np.abs(U_o[0]).sum()
    say(f"  lts fp32 rho L1 rel {rel:.3e}")
    assert rel <= 1e-5
