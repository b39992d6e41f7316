"""Pins of the oracle's MR-scheme variants (the paper names an AUSM+ flux and
a second-order Runge-Kutta step without fixing these details):

* AUSM+ with Liou's critical interface sound speed: a stationary normal
  shock (upstream and downstream states from the textbook normal-shock
  relations) passes exactly the physical flux, in either orientation and on
  every axis -- the property Liou chose that speed for; the mean speed
  fails it (control); consistency and supersonic upwinding;
* Heun's RK2: one step equals (Q + Q*)/2 - (dt/2) F(Q*), with the operator
  F taken from the midpoint rule's first stage (pinned separately); second
  order on a smooth wave; conservation; local time steps refuse it."""
import math

import numpy as np
import pytest

from paper_1603_05211_amd import inputs

G = 1.4


def phys_flux(w, axis, g=G):
    dim = len(w) - 2
    rho, v, p = w[0], np.asarray(w[1:1 + dim]), w[-1]
    rhoe = p / (g - 1) + 0.5 * rho * float(v @ v)
    vn = v[axis]
    f = [rho * vn] + [rho * v[k] * vn + (p if k == axis else 0.0) for k in range(dim)] + [(rhoe + p) * vn]
    return np.array(f)


def normal_shock(M1, rho1=1.0, p1=1.0, g=G):
    """Upstream (rho, u, p) with Mach number M1 > 1 and the downstream state
    of the stationary normal shock (Rankine-Hugoniot)."""
    c1 = math.sqrt(g * p1 / rho1)
    u1 = M1 * c1
    r = (g + 1) * M1 ** 2 / ((g - 1) * M1 ** 2 + 2)
    p2 = p1 * (1 + 2 * g / (g + 1) * (M1 ** 2 - 1))
    return (rho1, u1, p1), (rho1 * r, u1 / r, p2)


def prim(dim, axis, rho, u, p, vt=0.0):
    w = np.zeros(dim + 2)
    w[0], w[-1] = rho, p
    w[1 + axis] = u
    for k in range(dim):
        if k != axis:
            w[1 + k] = vt
    return w


@pytest.mark.parametrize("dim", [2, 3])
def test_critical_speed_resolves_stationary_shock_exactly(orc, dim):
    for M1 in (1.2, 2.0, 3.5):
        up, down = normal_shock(M1)
        for axis in range(dim):
            for orient in (+1, -1):
                if orient > 0:   # flow to +x: upstream on the left
                    wL, wR = prim(dim, axis, up[0], up[1], up[2]), prim(dim, axis, down[0], down[1], down[2])
                else:            # flow to -x: upstream on the right
                    wL = prim(dim, axis, down[0], -down[1], down[2])
                    wR = prim(dim, axis, up[0], -up[1], up[2])
                F = orc.ausm_plus(dim, G, axis, wL, wR, speed=orc.AUSM_CRITICAL)
                fL, fR = phys_flux(wL, axis), phys_flux(wR, axis)
                scale = np.abs(fL).max()
                assert np.abs(fL - fR).max() <= 1e-13 * scale       # the data are a shock
                assert np.abs(F - fL).max() <= 1e-13 * scale, (M1, axis, orient, F, fL)
                Fm = orc.ausm_plus(dim, G, axis, wL, wR, speed=orc.AUSM_MEAN)
                assert np.abs(Fm - fL).max() > 1e-3 * scale          # control: the mean speed is not exact


def test_critical_speed_consistency_and_upwinding(orc):
    rng = np.random.default_rng(11)
    for _ in range(200):
        dim = int(rng.integers(2, 4))
        axis = int(rng.integers(0, dim))
        w = np.concatenate([[rng.uniform(0.2, 3)], rng.uniform(-2, 2, dim), [rng.uniform(0.1, 3)]])
        F = orc.ausm_plus(dim, G, axis, w, w, speed=orc.AUSM_CRITICAL)
        f = phys_flux(w, axis)
        assert np.abs(F - f).max() <= 1e-13 * max(np.abs(f).max(), 1.0)
    # supersonic to the right with respect to both critical speeds: the left flux
    wL = np.array([1.0, 3.0, 0.2, 1.0])
    wR = np.array([0.7, 2.8, -0.1, 0.8])
    F = orc.ausm_plus(2, G, 0, wL, wR, speed=orc.AUSM_CRITICAL)
    assert np.abs(F - phys_flux(wL, 0)).max() <= 1e-13 * np.abs(phys_flux(wL, 0)).max()


def uniform(orc, n, Q, **kw):
    h = orc.Hierarchy(2, 1, n, **kw)
    h.init_finest(Q)
    return h


def test_heun_step_is_the_heun_combination_of_the_stage_operator(orc):
    """Q* = Q - dt F(Q) is the midpoint rule's first stage with 2 dt (exact:
    a power-of-two scaling); F(Q*) comes from that stage applied to Q*; the
    Heun step must equal (Q + Q*)/2 - (Q* - (Q* - dt/2 F(Q*)))."""
    n, dt = 48, 2e-3
    Q = orc.init_quadrant(n, G, inputs.quadrant_states(5))
    a = uniform(orc, n, Q)
    a.stage(1, 2 * dt)
    Qstar = a.level_stage(0).copy()
    b = uniform(orc, n, Qstar)
    b.stage(1, dt)
    Qs2 = b.level_stage(0).copy()          # Q* - (dt/2) F(Q*)
    expect = 0.5 * (Q + Qstar) - (Qstar - Qs2)
    c = uniform(orc, n, Q, rk=orc.RK_HEUN)
    c.step_fixed(dt)
    got = c.level(0)
    assert np.abs(got - expect).max() <= 1e-12 * np.abs(expect).max()
    m = uniform(orc, n, Q)
    m.step_fixed(dt)
    assert np.abs(m.level(0) - got).max() > 1e-9    # the midpoint rule differs


def test_heun_second_order_and_conservation(orc):
    errs = []
    for n in (32, 64, 128):
        x = np.arange(n + 1) / n
        avg = lambda s: 1 + 0.2 * (np.cos(2 * np.pi * (x[:-1] - s)) - np.cos(2 * np.pi * (x[1:] - s))) / (2 * np.pi / n)
        rho = np.broadcast_to(avg(0.0)[None, :], (n, n))
        W = np.stack([rho, np.ones((n, n)), np.zeros((n, n)), np.ones((n, n))])
        h = uniform(orc, n, orc.prim2cons(2, G, W), bc=orc.BC_PERIODIC, rk=orc.RK_HEUN)
        T0 = h.totals()
        dt = 0.2 / n
        steps = int(round(0.25 / dt))
        for _ in range(steps):
            h.step_fixed(dt)
        T1 = h.totals()
        assert np.all(np.abs(T1 - T0) <= 1e-13 * np.maximum(1.0, np.abs(T0)))
        errs.append(np.abs(h.level(0)[0][0] - avg(steps * dt)).sum() / n)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 1.6, (errs, rates)


@pytest.mark.parametrize("rk,speed", [(1, 0), (0, 1), (1, 1)])
def test_variants_on_an_adaptive_hierarchy_conserve(orc, rk, speed):
    Q = orc.init_quadrant(128, G, inputs.quadrant_states(6))
    h = orc.Hierarchy(2, 3, 32, bc=orc.BC_PERIODIC, eps=1e-3, rk=rk, ausm_speed=speed)
    h.init_finest(Q)
    T0 = h.totals()
    for _ in range(8):
        h.step(0.4)
    assert np.all(np.abs(h.totals() - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0)))


def test_local_time_steps_refuse_heun(orc):
    h = orc.Hierarchy(2, 2, 32, rk=orc.RK_HEUN)
    h.init_finest(orc.init_quadrant(64, G, inputs.quadrant_states(1)))
    with pytest.raises(ValueError):
        h.step_lts(0.4)
