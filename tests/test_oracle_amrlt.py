"""Pins of the oracle's AMRLT: the AMR scheme (one MUSCL-Hancock step per
level step) in the recursive level cycle with local time steps and the flux
correction (Sec. 2.2, Fig. 2).  As for the MR scheme's cycle: one level is
the global step, a fully refined hierarchy is the uniform finest run in
substeps, periodic runs conserve (control: the correction skipped), a
uniform state stays uniform, a linear profile crosses refinement boundaries
to rounding (control: ghost cells held at the coarse start state), a smooth
wave converges at second order, and an adaptive Sod run stays close to the
uniform run against the exact solution."""
import math

import numpy as np
import pytest

from oracle import exact_riemann as er
from paper_1603_05211_amd import inputs

from test_oracle_adaptive import check_hierarchy
from test_oracle_amr_hierarchy import bump

G = 1.4


def amr(orc, *a, **kw):
    return orc.Hierarchy(*a, scheme=orc.SCHEME_AMR, **kw)


def test_single_level_is_global_step(orc):
    Qf = orc.init_quadrant(64, G, inputs.quadrant_states(1))
    a, b = amr(orc, 2, 1, 64), amr(orc, 2, 1, 64)
    a.init_finest(Qf)
    b.init_finest(Qf)
    for _ in range(5):
        dta, _ = a.step_lts(0.45)
        assert dta == b.step(0.45)
    assert np.array_equal(a.level(0), b.level(0))


def test_eps_zero_equals_uniform_substeps(orc):
    Qf = orc.init_quadrant(128, G, inputs.quadrant_states(2))
    h = amr(orc, 2, 3, 32, eps=0.0)
    h.init_finest(Qf)
    u = amr(orc, 2, 1, 128)
    u.init_finest(Qf)
    for _ in range(3):
        dt0, upd = h.step_lts(0.45)
        assert upd == 4 * 128 * 128
        for _ in range(4):
            u.step_fixed(dt0 * 0.25)
    assert np.array_equal(h.level(2), u.level(0))


def _conservation(orc, dim, no_reflux=False, steps=6, smooth=False):
    if dim == 2:
        Qf = bump(orc) if smooth else orc.init_quadrant(128, G, inputs.quadrant_states(6))
        h = amr(orc, 2, 3, 32, bc=orc.BC_PERIODIC, eps=1e-3)
    else:
        e = inputs.ellipsoid(6)
        Qf = orc.init_ellipsoid(64, G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        h = amr(orc, 3, 2, 32, bc=orc.BC_PERIODIC, lo=-1.0, hi=1.0, eps=1e-3)
    h.init_finest(Qf)
    if no_reflux:
        orc.lib().orc_h_set_no_reflux(h._h, 1)
    T0 = h.totals()
    for _ in range(steps):
        h.step_lts(0.4)
    return h, T0, h.totals()


@pytest.mark.parametrize("dim,smooth", [(2, False), (2, True), (3, False)])
def test_conservation_periodic(orc, dim, smooth):
    h, T0, T1 = _conservation(orc, dim, smooth=smooth)
    check_hierarchy(h, periodic=True)
    assert len(h.patches()) > 0
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_without_correction_does_not_conserve(orc):
    _, T0, T1 = _conservation(orc, 2, no_reflux=True, smooth=True)
    drift = np.abs(T1 - T0) / np.maximum(1.0, np.abs(T0))
    assert drift.max() > 10 * 2e-13, drift


def test_free_stream_bitwise(orc):
    h = amr(orc, 2, 3, 32, eps=1e-3)
    h.init_finest(orc.init_quadrant(128, G, inputs.quadrant_states(8)))
    w = np.array([0.8, 0.35, -0.25, 1.1])
    q = orc.prim2cons(2, G, w.reshape(4, 1)).ravel()
    for l in range(3):
        h.level(l)[...] = q.reshape(4, 1, 1)
    for _ in range(4):
        h.step_lts(0.45, regrid=False)
    for l in range(3):
        assert np.array_equal(h.level(l), np.broadcast_to(q.reshape(4, 1, 1), h.level(l).shape))


def _fixed_hierarchy(orc, dim, L, n0, Qf, bands, bc=0):
    """Patches imposed (level l covers the slab bands[l-1] of the x axis)
    and kept fixed; every level the projection of the finest data."""
    h = amr(orc, dim, L, n0, bc=bc, eps=1e9)
    h.init_finest(Qf)
    for l in range(1, L):
        n = n0 << l
        a, b = bands[l - 1]
        m = np.zeros((n,) * dim, np.uint8)
        m[..., int(a * n):int(b * n)] = 1
        h.set_active(l, m)
        Ql = Qf
        for _ in range(L - 1 - l):
            Ql = orc.restrict(dim, Ql)
        h.level(l)[...] = Ql
    h.restrict_all()
    h.ghost()
    return h


def _linear_profile_error(orc, n0=64, L=3, steps=8, u=0.6, b=0.4):
    """A density profile linear in x advected at constant velocity and
    pressure: Minmod slopes of linear data are exact, the half step and
    AUSMDV of a moving contact are exact, the prediction is exact for
    quadratics and the time interpolation for linear-in-time data, so the
    only error is rounding unless a ghost cell is taken at the wrong time."""
    nf = n0 << (L - 1)
    x = (np.arange(nf) + 0.5) / nf
    shp = (nf, nf)
    W = np.stack([np.broadcast_to(1 + b * (x - 0.5), shp), np.full(shp, u), np.zeros(shp), np.ones(shp)])
    bands = [(0.25 + k / 8, 0.75 - k / 8) for k in range(L - 1)]
    h = _fixed_hierarchy(orc, 2, L, n0, orc.prim2cons(2, G, W), bands)
    for _ in range(steps):
        h.step_lts(0.4, regrid=False)
    worst = 0.0
    for l in range(1, L):
        n = n0 << l
        xc = (np.arange(n) + 0.5) / n
        exact = 1 + b * (xc - u * h.t - 0.5)
        sel = h.active(l).astype(bool) & (np.abs(xc - 0.5) < 0.2)
        worst = max(worst, np.abs(h.level(l)[0] - exact)[sel].max())
    return worst


def test_linear_profile_exact(orc):
    assert _linear_profile_error(orc) <= 1e-13


def test_linear_profile_catches_constant_theta(orc):
    with orc.planted(orc.PLANT_LTS_THETA):
        err = _linear_profile_error(orc)
    assert err > 1e-5, err


def test_smooth_wave_second_order(orc):
    errs = []
    for n0 in (16, 32, 64):
        nf = 2 * n0
        e = np.arange(nf + 1) / nf
        k = 2 * math.pi
        avg = lambda s: 1 + 0.2 * (np.cos(k * (e[:-1] - s)) - np.cos(k * (e[1:] - s))) / (k / nf)
        shp = (nf, nf)
        W = np.stack([np.broadcast_to(avg(0.0), shp), np.ones(shp), np.zeros(shp), np.ones(shp)])
        h = _fixed_hierarchy(orc, 2, 2, n0, orc.prim2cons(2, G, W), [(0.25, 0.75)], bc=orc.BC_PERIODIC)
        while h.t < 0.25 - 1e-15:
            h.step_lts(0.4, 0.25, regrid=False)
        errs.append(np.abs(h.composite()[0] - avg(h.t)[None, :]).mean())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 1.6, (errs, rates)


def test_accuracy_perturbation_sod(orc):
    L_, R_ = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    n = 256
    Qf = orc.init_riemann1d(2, n, G, 0, L_, R_)
    t_end = 0.15
    h = amr(orc, 2, 4, 32, eps=1e-3)
    h.init_finest(Qf)
    while h.t < t_end:
        h.step_lts(0.4, t_end)
        check_hierarchy(h)
    u = amr(orc, 2, 1, n)
    u.init_finest(Qf)
    while u.t < t_end:
        u.step(0.4, t_end)
    ex, _, _ = er.cell_averages(L_, R_, n, t_end)
    l1a = np.abs(h.composite()[0] - ex[None, :]).sum() / n ** 2
    l1u = np.abs(u.level(0)[0] - ex[None, :]).sum() / n ** 2
    assert abs(l1u - l1a) / l1u < 0.2, (l1u, l1a)
