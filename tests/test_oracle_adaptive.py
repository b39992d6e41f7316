"""Pins of the oracle's adaptive (MR-flagged block-patch) hierarchy.

Special cases that reduce to the uniform scheme, invariants of the
hierarchy (alignment, nesting, gradedness, flag coverage, the tiling rule),
conservation, free-stream preservation, threshold monotonicity, and the
paper's accuracy-perturbation measure against a uniform finest-grid run.
"""
import math

import numpy as np
import pytest

from oracle import exact_riemann as er
from paper_1603_05211_amd import inputs

G = 1.4


def coarsen_mask(m, dim):
    return m[0::2, 0::2] if dim == 2 else m[0::2, 0::2, 0::2]


def dilate(m, r, periodic=False):
    out = m.copy()
    dim = m.ndim
    n = m.shape[0]
    idx = np.arange(n)
    for ax in range(dim):
        acc = np.zeros_like(out)
        for s in range(-r, r + 1):
            j = (idx + s) % n if periodic else np.clip(idx + s, 0, n - 1)
            acc |= np.take(out, j, axis=ax)
        out = acc
    return out


def check_hierarchy(h, periodic=False):
    """Structural invariants of the hierarchy after init or regrid."""
    dim, L = h.dim, h.L
    P = h.patches()
    acts = [h.active(l).astype(bool) for l in range(L)]
    assert acts[0].all()
    # patches: block tiler: aligned cubes of pmin..pmax cells (powers of
    # two); Berger-Rigoutsos: boxes of whole pmin-blocks inside one
    # pmax-block; disjoint, union = active
    br = getattr(h, "tiler", 0) == 1
    for l in range(1, L):
        cover = np.zeros_like(acts[l], dtype=np.int32)
        for lv, ox, oy, oz, sx, sy, sz in P:
            if lv != l:
                continue
            ext = (sx, sy, sz) if dim == 3 else (sx, sy)
            org = (ox, oy, oz) if dim == 3 else (ox, oy)
            if dim == 2:
                assert oz == 0 and sz == 1
            if br:
                for o_, e_ in zip(org, ext):
                    assert o_ % h.pmin == 0 and e_ % h.pmin == 0 and 0 < e_ <= h.pmax
                    assert o_ // h.pmax == (o_ + e_ - 1) // h.pmax
            else:
                S = sx
                assert all(e_ == S for e_ in ext) and S in (8, 16, 32) and all(o_ % S == 0 for o_ in org)
            sl = tuple(slice(o_, o_ + e_) for o_, e_ in zip(org[::-1], ext[::-1]))
            cover[sl] += 1
        assert cover.max() <= 1
        assert np.array_equal(cover.astype(bool), acts[l])
    # proper nesting: level-l cells within 2 of the parents of level l+1 exist
    for l in range(0, L - 1):
        par = coarsen_mask(acts[l + 1], dim)
        if l >= 1:
            need = dilate(par, 2, periodic)
            assert not (need & ~acts[l]).any(), l
    # graded: a leaf's face neighbours are leaves of the same level, or
    # covered (finer leaves), or lie on the next coarser level
    return P, acts


def leaf_level_map(h):
    """Level of the leaf covering each finest cell."""
    dim, L = h.dim, h.L
    nF = h.n(L - 1)
    out = np.full((nF,) * dim, -1)
    for l in range(L):
        leaf = h.leaf_mask(l)
        k = 2 ** (L - 1 - l)
        up = leaf
        for ax in range(dim):
            up = np.repeat(up, k, axis=ax)
        out[up] = l
    return out


def test_init_hierarchy_invariants(orc):
    for seed in (0, 1, 2):
        prim = inputs.quadrant_states(seed)
        h = orc.Hierarchy(2, 4, 32, eps=1e-3)
        h.init_finest(orc.init_quadrant(256, G, prim))
        P, acts = check_hierarchy(h)
        lm = leaf_level_map(h)
        assert (lm >= 0).all()  # leaves tile the domain exactly once
        # gradedness: neighbouring leaves differ by at most one level
        for ax in range(2):
            d = np.abs(np.diff(lm, axis=ax))
            assert d.max() <= 1


def test_tiling_rule_and_flag_coverage(orc):
    """Every flagged cell's children are in a patch; every patch reached the
    efficiency eta (or has the smallest size); every block that was split
    (the parent block of a patch) fell short of eta."""
    prim = inputs.quadrant_states(5)
    h = orc.Hierarchy(2, 4, 32, eps=1e-3, eta=0.8)
    h.init_finest(orc.init_quadrant(256, G, prim))
    for _ in range(3):
        h.step(0.45)
    P, acts = check_hierarchy(h)
    for l in range(h.L - 1):
        F = h.flags(l).astype(bool)
        child_cov = coarsen_mask(acts[l + 1], 2)
        assert not (F & ~child_cov).any()
        for lv, ox, oy, oz, S, _, _ in P:
            if lv != l + 1:
                continue
            fill = F[oy // 2:(oy + S) // 2, ox // 2:(ox + S) // 2].mean()
            assert fill > 0
            assert S == 8 or fill >= 0.8
            if S < 32:
                px, py = ox - ox % (2 * S), oy - oy % (2 * S)
                pfill = F[py // 2:(py + 2 * S) // 2, px // 2:(px + 2 * S) // 2].mean()
                assert pfill < 0.8
        # the flags contain the raw flags dilated by one cell
        D = h.details(l)
        sig = D >= h.eps
        assert not (sig & ~F).any()


def test_flags_follow_details(orc):
    """Raw flags: significant details (D >= eps) and their children's parents
    (preventive refinement).  Checked on the initial analysis, where every
    detail is computed from the full finest data."""
    prim = inputs.quadrant_states(1)
    h = orc.Hierarchy(2, 4, 32, eps=2e-3)
    Qf = orc.init_quadrant(256, G, prim)
    h.init_finest(Qf)
    # independent detail computation: restrict, predict, compare densities
    lev = [None] * 4
    lev[3] = Qf
    for l in (2, 1, 0):
        lev[l] = orc.restrict(2, lev[l + 1])
    for l in range(3):
        pred = orc.predict(2, lev[l])[0]
        err = np.abs(lev[l + 1][0] - pred)
        D = err.reshape(h.n(l), 2, h.n(l), 2).max(axis=(1, 3))
        assert np.array_equal(D, h.details(l))
        sig = D >= h.eps
        raw = sig.copy()
        if l >= 1:
            Dp = (np.abs(lev[l][0] - orc.predict(2, lev[l - 1])[0])
                  .reshape(h.n(l - 1), 2, h.n(l - 1), 2).max(axis=(1, 3)))
            raw |= np.repeat(np.repeat(Dp >= h.eps, 2, 0), 2, 1)
        F = h.flags(l).astype(bool)
        assert not (dilate(raw, 1) & ~F).any()


def test_threshold_monotone(orc):
    prim = inputs.quadrant_states(2)
    Qf = orc.init_quadrant(256, G, prim)
    prev = None
    for eps in (1e-4, 1e-3, 1e-2, 1e-1):
        h = orc.Hierarchy(2, 4, 32, eps=eps)
        h.init_finest(Qf)
        acts = [h.active(l).astype(bool) for l in range(4)]
        if prev is not None:
            for a, b in zip(acts, prev):
                assert not (a & ~b).any()
        prev = acts
    # constant data: no details, no patches
    W = np.stack([np.full((256, 256), v) for v in (1.0, 0.2, 0.1, 1.0)])
    h = orc.Hierarchy(2, 4, 32, eps=1e-12)
    h.init_finest(orc.prim2cons(2, G, W))
    assert len(h.patches()) == 0


def test_eps_zero_equals_uniform_finest(orc):
    """eps = 0 refines everywhere: leaves are exactly the finest grid and the
    adaptive step reduces to the uniform scheme on it, bit for bit."""
    prim = inputs.quadrant_states(4)
    Qf = orc.init_quadrant(128, G, prim)
    h = orc.Hierarchy(2, 3, 32, eps=0.0)
    h.init_finest(Qf)
    u = orc.Hierarchy(2, 1, 128)
    u.init_finest(Qf)
    for _ in range(8):
        dta = h.step(0.45)
        dtu = u.step(0.45)
        assert dta == dtu
    assert np.array_equal(h.level(2), u.level(0))


def test_eps_huge_equals_uniform_coarse(orc):
    prim = inputs.quadrant_states(4)
    Qf = orc.init_quadrant(128, G, prim)
    h = orc.Hierarchy(2, 3, 32, eps=1e30)
    h.init_finest(Qf)
    assert len(h.patches()) == 0
    u = orc.Hierarchy(2, 1, 32)
    u.init_finest(orc.restrict(2, orc.restrict(2, Qf)))
    for _ in range(8):
        assert h.step(0.45) == u.step(0.45)
    assert np.array_equal(h.level(0), u.level(0))


@pytest.mark.parametrize("dim", [2, 3])
def test_adaptive_conservation_periodic(orc, dim):
    if dim == 2:
        Qf = orc.init_quadrant(128, G, inputs.quadrant_states(6))
        h = orc.Hierarchy(2, 3, 32, bc=orc.BC_PERIODIC, eps=1e-3)
    else:
        e = inputs.ellipsoid(6)
        Qf = orc.init_ellipsoid(64, G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        h = orc.Hierarchy(3, 2, 32, bc=orc.BC_PERIODIC, lo=-1.0, hi=1.0, eps=1e-3)
    h.init_finest(Qf)
    check_hierarchy(h, periodic=True)
    T0 = h.totals()
    npatch = []
    for _ in range(12):
        h.step(0.4)
        npatch.append(len(h.patches()))
    check_hierarchy(h, periodic=True)
    T1 = h.totals()
    assert len(set(npatch)) > 1 or dim == 3  # the mesh adapts while conserving
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_adaptive_free_stream_bitwise(orc):
    """Uniform state written onto a partially refined hierarchy stays
    bit-exact: prediction and projection reproduce constants, fine-flux
    means of equal fluxes are the flux itself."""
    prim = inputs.quadrant_states(8)
    h = orc.Hierarchy(2, 3, 32, eps=1e-3)
    h.init_finest(orc.init_quadrant(128, G, prim))
    assert len(h.patches()) > 0
    w = np.array([0.8, 0.35, -0.25, 1.1])
    q = orc.prim2cons(2, G, w.reshape(4, 1)).ravel()
    for l in range(3):
        h.level(l)[...] = q.reshape(4, 1, 1)
    for _ in range(10):
        h.step(0.45, regrid=False)
    for l in range(3):
        assert np.array_equal(h.level(l), np.broadcast_to(q.reshape(4, 1, 1), h.level(l).shape))


def test_mr_reconstruction(orc):
    """The composite (adaptive data projected up by prediction) reproduces
    the finest data exactly when no detail is dropped (eps = 0), and within a
    multiple of eps per level otherwise."""
    x = (np.arange(128) + 0.5) / 128
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.3 * np.tanh((X + 0.5 * Y - 0.7) / 0.03)
    W = np.stack([rho, 0.1 * np.ones_like(rho), -0.2 * np.ones_like(rho), np.ones_like(rho)])
    Qf = orc.prim2cons(2, G, W)
    h = orc.Hierarchy(2, 3, 32, eps=0.0)
    h.init_finest(Qf)
    assert np.array_equal(h.composite(), Qf)
    for eps in (1e-3, 1e-2):
        h = orc.Hierarchy(2, 3, 32, eps=eps)
        h.init_finest(Qf)
        err = np.abs(h.composite()[0] - Qf[0]).max()
        assert err <= 4 * 3 * eps, (eps, err)


def test_accuracy_perturbation_sod(orc):
    """The paper's accuracy perturbation |L1_FV - L1_a| / L1_FV (Sec. 3) of
    an adaptive Sod run against the uniform finest-grid run stays small."""
    L_, R_ = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    n = 256
    Qf = orc.init_riemann1d(2, n, G, 0, L_, R_)
    t_end = 0.15
    h = orc.Hierarchy(2, 4, 32, eps=1e-3)
    h.init_finest(Qf)
    while h.t < t_end:
        h.step(0.45, t_end)
    u = orc.Hierarchy(2, 1, n)
    u.init_finest(Qf)
    while u.t < t_end:
        u.step(0.45, t_end)
    ex, _, _ = er.cell_averages(L_, R_, n, t_end)
    comp = h.composite()[0]
    l1a = np.abs(comp - ex[None, :]).sum() / n ** 2
    l1u = np.abs(u.level(0)[0] - ex[None, :]).sum() / n ** 2
    leaves, _ = h.counts()
    assert leaves.sum() < 0.5 * n * n  # it did adapt
    assert abs(l1u - l1a) / l1u < 0.15, (l1u, l1a)


# --------------------------------------------------------------------------
# local time stepping (recursive level cycle with flux correction)
# --------------------------------------------------------------------------

def test_lts_single_level_is_global_step(orc):
    Qf = orc.init_quadrant(64, G, inputs.quadrant_states(1))
    a = orc.Hierarchy(2, 1, 64)
    b = orc.Hierarchy(2, 1, 64)
    a.init_finest(Qf)
    b.init_finest(Qf)
    for _ in range(5):
        dta, _ = a.step_lts(0.45)
        dtb = b.step(0.45)
        assert dta == dtb
    assert np.array_equal(a.level(0), b.level(0))


def test_lts_eps_zero_equals_uniform_substeps(orc):
    """Fully refined hierarchy: only the finest level has leaves and no ghost
    cells, so one level-0 step equals 2^(L-1) uniform steps of dt_0/2^(L-1)."""
    Qf = orc.init_quadrant(128, G, inputs.quadrant_states(2))
    h = orc.Hierarchy(2, 3, 32, eps=0.0)
    h.init_finest(Qf)
    u = orc.Hierarchy(2, 1, 128)
    u.init_finest(Qf)
    for _ in range(3):
        dt0, upd = h.step_lts(0.45)
        assert upd == 4 * 128 * 128
        for _ in range(4):
            u.step_fixed(dt0 * 0.25)
    assert np.array_equal(h.level(2), u.level(0))


@pytest.mark.parametrize("dim", [2, 3])
def test_lts_conservation_periodic(orc, dim):
    if dim == 2:
        Qf = orc.init_quadrant(128, G, inputs.quadrant_states(6))
        h = orc.Hierarchy(2, 3, 32, bc=orc.BC_PERIODIC, eps=1e-3)
    else:
        e = inputs.ellipsoid(6)
        Qf = orc.init_ellipsoid(64, G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        h = orc.Hierarchy(3, 2, 32, bc=orc.BC_PERIODIC, lo=-1.0, hi=1.0, eps=1e-3)
    h.init_finest(Qf)
    T0 = h.totals()
    for _ in range(6):
        h.step_lts(0.4)
    check_hierarchy(h, periodic=True)
    T1 = h.totals()
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_lts_without_correction_does_not_conserve(orc):
    """Control for the test above, with a mistake planted in the oracle: with
    the flux correction skipped, the totals drift well beyond rounding, so
    the conservation above is the correction's doing."""
    Qf = orc.init_quadrant(128, G, inputs.quadrant_states(6))
    h = orc.Hierarchy(2, 3, 32, bc=orc.BC_PERIODIC, eps=1e-3)
    h.init_finest(Qf)
    orc.lib().orc_h_set_no_reflux(h._h, 1)
    T0 = h.totals()
    for _ in range(6):
        h.step_lts(0.4)
    drift = np.abs(h.totals() - T0) / np.maximum(1.0, np.abs(T0))
    assert drift.max() > 10 * 2e-13, drift


def test_lts_free_stream_bitwise(orc):
    prim = inputs.quadrant_states(8)
    h = orc.Hierarchy(2, 3, 32, eps=1e-3)
    h.init_finest(orc.init_quadrant(128, G, prim))
    w = np.array([0.8, 0.35, -0.25, 1.1])
    q = orc.prim2cons(2, G, w.reshape(4, 1)).ravel()
    for l in range(3):
        h.level(l)[...] = q.reshape(4, 1, 1)
    for _ in range(4):
        h.step_lts(0.45, regrid=False)
    for l in range(3):
        assert np.array_equal(h.level(l), np.broadcast_to(q.reshape(4, 1, 1), h.level(l).shape))


def test_lts_accuracy_perturbation_sod(orc):
    L_, R_ = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    n = 256
    Qf = orc.init_riemann1d(2, n, G, 0, L_, R_)
    t_end = 0.15
    h = orc.Hierarchy(2, 4, 32, eps=1e-3)
    h.init_finest(Qf)
    while h.t < t_end:
        h.step_lts(0.4, t_end)
        check_hierarchy(h)
    u = orc.Hierarchy(2, 1, n)
    u.init_finest(Qf)
    while u.t < t_end:
        u.step(0.4, t_end)
    ex, _, _ = er.cell_averages(L_, R_, n, t_end)
    l1a = np.abs(h.composite()[0] - ex[None, :]).sum() / n ** 2
    l1u = np.abs(u.level(0)[0] - ex[None, :]).sum() / n ** 2
    assert abs(l1u - l1a) / l1u < 0.2, (l1u, l1a)


# --------------------------------------------------------------------------
# local time stepping: the time interpolation of ghost cells (theta)
# --------------------------------------------------------------------------

def _fixed_hierarchy(orc, dim, L, n0, Qf, bands, bc=0):
    """A hierarchy whose patches are imposed (level l covers the slab
    bands[l-1] of the x axis, as fractions of the domain) and kept fixed:
    every level holds the projection of the finest data, then ghost fill."""
    h = orc.Hierarchy(dim, L, n0, bc=bc, eps=1e9)
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


def _linear_profile_lts_error(orc, dim, n0, L, steps, u=0.6, b=0.4):
    """Largest error on the patches of levels >= 1, away from the domain
    boundary, after `steps` level-0 steps with local time steps of a density
    profile linear in x advected at constant velocity and pressure.  The
    exact solution rho = 1 + b (x - u t - 1/2) is linear in space and in
    time: the limited reconstruction, the flux (consistent for equal face
    states), the midpoint rule, the prediction (exact for quadratics) and
    a linear interpolation in time all reproduce it, so the error is
    rounding unless a ghost cell is taken at the wrong time."""
    nf = n0 << (L - 1)
    shp = (nf,) * dim
    x = (np.arange(nf) + 0.5) / nf
    W = np.stack([np.broadcast_to(1 + b * (x - 0.5), shp), np.full(shp, u)] +
                 [np.zeros(shp)] * (dim - 1) + [np.ones(shp)])
    Qf = orc.prim2cons(dim, G, W)
    bands = [(0.25 + k / 8, 0.75 - k / 8) for k in range(L - 1)]
    h = _fixed_hierarchy(orc, dim, L, n0, Qf, bands)
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


@pytest.mark.parametrize("dim,n0,L,steps,tol", [(2, 64, 3, 8, 1e-14), (3, 32, 3, 2, 1e-12)])
def test_lts_linear_profile_exact(orc, dim, n0, L, steps, tol):
    """Sec. 2.2 (ghost cells at refinement boundaries by space-time
    interpolation from the two coarse time levels): with the stage times
    theta = k/2 (first stage of substep k) and (2k+1)/4 (second stage) the
    linear profile is reproduced to rounding across the refinement
    boundaries of every level."""
    assert _linear_profile_lts_error(orc, dim, n0, L, steps) <= tol


def test_lts_linear_profile_catches_constant_theta(orc):
    """Control: ghost cells taken from the coarse state at the start of its
    step (theta = 0 at every stage) fail the pin above by nine decades."""
    with orc.planted(orc.PLANT_LTS_THETA):
        err = _linear_profile_lts_error(orc, 2, 64, 3, 8)
    assert err > 1e-5, err


def test_lts_smooth_wave_second_order(orc):
    """A smooth periodic density wave crossing fixed refinement boundaries
    under local time stepping converges at second order in L1 (the composite
    on the finest grid against exact cell averages; Sec. 3 error measure)."""
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
