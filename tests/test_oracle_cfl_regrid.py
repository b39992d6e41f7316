"""The CFL signal speed options and the regrid interval of the oracle.

CFL (Sec. 4.2: CFL about 0.4; the paper does not write the signal speed
out): dt = cfl dx_finest / S on a uniform state, S = sum_d (|v_d| + c) or
max_d (|v_d| + c), c = sqrt(gamma p / rho), in closed form for arbitrary
states in 2D and 3D; the max form is the sum form minus (d - 1) c for a
state moving along one axis.  Regrid interval (the AMR runs of Sec. 4
rebuild the hierarchy every step; the interval is a scheduling option): the
hierarchy stays as it is between regrids while the solution moves, changes
at a regrid, and an interval of one is the default run bit for bit; the
method stays conservative."""
import numpy as np
import pytest

from paper_1603_05211_amd import inputs

from test_oracle_adaptive import check_hierarchy

G = 1.4


def uniform_hierarchy(orc, dim, w, mode, L=3, n0=16):
    lo = 0.0 if dim == 2 else -1.0
    h = orc.Hierarchy(dim, L, n0, lo=lo, eps=1e-3, cfl_mode=mode, pmax=32 if dim == 2 else 16)
    nf = n0 << (L - 1)
    q = orc.prim2cons(dim, G, np.asarray(w, float).reshape(dim + 2, 1)).ravel()
    h.init_finest(np.broadcast_to(q.reshape((dim + 2,) + (1,) * dim), (dim + 2,) + (nf,) * dim).copy())
    return h


@pytest.mark.parametrize("dim", [2, 3])
def test_cfl_closed_forms(orc, dim):
    rng = np.random.default_rng(11 + dim)
    for _ in range(5):
        rho, p = rng.uniform(0.2, 3.0), rng.uniform(0.1, 5.0)
        v = rng.uniform(-2.0, 2.0, dim)
        w = [rho, *v, p]
        c = np.sqrt(G * p / rho)
        for mode, S in ((orc.CFL_SUM, np.sum(np.abs(v) + c)), (orc.CFL_MAX, np.max(np.abs(v)) + c)):
            h = uniform_hierarchy(orc, dim, w, mode)
            dt, smax = h.cfl(0.4)
            # a uniform state refines nothing: every leaf is on level 0
            assert len(h.patches()) == 0
            hi, lo = 1.0, (0.0 if dim == 2 else -1.0)
            dx = (hi - lo) / h.n(0)
            assert dt == pytest.approx(0.4 * dx / S, rel=1e-14)
            assert smax[0] == pytest.approx(S, rel=1e-14) and not smax[1:].any()


def test_max_form_along_one_axis(orc):
    """A state moving along x: the sum form counts c once per axis, the max
    form once, so S_sum - S_max = (d - 1) c."""
    for dim in (2, 3):
        w = [1.3, 0.7] + [0.0] * (dim - 1) + [2.0]
        c = np.sqrt(G * 2.0 / 1.3)
        s_sum = uniform_hierarchy(orc, dim, w, orc.CFL_SUM).cfl(0.4)[1][0]
        s_max = uniform_hierarchy(orc, dim, w, orc.CFL_MAX).cfl(0.4)[1][0]
        assert s_sum - s_max == pytest.approx((dim - 1) * c, rel=1e-13)


def test_cfl_mode_rejects_unknown(orc):
    with pytest.raises(ValueError):
        orc.Hierarchy(2, 2, 16, cfl_mode=2)
    with pytest.raises(ValueError):
        orc.Hierarchy(2, 2, 16, regrid_every=0)


def quadrant(orc, every, bc=0, scheme=0):
    h = orc.Hierarchy(2, 4, 32, bc=bc, eps=1e-3, regrid_every=every, scheme=scheme)
    h.init_finest(orc.init_quadrant(256, G, inputs.quadrant_states(3)))
    return h


def test_regrid_interval_one_is_the_default(orc):
    a, b = quadrant(orc, 1), quadrant(orc, 1)
    for _ in range(6):
        a.step(0.45)
        b.step(0.45, regrid=None)
    for l in range(a.L):
        assert np.array_equal(a.level(l), b.level(l)) and np.array_equal(a.active(l), b.active(l))


@pytest.mark.parametrize("every,scheme", [(3, 0), (2, 1)])
def test_hierarchy_fixed_between_regrids(orc, every, scheme):
    h = quadrant(orc, every, scheme=scheme)
    masks = [h.active(l).copy() for l in range(h.L)]
    changed = 0
    for n in range(1, 4 * every + 1):
        before = h.level(h.L - 1).copy()
        h.step(0.45, regrid=None)
        assert h.nsteps == n
        now = [h.active(l) for l in range(h.L)]
        same = all(np.array_equal(a, b) for a, b in zip(masks, now))
        if n % every:
            assert same, n   # no regrid after this step
        else:
            changed += 0 if same else 1
            check_hierarchy(h)
        assert not np.array_equal(before, h.level(h.L - 1))   # the solution moves every step
        masks = [m.copy() for m in now]
    assert changed >= 2   # the fronts move the hierarchy at (most) regrids


def test_regrid_interval_conserves(orc):
    h = quadrant(orc, 3, bc=orc.BC_PERIODIC)
    T0 = h.totals()
    for _ in range(9):
        h.step(0.4, regrid=None)
    assert np.all(np.abs(h.totals() - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0)))


def test_regrid_interval_lts(orc):
    h = orc.Hierarchy(2, 3, 32, eps=1e-3, regrid_every=2)
    h.init_finest(orc.init_quadrant(128, G, inputs.quadrant_states(5)))
    masks = [h.active(l).copy() for l in range(h.L)]
    h.step_lts(0.4, regrid=None)
    assert all(np.array_equal(a, h.active(l)) for l, a in enumerate(masks))
    h.step_lts(0.4, regrid=None)
    assert h.nsteps == 2
    check_hierarchy(h)
