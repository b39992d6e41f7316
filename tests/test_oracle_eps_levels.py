"""Pins of the oracle's level-dependent MR thresholds (a variant; the paper's
runs apply one eps on every level): eps_l = 2^(d (l + 2 - L)) eps for the
details of level l.  Independent numpy details and thresholds give the raw
flags every level's flags must contain (and, on the finest analysed level,
equal after the buffer); two levels reduce to the constant threshold bit
for bit; the smaller coarse thresholds refine at least where the constant
one does; the MR reconstruction error stays below the constant threshold's
on smooth data."""
import numpy as np

from paper_1603_05211_amd import inputs

from test_oracle_adaptive import dilate

G = 1.4


def details_np(orc, lev, l):
    pred = orc.predict(2, lev[l])[0]
    err = np.abs(lev[l + 1][0] - pred)
    n = lev[l].shape[-1]
    return err.reshape(n, 2, n, 2).max(axis=(1, 3))


def test_flags_follow_level_thresholds(orc):
    L, n0, eps = 4, 32, 2e-3
    Qf = orc.init_quadrant(n0 << (L - 1), G, inputs.quadrant_states(1))
    h = orc.Hierarchy(2, L, n0, eps=eps, eps_levels=True)
    h.init_finest(Qf)
    lev = [None] * L
    lev[L - 1] = Qf
    for l in range(L - 2, -1, -1):
        lev[l] = orc.restrict(2, lev[l + 1])
    thr = [eps * 2.0 ** (2 * (l + 2 - L)) for l in range(L - 1)]
    assert thr[L - 2] == eps and thr[0] == eps / 16
    for l in range(L - 1):
        D = details_np(orc, lev, l)
        assert np.array_equal(D, h.details(l))
        raw = D >= thr[l]
        if l >= 1:
            raw |= np.repeat(np.repeat(details_np(orc, lev, l - 1) >= thr[l - 1], 2, 0), 2, 1)
        F = h.flags(l).astype(bool)
        assert not (dilate(raw, 1) & ~F).any(), l
        if l == L - 2:
            assert np.array_equal(dilate(raw, 1), F)


def test_two_levels_equal_constant_threshold(orc):
    Qf = orc.init_quadrant(64, G, inputs.quadrant_states(3))
    a = orc.Hierarchy(2, 2, 32, eps=1e-3, eps_levels=True)
    b = orc.Hierarchy(2, 2, 32, eps=1e-3)
    a.init_finest(Qf)
    b.init_finest(Qf)
    for _ in range(6):
        assert a.step(0.45) == b.step(0.45)
    assert np.array_equal(a.level(1), b.level(1)) and np.array_equal(a.patches(), b.patches())


def smooth_front(orc, n=256, width=0.05):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.3 * np.tanh((X + 0.5 * Y - 0.7) / width)
    W = np.stack([rho, np.full_like(rho, 0.1), np.full_like(rho, -0.2), np.ones_like(rho)])
    return orc.prim2cons(2, G, W)


def test_level_thresholds_refine_at_least_as_much(orc):
    """On a smooth front the details shrink level by level; the smaller
    coarse thresholds keep more coarse cells significant."""
    Qf = smooth_front(orc)
    a = orc.Hierarchy(2, 4, 32, eps=1e-3, eps_levels=True)
    b = orc.Hierarchy(2, 4, 32, eps=1e-3)
    a.init_finest(Qf)
    b.init_finest(Qf)
    grew = False
    for l in range(4):
        A, B = a.active(l).astype(bool), b.active(l).astype(bool)
        assert not (B & ~A).any(), l
        grew |= bool((A & ~B).any())
    assert grew


def test_reconstruction_error_below_constant_threshold(orc):
    Qf = smooth_front(orc)
    errs = {}
    for lv in (False, True):
        h = orc.Hierarchy(2, 4, 32, eps=3e-3, eps_levels=lv)
        h.init_finest(Qf)
        errs[lv] = np.abs(h.composite()[0] - Qf[0]).mean()
    assert errs[True] <= errs[False], errs
