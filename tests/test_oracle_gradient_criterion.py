"""Pins of the oracle's AMR refinement criterion (Sec. 2.2): the scaled
gradient indicators |w(Q_{i+a}) - w(Q_i)| > eps_w, a in {0,1}^d, for w = rho
and w = p, followed by the one-cell buffer, the nesting closure and the
efficiency-rule tiling the hierarchy already has.  Independent numpy brute
force of the indicators and of the flags they give on the initial analysis;
strictness of the threshold; density only versus density and pressure;
monotonicity; constant data; adaptive runs conserve, keep a free stream and
stay close to the uniform finest run."""
import numpy as np
import pytest

from paper_1603_05211_amd import inputs

from test_oracle_adaptive import check_hierarchy, dilate

G = 1.4


def restrict_np(A, dim):
    """Mean of the 2^d children, in the oracle's pairwise order."""
    if dim == 2:
        return 0.25 * ((A[:, 0::2, 0::2] + A[:, 0::2, 1::2]) + (A[:, 1::2, 0::2] + A[:, 1::2, 1::2]))
    return 0.125 * (((A[:, 0::2, 0::2, 0::2] + A[:, 0::2, 0::2, 1::2]) + (A[:, 0::2, 1::2, 0::2] + A[:, 0::2, 1::2, 1::2]))
                    + ((A[:, 1::2, 0::2, 0::2] + A[:, 1::2, 0::2, 1::2]) + (A[:, 1::2, 1::2, 0::2] + A[:, 1::2, 1::2, 1::2])))


def pressure_np(Q, dim):
    """p = (gamma - 1) (E - (rho / 2) K), K = ((v1 v1 + v2 v2) + v3 v3)."""
    rho = Q[0]
    K = np.zeros_like(rho)
    for d in range(dim):
        v = Q[1 + d] / rho
        K = K + v * v
    return (G - 1.0) * (Q[dim + 1] - (0.5 * rho) * K)


def indicators_np(Q, dim):
    """Largest |rho(P + a) - rho(P)| and |p(P + a) - p(P)| over a in {0,1}^d,
    a != 0, with the outflow boundary map (clamped indices)."""
    n = Q.shape[-1]
    rho, p = Q[0], pressure_np(Q, dim)
    dr = np.zeros_like(rho)
    dp = np.zeros_like(rho)
    idx = np.minimum(np.arange(n) + 1, n - 1)
    for a in range(1, 1 << dim):
        sl = []
        for ax in range(dim):
            # array axes are (z,) y, x; bit 0 of a is x
            bit = (a >> (dim - 1 - ax)) & 1
            sl.append(idx if bit else np.arange(n))
        mesh = np.ix_(*sl)
        dr = np.maximum(dr, np.abs(rho[mesh] - rho))
        dp = np.maximum(dp, np.abs(p[mesh] - p))
    return dr, dp


@pytest.mark.parametrize("dim,use_p", [(2, False), (2, True), (3, True)])
def test_indicators_and_flags_brute_force(orc, dim, use_p):
    """On the initial analysis every level holds the restricted initial data
    and every cell is present: the oracle's largest density differences and
    its finest flags equal an independent numpy evaluation."""
    if dim == 2:
        L, n0 = 4, 16
        Qf = orc.init_quadrant(n0 << (L - 1), G, inputs.quadrant_states(3))
        eps, eps_p = 0.05, (0.05 if use_p else 0.0)
    else:
        L, n0 = 3, 8
        e = inputs.ellipsoid(1)
        Qf = orc.init_ellipsoid(n0 << (L - 1), G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        eps, eps_p = 0.05, 0.05
    h = orc.Hierarchy(dim, L, n0, lo=0.0 if dim == 2 else -1.0, eps=eps, criterion=orc.CRIT_GRADIENT,
                      eps_p=eps_p, pmax=16 if dim == 3 else 32)
    h.init_finest(Qf)
    lev = [None] * L
    lev[L - 1] = Qf
    for l in range(L - 2, -1, -1):
        lev[l] = restrict_np(lev[l + 1], dim)
    for l in range(L - 1):
        dr, dp = indicators_np(lev[l], dim)
        assert np.array_equal(dr, h.details(l)), l
        raw = (dr > eps) | ((dp > eps_p) if eps_p > 0 else False)
        F = h.flags(l).astype(bool)
        # every raw flag and its one-cell buffer is flagged
        assert not (dilate(raw, 1) & ~F).any(), l
        if l == L - 2:   # no finer level: exactly the buffered raw flags
            assert np.array_equal(dilate(raw, 1), F)
    check_hierarchy(h)


def test_threshold_is_strict_and_pressure_counts(orc):
    """A pure pressure jump of size 0.2 (density, velocity constant): flagged
    with eps_p < 0.2, not with eps_p = 0.2 (strict), never by density alone."""
    n0, L = 16, 3
    nf = n0 << (L - 1)
    W = np.stack([np.full((nf, nf), 1.0), np.zeros((nf, nf)), np.zeros((nf, nf)), np.full((nf, nf), 1.0)])
    W[3][:, nf // 2:] = 1.2   # aligned: every coarser level keeps the sharp 0.2 jump
    Qf = orc.prim2cons(2, G, W)
    for eps_p, expect in ((0.0, False), (0.19, True), (0.2, False)):
        h = orc.Hierarchy(2, L, n0, eps=0.05, criterion=orc.CRIT_GRADIENT, eps_p=eps_p)
        h.init_finest(Qf)
        assert (len(h.patches()) > 0) == expect, (eps_p, len(h.patches()))


def test_gradient_threshold_monotone_and_constant_data(orc):
    Qf = orc.init_quadrant(128, G, inputs.quadrant_states(2))
    prev = None
    for eps in (0.01, 0.05, 0.2, 0.5):
        h = orc.Hierarchy(2, 3, 32, eps=eps, criterion=orc.CRIT_GRADIENT, eps_p=eps)
        h.init_finest(Qf)
        acts = [h.active(l).astype(bool) for l in range(3)]
        if prev is not None:
            for a, b in zip(acts, prev):
                assert not (a & ~b).any()
        prev = acts
    W = np.stack([np.full((128, 128), v) for v in (1.0, 0.2, 0.1, 1.0)])
    h = orc.Hierarchy(2, 3, 32, eps=1e-14, criterion=orc.CRIT_GRADIENT, eps_p=1e-14)
    h.init_finest(orc.prim2cons(2, G, W))
    assert len(h.patches()) == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_adaptive_conservation_periodic(orc, dim):
    if dim == 2:
        Q = orc.init_quadrant(128, G, inputs.quadrant_states(4))
        h = orc.Hierarchy(2, 3, 32, bc=orc.BC_PERIODIC, eps=0.05, criterion=orc.CRIT_GRADIENT, eps_p=0.05)
    else:
        e = inputs.ellipsoid(4)
        Q = orc.init_ellipsoid(32, G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        h = orc.Hierarchy(3, 3, 8, bc=orc.BC_PERIODIC, lo=-1.0, eps=0.05, criterion=orc.CRIT_GRADIENT,
                          eps_p=0.05, pmax=16)
    h.init_finest(Q)
    T0 = h.totals()
    for _ in range(10):
        h.step(0.4)
        check_hierarchy(h, periodic=True)
    T1 = h.totals()
    assert np.all(np.abs(T1 - T0) <= 1e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_gradient_adaptive_free_stream_and_accuracy(orc):
    """A uniform state refines nothing and stays exactly uniform; on the
    four-quadrant data the adaptive run with the paper's 2D threshold
    (eps_rho = 0.05) stays within 15 % of the uniform finest run's L1 density
    distance to a fine reference (the accuracy perturbation of Sec. 3)."""
    W = np.stack([np.full((128, 128), v) for v in (0.9, 0.3, -0.7, 1.3)])
    Q0 = orc.prim2cons(2, G, W)
    h = orc.Hierarchy(2, 3, 32, eps=0.05, criterion=orc.CRIT_GRADIENT)
    h.init_finest(Q0)
    for _ in range(10):
        h.step(0.45)
    assert len(h.patches()) == 0 and np.array_equal(h.level(0), orc.restrict(2, orc.restrict(2, Q0)))
    prim = inputs.quadrant_states(0)
    t_end = 0.1
    ref = orc.Hierarchy(2, 1, 512)
    ref.init_finest(orc.init_quadrant(512, G, prim))
    while ref.t < t_end:
        ref.step(0.45, t_end)
    r = orc.restrict(2, ref.level(0))
    uni = orc.Hierarchy(2, 1, 256)
    uni.init_finest(orc.init_quadrant(256, G, prim))
    while uni.t < t_end:
        uni.step(0.45, t_end)
    ada = orc.Hierarchy(2, 4, 32, eps=0.05, criterion=orc.CRIT_GRADIENT)
    ada.init_finest(orc.init_quadrant(256, G, prim))
    while ada.t < t_end:
        ada.step(0.45, t_end)
    e_u = np.abs(uni.level(0)[0] - r[0]).mean()
    e_a = np.abs(ada.composite()[0] - r[0]).mean()
    assert e_a <= 1.15 * e_u, (e_a, e_u)
