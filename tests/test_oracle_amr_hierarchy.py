"""Pins of the oracle's AMR scheme on an adaptive hierarchy (Sec. 2 scheme,
Sec. 2.2 hierarchy, global time step): every leaf advanced by one
MUSCL-Hancock step, a face next to a covered cell taking the mean of the
finer level's fluxes (each with the finer level's half-step predictor), then
the projection and the refinement.  Pinned by what fixes it from outside:
with every cell refined the run is the uniform finest-grid run bit for bit,
with none the uniform coarse run; with periodic boundaries mass, momentum and
energy are conserved to rounding while the mesh adapts; a uniform state on a
partially refined hierarchy stays uniform bit for bit; an adaptive Sod run
stays close to the uniform finest run against the exact solution.  A planted
control (a leaf taking its own level's flux next to a covered cell) shows the
conservation pin catches a missing fine-flux mean."""
import numpy as np
import pytest

from oracle import exact_riemann as er
from paper_1603_05211_amd import inputs

from test_oracle_adaptive import check_hierarchy

G = 1.4


def amr(orc, dim, L, n0, **kw):
    return orc.Hierarchy(dim, L, n0, scheme=orc.SCHEME_AMR, **kw)


def test_eps_zero_equals_uniform_finest(orc):
    """eps = 0 refines everywhere: the leaves are the finest grid, whose
    boundary is the domain's, and the step is the uniform scheme on it."""
    Qf = orc.init_quadrant(128, G, inputs.quadrant_states(4))
    h = amr(orc, 2, 3, 32, eps=0.0)
    h.init_finest(Qf)
    u = amr(orc, 2, 1, 128)
    u.init_finest(Qf)
    for _ in range(8):
        assert h.step(0.45) == u.step(0.45)
    assert np.array_equal(h.level(2), u.level(0))


def test_eps_huge_equals_uniform_coarse(orc):
    Qf = orc.init_quadrant(128, G, inputs.quadrant_states(4))
    h = amr(orc, 2, 3, 32, eps=1e30)
    h.init_finest(Qf)
    assert len(h.patches()) == 0
    u = amr(orc, 2, 1, 32)
    u.init_finest(orc.restrict(2, orc.restrict(2, Qf)))
    for _ in range(8):
        assert h.step(0.45) == u.step(0.45)
    assert np.array_equal(h.level(0), u.level(0))


def bump(orc, n=128):
    """A Gaussian density bump advected diagonally on [0,1]^2: the patch
    boundary crosses smooth gradients, so coarse and fine fluxes differ at
    every refinement boundary."""
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.3 * np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.01)
    W = np.stack([rho, np.full_like(rho, 0.5), np.full_like(rho, 0.3), np.ones_like(rho)])
    return orc.prim2cons(2, G, W)


def conservation_run(orc, dim, steps=12, criterion=None, smooth=False):
    if dim == 2:
        Qf = bump(orc) if smooth else orc.init_quadrant(128, G, inputs.quadrant_states(6))
        kw = dict(bc=orc.BC_PERIODIC, eps=1e-3)
        if criterion is not None:
            kw.update(criterion=criterion, eps=0.05, eps_p=0.05)
        h = amr(orc, 2, 3, 32, **kw)
    else:
        e = inputs.ellipsoid(6)
        Qf = orc.init_ellipsoid(64, G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        h = amr(orc, 3, 2, 32, bc=orc.BC_PERIODIC, lo=-1.0, hi=1.0, eps=1e-3)
    h.init_finest(Qf)
    T0 = h.totals()
    npatch = []
    for _ in range(steps):
        h.step(0.4)
        npatch.append(len(h.patches()))
    return h, T0, h.totals(), npatch


@pytest.mark.parametrize("dim,smooth", [(2, False), (2, True), (3, False)])
def test_conservation_periodic(orc, dim, smooth):
    h, T0, T1, npatch = conservation_run(orc, dim, smooth=smooth)
    check_hierarchy(h, periodic=True)
    assert min(npatch) > 0
    assert len(set(npatch)) > 1 or dim == 3 or smooth   # the mesh adapts while conserving
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_conservation_periodic_gradient_criterion(orc):
    """The AMR method proper: AMR scheme with the scaled-gradient criterion."""
    h, T0, T1, npatch = conservation_run(orc, 2, criterion=orc.CRIT_GRADIENT)
    check_hierarchy(h, periodic=True)
    assert min(npatch) > 0
    assert np.all(np.abs(T1 - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_conservation_catches_missing_fine_mean(orc):
    with orc.planted(orc.PLANT_NO_FINE_MEAN):
        _, T0, T1, _ = conservation_run(orc, 2, steps=4, smooth=True)
    rel = np.abs(T1 - T0) / np.maximum(1.0, np.abs(T0))
    assert rel.max() > 1e-8, rel


def test_free_stream_bitwise(orc):
    """A uniform state on a partially refined hierarchy stays bit-exact:
    Minmod slopes vanish, the half step adds nothing, AUSMDV of equal states
    is the physical flux, fine-flux means of equal fluxes are the flux."""
    h = amr(orc, 2, 3, 32, eps=1e-3)
    h.init_finest(orc.init_quadrant(128, G, inputs.quadrant_states(8)))
    assert len(h.patches()) > 0
    w = np.array([0.8, 0.35, -0.25, 1.1])
    q = orc.prim2cons(2, G, w.reshape(4, 1)).ravel()
    for l in range(3):
        h.level(l)[...] = q.reshape(4, 1, 1)
    for _ in range(10):
        h.step(0.45, regrid=False)
    for l in range(3):
        assert np.array_equal(h.level(l), np.broadcast_to(q.reshape(4, 1, 1), h.level(l).shape))


def test_accuracy_perturbation_sod(orc):
    """The accuracy perturbation |L1_FV - L1_a| / L1_FV (Sec. 3) of an
    adaptive AMR-scheme Sod run against the uniform finest-grid AMR-scheme
    run, both measured against the exact solution."""
    L_, R_ = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    n = 256
    Qf = orc.init_riemann1d(2, n, G, 0, L_, R_)
    t_end = 0.15
    h = amr(orc, 2, 4, 32, eps=1e-3)
    h.init_finest(Qf)
    while h.t < t_end:
        h.step(0.45, t_end)
    u = amr(orc, 2, 1, n)
    u.init_finest(Qf)
    while u.t < t_end:
        u.step(0.45, t_end)
    ex, _, _ = er.cell_averages(L_, R_, n, t_end)
    l1a = np.abs(h.composite()[0] - ex[None, :]).sum() / n ** 2
    l1u = np.abs(u.level(0)[0] - ex[None, :]).sum() / n ** 2
    leaves, _ = h.counts()
    assert leaves.sum() < 0.5 * n * n   # it did adapt
    assert abs(l1u - l1a) / l1u < 0.15, (l1u, l1a)
