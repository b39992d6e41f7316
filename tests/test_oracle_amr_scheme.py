"""Pins of the oracle's AMR scheme (Sec. 2: unsplit MUSCL-Hancock with the
Minmod limiter in primitive variables and the AUSMDV flux of Wada and Liou
1997) against what the mathematics fixes: the minmod function, the
Rankine-Hugoniot relations of the exact Riemann solution (physical flux),
consistency, upwinding and exact contact resolution of AUSMDV, Wada-Liou's
blended form of the split functions, convergence to exact Riemann solutions,
second order on a smooth wave, exact reduction to 1D, symmetry, conservation
and free stream.  Planted-mistake controls show the AUSMDV weights and the
Hancock half step are caught."""
import math

import numpy as np
import pytest

from oracle import exact_riemann as er
from paper_1603_05211_amd import inputs

G = 1.4


def phys_flux_def(w, axis, g=G):
    """f_axis(q) written from the flux vectors: (rho v_n, rho v v_n + p e_n,
    (rho e + p) v_n)."""
    dim = len(w) - 2
    rho, v, p = w[0], np.asarray(w[1:1 + dim]), w[-1]
    rhoe = p / (g - 1) + 0.5 * rho * float(v @ v)
    vn = v[axis]
    f = [rho * vn]
    for k in range(dim):
        f.append(rho * v[k] * vn + (p if k == axis else 0.0))
    f.append((rhoe + p) * vn)
    return np.array(f)


def close(a, b, rel=1e-13):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() <= rel * scale


# --------------------------------------------------------------------------
# pointwise pieces
# --------------------------------------------------------------------------

def test_minmod_is_the_minmod_function(orc):
    rng = np.random.default_rng(3)
    vals = np.concatenate([rng.normal(size=400), [0.0, 0.0, 1.0, -1.0, 2.0, 2.0]])
    for _ in range(2000):
        wm, w0, wp = rng.choice(vals, 3)
        a, b = w0 - wm, wp - w0
        ref = 0.5 * (np.sign(a) + np.sign(b)) * min(abs(a), abs(b))
        assert orc.minmod(wm, w0, wp) == ref, (wm, w0, wp)


def test_physical_flux_obeys_rankine_hugoniot(orc):
    """Across the right shock of an exact Riemann solution the oracle's
    physical flux jumps by the shock speed times the jump of the conserved
    state (Sec. 2 conservation law)."""
    for L, R in [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)), ((1.2, 0.4, 2.0), (0.5, -0.3, 0.4))]:
        ps, us = er.star_state(L, R)
        # right-star and right states, just either side of the right shock
        xi = np.linspace(us + 1e-9, 20.0, 200001)
        rho, u, p = er.sample(L, R, xi)
        j = int(np.argmax(np.abs(np.diff(rho))))
        wa = [rho[j], u[j], 0.0, p[j]]
        wb = [rho[j + 1], u[j + 1], 0.0, p[j + 1]]
        qa, qb = orc.prim2cons(2, G, np.array(wa)), orc.prim2cons(2, G, np.array(wb))
        fa, fb = orc.phys_flux(2, G, 0, wa), orc.phys_flux(2, G, 0, wb)
        S = (fa[0] - fb[0]) / (qa[0] - qb[0])
        assert np.allclose(fa - fb, S * (qa - qb), rtol=1e-9, atol=1e-9)


def _states(rng, dim, n, mach=(0.0, 0.9)):
    out = []
    for _ in range(n):
        rho = rng.uniform(0.2, 3.0)
        p = rng.uniform(0.1, 3.0)
        c = math.sqrt(G * p / rho)
        v = rng.uniform(-1, 1, dim)
        v = v / max(np.linalg.norm(v), 1e-12) * rng.uniform(*mach) * c
        out.append(np.array([rho, *v, p]))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_ausmdv_consistency(orc, dim):
    rng = np.random.default_rng(5 + dim)
    for w in _states(rng, dim, 300, (0.0, 2.5)):
        for ax in range(dim):
            assert close(orc.ausmdv(dim, G, ax, w, w), phys_flux_def(w, ax), 4e-15), (w, ax)


@pytest.mark.parametrize("dim", [2, 3])
def test_ausmdv_supersonic_upwinding(orc, dim):
    rng = np.random.default_rng(11 + dim)
    for _ in range(200):
        wl, wr = _states(rng, dim, 2, (0.0, 0.5))
        ax = int(rng.integers(dim))
        cm = max(math.sqrt(G * wl[-1] / wl[0]), math.sqrt(G * wr[-1] / wr[0]))
        sgn = 1 if rng.uniform() < 0.5 else -1
        wl[1 + ax] = sgn * cm * rng.uniform(1.05, 3.0)
        wr[1 + ax] = sgn * cm * rng.uniform(1.05, 3.0)
        F = orc.ausmdv(dim, G, ax, wl, wr)
        ref = phys_flux_def(wl if sgn > 0 else wr, ax)
        assert close(F, ref, 1e-14), (wl, wr, F, ref)


def test_ausmdv_stationary_contact(orc):
    """u = 0 and equal pressure on both sides, a density and tangential
    velocity jump: no mass, tangential momentum or energy crosses the face,
    the normal momentum flux is the pressure."""
    rng = np.random.default_rng(17)
    for _ in range(200):
        p = rng.uniform(0.1, 3.0)
        wl = np.array([rng.uniform(0.1, 3.0), 0.0, rng.uniform(-1, 1), p])
        wr = np.array([rng.uniform(0.1, 3.0), 0.0, rng.uniform(-1, 1), p])
        F = orc.ausmdv(2, G, 0, wl, wr)
        scale = p + wl[0] + wr[0]
        assert abs(F[0]) <= 1e-15 * scale and abs(F[2]) <= 1e-15 * scale and abs(F[3]) <= 1e-14 * scale
        assert abs(F[1] - p) <= 1e-15 * scale


def test_ausmdv_moving_contact_is_the_exact_upwind_flux(orc):
    """A contact moving at subsonic speed u (equal u and p, density and
    tangential velocity jumps): the flux equals the physical flux of the
    upwind state.  This holds only with the pressure-ratio weights alpha and
    the balanced pressure polynomials."""
    rng = np.random.default_rng(19)
    for dim in (2, 3):
        for _ in range(300):
            p = rng.uniform(0.1, 3.0)
            rl, rr = rng.uniform(0.1, 3.0, 2)
            cmin = math.sqrt(G * p / max(rl, rr))
            u = rng.uniform(-0.95, 0.95) * cmin
            ax = int(rng.integers(dim))
            wl = np.array([rl, *rng.uniform(-1, 1, dim), p])
            wr = np.array([rr, *rng.uniform(-1, 1, dim), p])
            wl[1 + ax] = wr[1 + ax] = u
            F = orc.ausmdv(dim, G, ax, wl, wr)
            ref = phys_flux_def(wl if u >= 0 else wr, ax)
            assert close(F, ref, 1e-13), (dim, wl, wr, F, ref)


def _ausmdv_blended(wl, wr, ax, g=G, K=10.0):
    """AUSMDV written in Wada-Liou's blended form: u+ = a (u + c)^2 / 4c +
    (1 - a)(u + |u|)/2, the pressure polynomial expanded as
    p [ (1 +- M)/2 +- M (1 - M^2)/4 ], momentum (1/2 + s) AUSMV + (1/2 - s)
    AUSMD, every other quantity upwinded with the mass flux."""
    dim = len(wl) - 2
    rl, pl, ul = wl[0], wl[-1], wl[1 + ax]
    rr, pr, ur = wr[0], wr[-1], wr[1 + ax]
    cm = max(math.sqrt(g * pl / rl), math.sqrt(g * pr / rr))
    al = 2 * (pl / rl) / (pl / rl + pr / rr)
    ar = 2 * (pr / rr) / (pl / rl + pr / rr)
    if abs(ul) <= cm:
        Ml = ul / cm
        up = al * (ul + cm) ** 2 / (4 * cm) + (1 - al) * 0.5 * (ul + abs(ul))
        pp = pl * (0.5 * (1 + Ml) + 0.25 * Ml * (1 - Ml * Ml))
    else:
        up = 0.5 * (ul + abs(ul))
        pp = pl * 0.5 * (ul + abs(ul)) / ul
    if abs(ur) <= cm:
        Mr = ur / cm
        um = -ar * (ur - cm) ** 2 / (4 * cm) + (1 - ar) * 0.5 * (ur - abs(ur))
        pm = pr * (0.5 * (1 - Mr) - 0.25 * Mr * (1 - Mr * Mr))
    else:
        um = 0.5 * (ur - abs(ur))
        pm = pr * 0.5 * (ur - abs(ur)) / ur
    m = up * rl + um * rr
    s = 0.5 * min(1.0, K * abs(pr - pl) / min(pl, pr))
    mom = (0.5 + s) * (up * rl * ul + um * rr * ur) + (0.5 - s) * 0.5 * (m * (ul + ur) - abs(m) * (ur - ul))
    H = lambda w: (w[-1] / (g - 1) + 0.5 * w[0] * float(np.dot(w[1:1 + dim], w[1:1 + dim])) + w[-1]) / w[0]
    up_ = lambda a, b: 0.5 * (m * (a + b) - abs(m) * (b - a))
    F = [m]
    for k in range(dim):
        F.append(mom + pp + pm if k == ax else up_(wl[1 + k], wr[1 + k]))
    F.append(up_(H(wl), H(wr)))
    return np.array(F)


def _ausmdv_max_dev(orc, seed=23):
    rng = np.random.default_rng(seed)
    dev = 0.0
    for dim in (2, 3):
        for _ in range(300):
            wl, wr = _states(rng, dim, 2, (0.0, 1.4))
            ax = int(rng.integers(dim))
            F = orc.ausmdv(dim, G, ax, wl, wr)
            ref = _ausmdv_blended(wl, wr, ax)
            dev = max(dev, np.abs(F - ref).max() / max(np.abs(ref).max(), 1e-300))
    return dev


def test_ausmdv_matches_blended_form(orc):
    assert _ausmdv_max_dev(orc) < 1e-12


def test_ausmdv_pins_catch_unit_weights(orc):
    """With alpha_L = alpha_R = 1 planted the blended-form and moving-contact
    pins fail."""
    with orc.planted(orc.PLANT_AUSMDV_ALPHA):
        assert _ausmdv_max_dev(orc) > 1e-4
        wl, wr = np.array([2.0, 0.3, 0.0, 1.0]), np.array([0.5, 0.3, 0.0, 1.0])
        F = orc.ausmdv(2, G, 0, wl, wr)
        assert not close(F, phys_flux_def(wl, 0), 1e-6)


# --------------------------------------------------------------------------
# the scheme
# --------------------------------------------------------------------------

def run_amr(orc, dim, n, Q0, steps=None, t_end=np.inf, cfl=0.45, bc=0, lo=0.0, hi=1.0, dt=None):
    h = orc.Hierarchy(dim, 1, n, bc=bc, lo=lo, hi=hi, scheme=orc.SCHEME_AMR)
    h.init_finest(Q0)
    if dt is not None:
        for _ in range(steps):
            h.step_fixed(dt)
        return h
    k = 0
    while h.t < t_end and (steps is None or k < steps):
        h.step(cfl, t_end)
        k += 1
    return h


@pytest.mark.parametrize("axis", [0, 1])
def test_hancock_sod_converges_to_exact_solution(orc, axis):
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for n in (32, 64, 128):
        Q0 = orc.init_riemann1d(2, n, G, axis, L, R)
        h = run_amr(orc, 2, n, Q0, t_end=0.2)
        rho = h.level(0)[0]
        line = rho[0, :] if axis == 0 else rho[:, 0]
        assert np.array_equal(rho, np.broadcast_to(line[None, :] if axis == 0 else line[:, None], rho.shape))
        ex_rho, _, _ = er.cell_averages(L, R, n, 0.2)
        errs.append(np.abs(line - ex_rho).sum() / n)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[-1] < 0.01
    assert all(0.5 <= r <= 1.4 for r in rates), (errs, rates)


def test_hancock_seeded_riemann_problems_converge(orc):
    """Seeded 1D Riemann problems: the error falls with the grid, and on the
    finer grid it is at most 1.3 times the MR scheme's (Sec. 2: the
    MUSCL-Hancock method is slightly less accurate)."""
    for seed in (0, 1, 2):
        L, R = inputs.riemann_1d(seed)
        errs, mr = [], None
        for n in (64, 128):
            Q0 = orc.init_riemann1d(2, n, G, 0, L, R)
            h = run_amr(orc, 2, n, Q0, t_end=0.1)
            ex_rho, _, _ = er.cell_averages(L, R, n, 0.1)
            errs.append(np.abs(h.level(0)[0][0] - ex_rho).sum() / n)
            if n == 128:
                g = orc.Hierarchy(2, 1, n)
                g.init_finest(Q0)
                while g.t < 0.1:
                    g.step(0.45, 0.1)
                mr = np.abs(g.level(0)[0][0] - ex_rho).sum() / n
        assert errs[1] < errs[0] * 0.73, (seed, errs)
        assert errs[1] < 1.3 * mr and errs[1] < 0.025 * max(L[0], R[0]), (seed, errs, mr)


def test_hancock_2d_3d_reduce_to_same_1d_solution(orc):
    L, R = (1.0, 0.3, 1.0), (0.3, -0.2, 0.5)
    n = 16
    h2 = run_amr(orc, 2, n, orc.init_riemann1d(2, n, G, 0, L, R), steps=10, dt=0.004)
    h3 = run_amr(orc, 3, n, orc.init_riemann1d(3, n, G, 0, L, R), steps=10, dt=0.004)
    a2, a3 = h2.level(0), h3.level(0)
    for f2, f3 in [(0, 0), (1, 1), (3, 4)]:
        assert np.array_equal(a3[f3], np.broadcast_to(a2[f2][None], a3[f3].shape))
    assert np.all(a3[2] == 0) and np.all(a3[3] == 0)


def test_hancock_transpose_symmetry_bitwise(orc):
    n = 32
    Q = orc.init_quadrant(n, G, inputs.quadrant_states(7))
    QT = np.ascontiguousarray(np.stack([Q[0].T, Q[2].T, Q[1].T, Q[3].T]))
    h1 = run_amr(orc, 2, n, Q, steps=5, dt=0.002)
    h2 = run_amr(orc, 2, n, QT, steps=5, dt=0.002)
    A, B = h1.level(0), h2.level(0)
    assert np.array_equal(A[0], B[0].T) and np.array_equal(A[3], B[3].T)
    assert np.array_equal(A[1], B[2].T) and np.array_equal(A[2], B[1].T)


def _smooth_rates(orc):
    errs = []
    t_end = 0.25
    for n in (32, 64, 128):
        x = np.arange(n + 1) / n
        avg = lambda xe, t: 1 + 0.2 * (-np.cos(2 * np.pi * (xe[1:] - t)) + np.cos(2 * np.pi * (xe[:-1] - t))) / (2 * np.pi * (xe[1:] - xe[:-1]))
        rho = np.broadcast_to(avg(x, 0.0)[None, :], (n, n))
        W = np.stack([rho, np.ones((n, n)), np.zeros((n, n)), np.ones((n, n))])
        h = orc.Hierarchy(2, 1, n, bc=orc.BC_PERIODIC, scheme=orc.SCHEME_AMR)
        h.init_finest(orc.prim2cons(2, G, W))
        dt = 0.2 / n
        steps = int(round(t_end / dt))
        for _ in range(steps):
            h.step_fixed(dt)
        errs.append(np.abs(h.level(0)[0][0] - avg(x, steps * dt)).sum() / n)
    return errs, [math.log2(errs[i] / errs[i + 1]) for i in range(2)]


def test_hancock_smooth_advection_second_order(orc):
    """The advected density wave rho = 1 + 0.2 sin(2 pi (x - t)) (closed-form
    cell averages): MUSCL-Hancock is second order in time through its half
    step (Minmod clips the extrema, so the order is measured at 1.6)."""
    errs, rates = _smooth_rates(orc)
    assert rates[-1] > 1.6, (errs, rates)


def test_hancock_pin_catches_missing_half_step(orc):
    with orc.planted(orc.PLANT_HANCOCK_NOPRED):
        errs, rates = _smooth_rates(orc)
    assert not (rates[-1] > 1.6 and errs[-1] < 1e-3), (errs, rates)


def test_hancock_conservation_periodic(orc):
    prim = inputs.quadrant_states(3)
    for dim, n in ((2, 48), (3, 12)):
        if dim == 2:
            Q = orc.init_quadrant(n, G, prim)
        else:
            e = inputs.ellipsoid(3)
            Q = orc.init_ellipsoid(n, G, e.a, e.b, e.c, e.theta, e.phi, e.states)
        h = orc.Hierarchy(dim, 1, n, bc=orc.BC_PERIODIC, lo=0.0 if dim == 2 else -1.0, scheme=orc.SCHEME_AMR)
        h.init_finest(Q)
        T0 = h.totals()
        for _ in range(30):
            h.step(0.4)
        T1 = h.totals()
        assert np.all(np.abs(T1 - T0) <= 1e-13 * np.maximum(1.0, np.abs(T0))), (T0, T1)


def test_hancock_free_stream_bitwise(orc):
    for dim in (2, 3):
        n = 16
        w = [0.9, 0.3, -0.7, 1.3] if dim == 2 else [0.9, 0.3, -0.7, 0.2, 1.3]
        Q0 = orc.prim2cons(dim, G, np.stack([np.full((n,) * dim, v) for v in w]))
        h = run_amr(orc, dim, n, Q0, steps=20)
        # the half step adds f(W) - f(W) = 0; AUSMDV(w, w) = f(w) on every face
        assert np.allclose(h.level(0), Q0, rtol=0, atol=4e-15 * np.abs(Q0).max())


def test_hancock_stationary_contact_preserved(orc):
    n = 32
    W = np.zeros((4, n, n))
    W[0] = np.where(np.arange(n)[None, :] < n // 2, 1.0, 0.2)
    W[3] = 0.7
    Q0 = orc.prim2cons(2, G, W)
    h = run_amr(orc, 2, n, Q0, steps=20)
    assert np.allclose(h.level(0), Q0, rtol=0, atol=1e-14)


def test_hancock_3d_axes_agree_bitwise(orc):
    """1D Riemann data along z in 3D gives, bit for bit, the solution along x
    with the momentum components exchanged: the flux differences, slopes and
    half-step terms of the other axes are exact zeros, so the z-axis code
    (face states, evolution and fluxes along z) is pinned by the x-axis one."""
    L, R = (1.0, 0.3, 1.0), (0.3, -0.2, 0.5)
    n = 16
    hx = run_amr(orc, 3, n, orc.init_riemann1d(3, n, G, 0, L, R), steps=8, dt=0.004)
    hz = run_amr(orc, 3, n, orc.init_riemann1d(3, n, G, 2, L, R), steps=8, dt=0.004)
    ax, az = hx.level(0), hz.level(0)
    # x-data varies along the last array axis, z-data along the first
    assert np.array_equal(ax[0], np.transpose(az[0], (2, 1, 0)))
    assert np.array_equal(ax[1], np.transpose(az[3], (2, 1, 0)))
    assert np.array_equal(ax[4], np.transpose(az[4], (2, 1, 0)))
    assert np.all(az[1] == 0) and np.all(az[2] == 0)
