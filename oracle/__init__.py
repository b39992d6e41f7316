"""Plain FP64 CPU oracle of the adaptive finite-volume Euler method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the GPU library (``paper_1603_05211_amd``) and imports nothing from
it.  The numerics live in ``oracle.c`` (plain C, one cell at a time); this
module only marshals numpy arrays through ctypes.

What pins each part (tests/test_oracle_pins.py, tests/test_oracle_adaptive.py):

* primitive/conserved maps ....... definitions of Sec. 2 (round trip, closed forms)
* van Albada slope ............... limiter function phi(r) = (r^2 + r)/(r^2 + 1)
* AUSM+ flux ..................... consistency F(w, w) = f(w) with the physical
                                   flux; supersonic upwinding; exact stationary contact;
                                   Liou's expanded split polynomials (alpha, beta) on
                                   asymmetric subsonic pairs
* MUSCL + AUSM+ + midpoint RK2 ... exact Riemann solutions (Sod, seeded), order on a
                                   smooth periodic wave, exact 2D/3D reduction to 1D,
                                   transpose symmetry, conservation, free stream
* CFL time step .................. closed form for a uniform state
* totals ......................... exact sum (math.fsum)
* restriction / prediction ....... mean of children; exact-rational bi- and
                                   triquadratic interpolation; exact on 2D and 3D
                                   tensor quadratics; conservative
* details / flags / tiling ....... independent detail computation, flag coverage,
                                   the efficiency rule, nesting, gradedness,
                                   threshold monotonicity
* adaptive step .................. eps = 0 equals the uniform finest run bit for bit,
                                   eps = inf equals the uniform coarse run, periodic
                                   conservation, free stream, accuracy perturbation
                                   (Sec. 3) against the uniform finest run
* Minmod slope .................. the minmod function (sign(a) + sign(b))/2 min(|a|, |b|)
* AUSMDV flux .................... consistency with the physical flux; supersonic
                                   upwinding; stationary contact (zero mass flux);
                                   moving contact = exact upwind flux (pins the
                                   pressure-ratio weights); Wada-Liou's blended form of
                                   the split velocities and expanded pressure polynomials
* MUSCL-Hancock + AUSMDV ......... exact Riemann solutions, second order on a smooth
                                   wave (fails without the half-step evolution),
                                   reduction to 1D, symmetry, conservation, free stream
* gradient criterion (AMR) ....... independent numpy brute force of the indicators and
                                   of the flags they give; strict threshold; density only
                                   vs density and pressure; monotone in the thresholds;
                                   adaptive runs: conservation, free stream, accuracy
* local time stepping ............ one level = global step; eps = 0 = uniform substeps;
                                   conservation; a linear profile reproduced to rounding
                                   across refinement boundaries (pins the ghost times
                                   theta); second order on a smooth wave

Planted-mistake controls (``planted``) show that the AUSM+, 3D prediction and
ghost-time pins fail when alpha = beta = 0, the z pass is mirrored, or theta
is held at 0.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_TRANSMISSIVE = 0
BC_PERIODIC = 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unused-function",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        vp = C.c_void_p
        sig = {
            "orc_prim2cons": (None, [C.c_int, C.c_double, C.c_int64, dp, dp]),
            "orc_cons2prim": (None, [C.c_int, C.c_double, C.c_int64, dp, dp]),
            "orc_ausm_plus": (None, [C.c_int, C.c_double, C.c_int, dp, dp, dp]),
            "orc_slope": (C.c_double, [C.c_double, C.c_double, C.c_double]),
            "orc_minmod": (C.c_double, [C.c_double, C.c_double, C.c_double]),
            "orc_ausmdv": (None, [C.c_int, C.c_double, C.c_int, dp, dp, dp]),
            "orc_phys_flux": (None, [C.c_int, C.c_double, C.c_int, dp, dp]),
            "orc_h_set_scheme": (C.c_int, [vp, C.c_int]),
            "orc_h_set_variants": (C.c_int, [vp, C.c_int, C.c_int]),
            "orc_h_set_tiler": (C.c_int, [vp, C.c_int]),
            "orc_h_set_cfl_mode": (C.c_int, [vp, C.c_int]),
            "orc_br_cluster": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, i32p, i32p]),
            "orc_ausm_plus_speed": (None, [C.c_int, C.c_double, C.c_int, dp, dp, dp, C.c_int]),
            "orc_h_set_eps_levels": (None, [vp, C.c_int]),
            "orc_h_set_criterion": (C.c_int, [vp, C.c_int, C.c_double]),
            "orc_restrict": (None, [C.c_int, C.c_int, C.c_int, dp, dp]),
            "orc_predict": (None, [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]),
            "orc_h_new": (vp, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]),
            "orc_h_free": (None, [vp]),
            "orc_h_level": (dp, [vp, C.c_int]),
            "orc_h_level_stage": (dp, [vp, C.c_int]),
            "orc_h_active": (u8p, [vp, C.c_int]),
            "orc_h_flags": (u8p, [vp, C.c_int]),
            "orc_h_details": (dp, [vp, C.c_int]),
            "orc_h_n": (C.c_int, [vp, C.c_int]),
            "orc_h_dx": (C.c_double, [vp, C.c_int]),
            "orc_h_restrict": (None, [vp]),
            "orc_h_ghost": (None, [vp]),
            "orc_h_cfl": (C.c_double, [vp, C.c_double, C.c_double, C.c_double, dp]),
            "orc_h_totals": (None, [vp, dp]),
            "orc_h_counts": (None, [vp, i64p, i64p]),
            "orc_h_init": (None, [vp]),
            "orc_h_regrid": (None, [vp]),
            "orc_h_analyse": (None, [vp]),
            "orc_h_set_eps": (None, [vp, C.c_double]),
            "orc_h_npatch": (C.c_int, [vp]),
            "orc_h_set_no_reflux": (None, [vp, C.c_int]),
            "orc_set_plant": (None, [C.c_int]),
            "orc_h_set_active": (None, [vp, C.c_int, u8p]),
            "orc_h_patches": (None, [vp, i32p]),
            "orc_h_stage": (None, [vp, C.c_int, C.c_double]),
            "orc_h_step": (C.c_double, [vp, C.c_double, C.c_double, C.c_double, C.c_int]),
            "orc_h_step_fixed": (None, [vp, C.c_double]),
            "orc_h_step_lts": (C.c_double, [vp, C.c_double, C.c_double, C.c_double, C.c_int, i64p]),
            "orc_init_quadrant": (None, [C.c_int, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, dp, dp]),
            "orc_init_ellipsoid": (None, [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp, dp]),
            "orc_init_riemann1d": (None, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.c_double, dp, dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


PLANT_NONE, PLANT_AUSM_AB, PLANT_PRED_ZSWAP, PLANT_LTS_THETA = 0, 1, 2, 3
PLANT_AUSMDV_ALPHA, PLANT_HANCOCK_NOPRED, PLANT_NO_FINE_MEAN = 4, 5, 6
SCHEME_MR, SCHEME_AMR = 0, 1
RK_MIDPOINT, RK_HEUN = 0, 1
AUSM_MEAN, AUSM_CRITICAL = 0, 1
TILER_BLOCKS, TILER_BR = 0, 1
CFL_SUM, CFL_MAX = 0, 1
CRIT_MR, CRIT_GRADIENT = 0, 1


class planted:
    """Context manager of the tests' planted-mistake controls: inside the
    block the oracle computes with one known mistake (see oracle.c), so a
    test can show that its pin would catch it."""

    def __init__(self, which: int):
        self.which = which

    def __enter__(self):
        lib().orc_set_plant(self.which)
        return self

    def __exit__(self, *exc):
        lib().orc_set_plant(PLANT_NONE)
        return False


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- pointwise

def prim2cons(dim: int, gamma: float, W: np.ndarray) -> np.ndarray:
    W = _f64(W)
    ncell = W.size // (dim + 2)
    Q = np.empty_like(W)
    lib().orc_prim2cons(dim, gamma, ncell, _dp(W), _dp(Q))
    return Q


def cons2prim(dim: int, gamma: float, Q: np.ndarray) -> np.ndarray:
    Q = _f64(Q)
    ncell = Q.size // (dim + 2)
    W = np.empty_like(Q)
    lib().orc_cons2prim(dim, gamma, ncell, _dp(Q), _dp(W))
    return W


def ausm_plus(dim: int, gamma: float, axis: int, wL, wR, speed: int = AUSM_MEAN) -> np.ndarray:
    """AUSM+ across a face; speed selects the interface sound speed."""
    wL, wR = _f64(wL), _f64(wR)
    F = np.empty(dim + 2)
    if speed == AUSM_MEAN:
        lib().orc_ausm_plus(dim, gamma, axis, _dp(wL), _dp(wR), _dp(F))
    else:
        lib().orc_ausm_plus_speed(dim, gamma, axis, _dp(wL), _dp(wR), _dp(F), speed)
    return F


def br_cluster(W: np.ndarray, q: int, eta: float) -> np.ndarray:
    """Berger-Rigoutsos boxes of a (R, R) or (R, R, R) grid of sub-block
    weights (index [(z,) y, x]; q^d parent cells per sub-block): rows
    {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z} in the order found."""
    W = np.ascontiguousarray(W, dtype=np.int32)
    dim, R = W.ndim, W.shape[0]
    out = np.zeros((512, 6), dtype=np.int32)
    n = lib().orc_br_cluster(dim, R, q, eta, W.ctypes.data_as(C.POINTER(C.c_int32)),
                             out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out[:n]


def slope(wm: float, w0: float, wp: float) -> float:
    return lib().orc_slope(wm, w0, wp)


def minmod(wm: float, w0: float, wp: float) -> float:
    return lib().orc_minmod(wm, w0, wp)


def ausmdv(dim: int, gamma: float, axis: int, wL, wR) -> np.ndarray:
    wL, wR = _f64(wL), _f64(wR)
    F = np.empty(dim + 2)
    lib().orc_ausmdv(dim, gamma, axis, _dp(wL), _dp(wR), _dp(F))
    return F


def phys_flux(dim: int, gamma: float, axis: int, w) -> np.ndarray:
    w = _f64(w)
    F = np.empty(dim + 2)
    lib().orc_phys_flux(dim, gamma, axis, _dp(w), _dp(F))
    return F


def restrict(dim: int, Af: np.ndarray) -> np.ndarray:
    """Af: (nv, nf, nf[, nf]) -> (nv, nf/2, ...)."""
    Af = _f64(Af)
    nv, nf = Af.shape[0], Af.shape[-1]
    nc = nf // 2
    Ac = np.empty((nv,) + (nc,) * dim)
    lib().orc_restrict(dim, nv, nc, _dp(Af), _dp(Ac))
    return Ac


def predict(dim: int, Ac: np.ndarray, bc: int = BC_TRANSMISSIVE) -> np.ndarray:
    """Ac: (nv, nc, ...) -> predicted children (nv, 2nc, ...)."""
    Ac = _f64(Ac)
    nv, nc = Ac.shape[0], Ac.shape[-1]
    Af = np.empty((nv,) + (2 * nc,) * dim)
    lib().orc_predict(dim, nv, nc, bc, _dp(Ac), _dp(Af))
    return Af


# ---------------------------------------------------------------- initial data

def init_quadrant(n: int, gamma: float, prim, lo=0.0, hi=1.0, x0=0.5, y0=0.5) -> np.ndarray:
    """prim: (4, 4) rows = quadrants I..IV, columns (rho, v1, v2, p)."""
    prim = _f64(prim).reshape(16)
    Q = np.empty((4, n, n))
    lib().orc_init_quadrant(n, lo, hi, gamma, x0, y0, _dp(prim), _dp(Q))
    return Q


def init_ellipsoid(n: int, gamma: float, a, b, c, theta, phi, states, lo=-1.0, hi=1.0,
                   rc=1.0) -> np.ndarray:
    """states = (rho_in, p_in, rho_out, p_out); cos/sin are taken here on the host."""
    e = _f64([a, b, c, np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi), rc, 0, 0, 0])
    st = _f64(states)
    Q = np.empty((5, n, n, n))
    lib().orc_init_ellipsoid(n, lo, hi, gamma, _dp(e), _dp(st), _dp(Q))
    return Q


def init_riemann1d(dim: int, n: int, gamma: float, axis: int, left, right, x0=0.5,
                   lo=0.0, hi=1.0) -> np.ndarray:
    """left/right = (rho, u, p) with u along ``axis``."""
    lr = _f64(list(left) + list(right))
    Q = np.empty((dim + 2,) + (n,) * dim)
    lib().orc_init_riemann1d(dim, n, lo, hi, gamma, axis, x0, _dp(lr), _dp(Q))
    return Q


# ---------------------------------------------------------------- hierarchy

class Hierarchy:
    """Dense per-level storage of a block-patch hierarchy (see oracle.c)."""

    def __init__(self, dim: int, levels: int, n0: int, bc: int = BC_TRANSMISSIVE,
                 gamma: float = 1.4, lo: float = 0.0, hi: float = 1.0, eps: float = 1e-3,
                 eta: float = 0.8, pmin: int = 8, pmax: int = 32, scheme: int = SCHEME_MR,
                 criterion: int = CRIT_MR, eps_p: float = 0.0, eps_levels: bool = False, rk: int = RK_MIDPOINT,
                 ausm_speed: int = AUSM_MEAN, tiler: int = TILER_BLOCKS, cfl_mode: int = CFL_SUM,
                 regrid_every: int = 1):
        self.dim, self.L, self.n0, self.bc = dim, levels, n0, bc
        self.gamma, self.lo, self.hi, self.eps, self.eta = gamma, lo, hi, eps, eta
        self.pmin, self.pmax = pmin, pmax
        self.nv = dim + 2
        self._h = lib().orc_h_new(dim, levels, n0, bc, gamma, lo, hi, eps, eta, pmin, pmax)
        if not self._h:
            raise ValueError("invalid hierarchy parameters")
        if lib().orc_h_set_scheme(self._h, scheme) != 0:
            raise ValueError("unknown finite-volume scheme")
        self.scheme = scheme
        if lib().orc_h_set_criterion(self._h, criterion, eps_p) != 0:
            raise ValueError("unknown refinement criterion")
        self.criterion, self.eps_p = criterion, eps_p
        lib().orc_h_set_eps_levels(self._h, int(eps_levels))
        self.eps_levels = bool(eps_levels)
        if lib().orc_h_set_variants(self._h, rk, ausm_speed) != 0:
            raise ValueError("unknown time stepping or AUSM+ sound speed")
        self.rk, self.ausm_speed = rk, ausm_speed
        if lib().orc_h_set_tiler(self._h, tiler) != 0:
            raise ValueError("unknown tiler, or pmax / pmin above 8 for Berger-Rigoutsos")
        self.tiler = tiler
        if lib().orc_h_set_cfl_mode(self._h, cfl_mode) != 0:
            raise ValueError("unknown CFL signal speed")
        self.cfl_mode = cfl_mode
        if regrid_every < 1:
            raise ValueError("regrid_every must be >= 1")
        # the hierarchy is rebuilt after step n (counted from initialisation,
        # level-0 steps with local time stepping) when n is a multiple of
        # regrid_every
        self.regrid_every = regrid_every
        self.nsteps = 0
        self.t = 0.0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_h_free(h)
            self._h = None

    def n(self, l: int) -> int:
        return lib().orc_h_n(self._h, l)

    def dx(self, l: int) -> float:
        return lib().orc_h_dx(self._h, l)

    def _view(self, ptr, shape, dtype):
        count = int(np.prod(shape))
        arr = np.ctypeslib.as_array(ptr, shape=(count,))
        return arr.view(dtype).reshape(shape) if arr.dtype != dtype else arr.reshape(shape)

    def level(self, l: int) -> np.ndarray:
        """Live view (nv, n, n[, n]) of level l, index [f, (z,) y, x]."""
        n = self.n(l)
        return self._view(lib().orc_h_level(self._h, l), (self.nv,) + (n,) * self.dim, np.float64)

    def level_stage(self, l: int) -> np.ndarray:
        n = self.n(l)
        return self._view(lib().orc_h_level_stage(self._h, l), (self.nv,) + (n,) * self.dim,
                          np.float64)

    def active(self, l: int) -> np.ndarray:
        n = self.n(l)
        return self._view(lib().orc_h_active(self._h, l), (n,) * self.dim, np.uint8).copy()

    def flags(self, l: int) -> np.ndarray:
        n = self.n(l)
        return self._view(lib().orc_h_flags(self._h, l), (n,) * self.dim, np.uint8).copy()

    def details(self, l: int) -> np.ndarray:
        n = self.n(l)
        return self._view(lib().orc_h_details(self._h, l), (n,) * self.dim, np.float64).copy()

    def leaf_mask(self, l: int) -> np.ndarray:
        act = self.active(l).astype(bool)
        if l + 1 < self.L:
            fine = self.active(l + 1).astype(bool)
            if self.dim == 2:
                cov = fine[0::2, 0::2]
            else:
                cov = fine[0::2, 0::2, 0::2]
            act &= ~cov
        return act

    # ---- set-up
    def set_active(self, l: int, mask: np.ndarray):
        """Impose the patch membership of level l >= 1 (test-only: a fixed
        hierarchy for runs without regrid).  Project and fill ghost cells
        afterwards (restrict_all, ghost)."""
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape == (self.n(l),) * self.dim
        lib().orc_h_set_active(self._h, l, m.ctypes.data_as(C.POINTER(C.c_uint8)))

    def init_finest(self, Q: np.ndarray):
        """Write finest-level data, restrict, analyse, flag, tile, fill ghosts."""
        self.level(self.L - 1)[...] = Q
        lib().orc_h_init(self._h)
        self.t = 0.0
        self.nsteps = 0

    # ---- operations
    def cfl(self, cfl: float, t_end: float = np.inf):
        smax = np.zeros(self.L)
        dt = lib().orc_h_cfl(self._h, cfl, self.t, t_end, _dp(smax))
        return dt, smax

    def _regrid_now(self, regrid):
        """regrid True / False as given; None: by the step count and
        regrid_every (this step is step nsteps + 1)."""
        return (self.nsteps + 1) % self.regrid_every == 0 if regrid is None else bool(regrid)

    def step(self, cfl: float, t_end: float = np.inf, regrid=True) -> float:
        """One step (regrid=None: regrid as regrid_every says)."""
        rg = self._regrid_now(regrid)
        taken = self.t < t_end
        dt = lib().orc_h_step(self._h, cfl, self.t, t_end, int(rg))
        self.t = self.t + dt
        self.nsteps += 1 if taken else 0
        return dt

    def step_lts(self, cfl: float, t_end: float = np.inf, regrid=True):
        """One level-0 step with local time steps; returns (dt_0, leaf updates)
        (regrid=None: regrid as regrid_every says)."""
        rg = self._regrid_now(regrid)
        taken = self.t < t_end
        upd = C.c_int64(0)
        dt = lib().orc_h_step_lts(self._h, cfl, self.t, t_end, int(rg), C.byref(upd))
        if dt == -2.0:
            raise ValueError("local time steps use the midpoint rule")
        if dt < 0:
            raise MemoryError("oracle: local time stepping buffers")
        self.t = self.t + dt
        self.nsteps += 1 if taken else 0
        return dt, upd.value

    def step_fixed(self, dt: float):
        lib().orc_h_step_fixed(self._h, dt)
        self.t = self.t + dt

    def stage(self, stage: int, dt: float):
        lib().orc_h_stage(self._h, stage, dt)

    def restrict_all(self):
        lib().orc_h_restrict(self._h)

    def ghost(self):
        lib().orc_h_ghost(self._h)

    def regrid(self):
        lib().orc_h_regrid(self._h)

    def set_eps(self, eps: float):
        """Replace the detail threshold for later analyses."""
        self.eps = eps
        lib().orc_h_set_eps(self._h, eps)

    def totals(self) -> np.ndarray:
        tot = np.zeros(self.nv)
        lib().orc_h_totals(self._h, _dp(tot))
        return tot

    def counts(self):
        leaves = np.zeros(self.L, dtype=np.int64)
        active = np.zeros(self.L, dtype=np.int64)
        lib().orc_h_counts(self._h, leaves.ctypes.data_as(C.POINTER(C.c_int64)),
                           active.ctypes.data_as(C.POINTER(C.c_int64)))
        return leaves, active

    def patches(self) -> np.ndarray:
        """Rows {level, ox, oy, oz, sx, sy, sz} (2D: oz = 0, sz = 1)."""
        npch = lib().orc_h_npatch(self._h)
        out = np.zeros((max(npch, 1), 7), dtype=np.int32)
        lib().orc_h_patches(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out[:npch]

    def composite(self) -> np.ndarray:
        """Project the adaptive solution up to the finest uniform grid by
        recursive prediction (error assessment, Sec. 3): leaves keep their
        values, refined regions are taken from finer levels."""
        U = self.level(0).copy()
        for l in range(1, self.L):
            P = predict(self.dim, U, self.bc)
            act = self.active(l).astype(bool)
            P[:, act] = self.level(l)[:, act]
            U = P
        return U
