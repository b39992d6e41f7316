"""MI355X-native adaptive finite-volume solver for the compressible Euler
equations (MUSCL / van Albada / AUSM+ / midpoint RK2 on a block-patch
hierarchy refined by multiresolution details), after arXiv:1603.05211.

Every step runs in the gfx950 HIP kernels of ``libeu.so`` behind the C-ABI of
``include/eu.h``; this module only marshals arguments and owns the device
buffers (torch tensors).  The same entry-point names as the C-ABI are exposed
as methods of :class:`Solver`.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _abi
from ._abi import (EU_BC_PERIODIC, EU_BC_TRANSMISSIVE, EU_DT_GLOBAL, EU_DT_LTS, EU_FP32, EU_FP64,
                   EU_CRIT_GRADIENT, EU_CRIT_MR, EU_GHOST, EU_SCHEME_AMR, EU_SCHEME_MR, EU_STAGE_SCHEDULES, EU_STRIP_SCHEDULE0, EU_IC_ELLIPSOID, EU_IC_QUADRANT, EU_IC_RIEMANN1D, EU_IC_UNIFORM,
                   EU_PROLONG, EU_RESTRICT, EU_RK_MIDPOINT, EU_RK_HEUN, EU_AUSM_MEAN, EU_AUSM_CRITICAL,
                   EU_TILER_BLOCKS, EU_TILER_BR, EU_CFL_SUM, EU_CFL_MAX)

__all__ = ["Solver", "EuError", "EU_FP32", "EU_FP64", "EU_BC_PERIODIC", "EU_BC_TRANSMISSIVE",
           "EU_RESTRICT", "EU_PROLONG", "EU_GHOST", "EU_DT_GLOBAL", "EU_DT_LTS", "EU_STAGE_SCHEDULES",
           "EU_STRIP_SCHEDULE0", "EU_SCHEME_MR", "EU_SCHEME_AMR", "EU_CRIT_MR", "EU_CRIT_GRADIENT",
           "EU_RK_MIDPOINT", "EU_RK_HEUN", "EU_AUSM_MEAN", "EU_AUSM_CRITICAL",
           "EU_TILER_BLOCKS", "EU_TILER_BR", "EU_CFL_SUM", "EU_CFL_MAX"]


class EuError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_abi.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Solver:
    """One context of the C library on caller-owned (torch) device buffers.

    mode: a single hierarchy (levels >= 1; levels = 1 is a uniform grid) or a
    batch of independent uniform grids (``sides`` given).
    """

    def __init__(self, dim: int, n0: int = 128, levels: int = 1, precision: int = EU_FP64,
                 bc: int = EU_BC_TRANSMISSIVE, cfl: float = 0.45, t_end: float = math.inf,
                 eps: float = 1e-3, eta: float = 0.8, patch_min: int = 8, patch_max: int = 32,
                 lo: float = 0.0, hi: float = 1.0, gamma: float = 1.4, sides=None,
                 time_mode: int = EU_DT_GLOBAL, device: str = "cuda:0", stream=None,
                 scheme: int = EU_SCHEME_MR, criterion: int = EU_CRIT_MR, eps_p: float = 0.0,
                 eps_levels: int = 0, rk: int = EU_RK_MIDPOINT, ausm_speed: int = EU_AUSM_MEAN,
                 tiler: int = EU_TILER_BLOCKS, cfl_mode: int = EU_CFL_SUM, regrid_every: int = 1):
        import torch
        self._lib = _abi.load()
        self.torch = torch
        self.dim, self.levels, self.n0, self.precision = dim, levels, n0, precision
        self.nv = dim + 2
        self.lo, self.hi, self.gamma = lo, hi, gamma
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._sides = None
        cfg = _abi.EuConfig()
        cfg.dim, cfg.precision, cfg.gamma, cfg.lo, cfg.hi = dim, precision, gamma, lo, hi
        cfg.n0, cfg.levels, cfg.bc, cfg.cfl, cfg.t_end = n0, levels, bc, cfl, t_end
        cfg.eps, cfg.eta, cfg.patch_min, cfg.patch_max = eps, eta, patch_min, patch_max
        cfg.time_mode = time_mode
        cfg.scheme = scheme
        self.scheme = scheme
        cfg.criterion, cfg.eps_p = criterion, eps_p
        self.criterion, self.eps_p = criterion, eps_p
        cfg.eps_levels = eps_levels
        cfg.rk, cfg.ausm_speed, cfg.tiler = rk, ausm_speed, tiler
        cfg.cfl_mode, cfg.regrid_every = cfl_mode, regrid_every
        if sides is not None:
            self._sides = (C.c_int32 * len(sides))(*[int(s) for s in sides])
            cfg.n_instances = len(sides)
            cfg.inst_side_host = C.cast(self._sides, C.POINTER(C.c_int32))
            self.n_instances = len(sides)
        else:
            cfg.n_instances = 1
            self.n_instances = 1
        cfg.stream = C.c_void_p(self.stream.cuda_stream)
        self._cfg = cfg
        sb, kb = C.c_size_t(0), C.c_size_t(0)
        self._check(self._lib.eu_query_sizes(C.byref(cfg), C.byref(sb), C.byref(kb)), "eu_query_sizes")
        self.state_bytes, self.scratch_bytes = sb.value, kb.value
        self.state = torch.empty(max(sb.value, 256), dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(max(kb.value, 256), dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p()
        self._check(self._lib.eu_create(C.byref(cfg), C.c_void_p(self.state.data_ptr()), sb.value,
                                        C.c_void_p(self.scratch.data_ptr()), kb.value, C.byref(ctx)),
                    "eu_create")
        self._ctx = ctx
        self.sides = list(sides) if sides is not None else [n0 << l for l in range(levels)]

    # ------------------------------------------------------------------ plumbing
    def _check(self, code: int, what: str):
        if code != _abi.EU_OK:
            msg = ""
            if getattr(self, "_ctx", None):
                raw = self._lib.eu_last_error(self._ctx)
                msg = raw.decode() if raw else ""
            raise EuError(code, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.eu_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n(self, level: int) -> int:
        return self.sides[level] if self.n_instances > 1 else self.n0 << level

    # ------------------------------------------------------------------ set-up
    def init_state(self, kind: int, **kw):
        p = _abi.EuProblem()
        p.kind = kind
        q = np.asarray(kw.get("quad", np.zeros((4, 4))), dtype=np.float64).reshape(4, 4)
        for i in range(4):
            for j in range(4):
                p.quad[i][j] = q[i, j]
        p.x0, p.y0 = kw.get("x0", 0.5), kw.get("y0", 0.5)
        for i, v in enumerate(kw.get("ell", [1, 1, 1, 1, 0, 1, 0, 1])):
            p.ell[i] = v
        for i, v in enumerate(kw.get("ell_states", [1, 1, 1, 1])):
            p.ell_states[i] = v
        for i, v in enumerate(kw.get("lr", [1, 0, 1, 1, 0, 1])):
            p.lr[i] = v
        p.axis = kw.get("axis", 0)
        p.split = kw.get("split", 0.5)
        for i, v in enumerate(kw.get("uniform", [1, 0, 0, 0, 1])):
            p.uniform[i] = v
        keep = None
        if "inst_quad" in kw:
            keep = np.ascontiguousarray(np.asarray(kw["inst_quad"], dtype=np.float64).reshape(-1))
            p.inst_quad_host = _dp(keep)
        self._check(self._lib.eu_init_state(self._ctx, C.byref(p)), "eu_init_state")

    def init_quadrant(self, prim, x0=0.5, y0=0.5):
        self.init_state(EU_IC_QUADRANT, quad=prim, x0=x0, y0=y0)

    def init_quadrant_batch(self, states):
        self.init_state(EU_IC_QUADRANT, inst_quad=states)

    def init_ellipsoid(self, a, b, c, theta, phi, states, rc=1.0):
        self.init_state(EU_IC_ELLIPSOID,
                        ell=[a, b, c, math.cos(theta), math.sin(theta), math.cos(phi), math.sin(phi), rc],
                        ell_states=states)

    def init_riemann1d(self, axis, left, right, split=0.5):
        self.init_state(EU_IC_RIEMANN1D, axis=axis, lr=list(left) + list(right), split=split)

    def init_uniform(self, prim):
        self.init_state(EU_IC_UNIFORM, uniform=list(prim))

    def set_finest(self, Q: np.ndarray, inst: int = 0):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        self._check(self._lib.eu_set_finest(self._ctx, inst, _dp(Q)), "eu_set_finest")

    # ------------------------------------------------------------------ the method
    def mr_decompose(self):
        self._check(self._lib.eu_mr_decompose(self._ctx), "eu_mr_decompose")

    def mr_flag(self, eps: float = -1.0):
        """Threshold, closure, tiling and new cells (eu_mr_flag); eps >= 0
        replaces the threshold.  Returns the flagged cells per level."""
        out = np.zeros(self.levels, dtype=np.int64)
        self._check(self._lib.eu_mr_flag(self._ctx, float(eps), out.ctypes.data_as(C.POINTER(C.c_int64))),
                    "eu_mr_flag")
        return out

    def project(self, mode: int):
        self._check(self._lib.eu_project(self._ctx, mode), "eu_project")

    def cfl_dt(self, host: bool = True, cfl: float = -1.0, t_remaining: float = -1.0, dt_out=None):
        """eu_cfl_dt: cfl > 0 replaces the configured CFL number, t_remaining
        >= 0 clips the step; dt_out (a float64 CUDA tensor, optional)
        receives the step's dt on the device.  Returns dt (instance 0) when
        host is set."""
        dev = None
        if dt_out is not None:
            assert dt_out.dtype == self.torch.float64 and dt_out.is_cuda and dt_out.numel() >= self.n_instances
            dev = C.c_void_p(dt_out.data_ptr())
        if not host:
            self._check(self._lib.eu_cfl_dt(self._ctx, float(cfl), float(t_remaining), dev, None), "eu_cfl_dt")
            return None
        dt = C.c_double(0.0)
        self._check(self._lib.eu_cfl_dt(self._ctx, float(cfl), float(t_remaining), dev, C.byref(dt)),
                    "eu_cfl_dt")
        return dt.value

    def fv_step(self, dt=None, level: int = -1):
        """eu_fv_step: dt (a float64 CUDA tensor, optional) replaces the dt of
        the last cfl_dt; level -1 = every level (>= 0: local time stepping
        from that level)."""
        dev = None
        if dt is not None:
            assert dt.dtype == self.torch.float64 and dt.is_cuda and dt.numel() >= self.n_instances
            dev = C.c_void_p(dt.data_ptr())
        self._check(self._lib.eu_fv_step(self._ctx, dev, int(level)), "eu_fv_step")

    def step(self, regrid: bool = True):
        self._check(self._lib.eu_step(self._ctx, int(regrid)), "eu_step")

    def advance(self, nsteps: int, use_graph: bool = True) -> int:
        done = C.c_int(0)
        self._check(self._lib.eu_advance(self._ctx, nsteps, int(use_graph), C.byref(done)), "eu_advance")
        return done.value

    def conserved_totals(self, out_dev=None, host: bool = True):
        """eu_conserved_totals: out_dev (a float64 CUDA tensor of n_instances
        x nv, optional) receives the totals on the device without a
        synchronisation; with host set they are also returned."""
        dev = None
        if out_dev is not None:
            assert out_dev.dtype == self.torch.float64 and out_dev.is_cuda
            assert out_dev.numel() >= self.n_instances * self.nv
            dev = C.c_void_p(out_dev.data_ptr())
        if not host:
            self._check(self._lib.eu_conserved_totals(self._ctx, dev, None), "eu_conserved_totals")
            return None
        out = np.zeros(self.n_instances * self.nv)
        self._check(self._lib.eu_conserved_totals(self._ctx, dev, _dp(out)), "eu_conserved_totals")
        return out.reshape(self.n_instances, self.nv) if self.n_instances > 1 else out

    def conserved_totals_static(self, out_dev):
        """eu_conserved_totals_static: the totals into out_dev (a float64
        CUDA tensor of n_instances x nv) on the stream, with the library's
        static device scratch instead of the context's (no allocation)."""
        assert out_dev.dtype == self.torch.float64 and out_dev.is_cuda
        assert out_dev.numel() >= self.n_instances * self.nv
        self._check(self._lib.eu_conserved_totals_static(self._ctx, C.c_void_p(out_dev.data_ptr())),
                    "eu_conserved_totals_static")

    # ------------------------------------------------------------------ read-back
    def level(self, level: int = 0, which: int = 0, inst: int = 0) -> np.ndarray:
        n = self.n(inst if self.n_instances > 1 else level)
        out = np.empty((self.nv,) + (n,) * self.dim)
        self._check(self._lib.eu_copy_level(self._ctx, inst, level, which, _dp(out)), "eu_copy_level")
        return out

    def composite(self) -> np.ndarray:
        """The adaptive solution projected onto the finest uniform grid
        (eu_copy_uniform); overwrites the stage array."""
        n = self.n(self.levels - 1)
        out = np.empty((self.nv,) + (n,) * self.dim)
        self._check(self._lib.eu_copy_uniform(self._ctx, _dp(out)), "eu_copy_uniform")
        return out

    def active(self, level: int) -> np.ndarray:
        n = self.n(level)
        out = np.empty((n,) * self.dim, dtype=np.uint8)
        self._check(self._lib.eu_get_active(self._ctx, level, out.ctypes.data_as(C.POINTER(C.c_uint8))),
                    "eu_get_active")
        return out

    def flags(self, level: int) -> np.ndarray:
        n = self.n(level)
        out = np.empty((n,) * self.dim, dtype=np.uint8)
        self._check(self._lib.eu_get_flags(self._ctx, level, out.ctypes.data_as(C.POINTER(C.c_uint8))),
                    "eu_get_flags")
        return out

    def details(self, level: int) -> np.ndarray:
        n = self.n(level)
        out = np.empty((n,) * self.dim)
        self._check(self._lib.eu_get_details(self._ctx, level, _dp(out)), "eu_get_details")
        return out

    def patches(self) -> np.ndarray:
        npch = C.c_int(0)
        self._check(self._lib.eu_patch_table(self._ctx, None, 0, C.byref(npch)), "eu_patch_table")
        out = np.zeros((max(npch.value, 1), 7), dtype=np.int32)
        self._check(self._lib.eu_patch_table(self._ctx, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                             npch.value, C.byref(npch)), "eu_patch_table")
        return out[:npch.value]

    def counters(self):
        leaves = np.zeros(self.levels, dtype=np.int64)
        active = np.zeros(self.levels, dtype=np.int64)
        self._check(self._lib.eu_counters(self._ctx, leaves.ctypes.data_as(C.POINTER(C.c_int64)),
                                          active.ctypes.data_as(C.POINTER(C.c_int64))), "eu_counters")
        return leaves, active

    def leaf_updates(self):
        u, st = C.c_int64(0), C.c_int(0)
        self._check(self._lib.eu_leaf_updates(self._ctx, C.byref(u), C.byref(st)), "eu_leaf_updates")
        return u.value, st.value

    def time(self):
        t, dt = C.c_double(0.0), C.c_double(0.0)
        self._check(self._lib.eu_time(self._ctx, C.byref(t), C.byref(dt)), "eu_time")
        return t.value, dt.value

    def profile(self, enable: bool):
        self._check(self._lib.eu_profile(self._ctx, int(enable)), "eu_profile")

    def kernel_time(self):
        ms, n = C.c_double(0.0), C.c_int64(0)
        self._check(self._lib.eu_kernel_time(self._ctx, C.byref(ms), C.byref(n)), "eu_kernel_time")
        return ms.value, n.value

    def autotune(self, reps: int = 20):
        """Time every finite-volume schedule that applies on the current state
        and keep the fastest; returns (variant, per-variant ms per pass, inf
        where a schedule does not apply)."""
        var = C.c_int(0)
        ms = (C.c_float * EU_STAGE_SCHEDULES)()
        self._check(self._lib.eu_autotune(self._ctx, reps, C.byref(var), ms), "eu_autotune")
        return var.value, list(ms)

    def stage_time(self, reps: int = 10):
        """Mean duration of one pass of the finite-volume update on the
        current state (reps passes replayed from one HIP graph between two HIP
        events); returns (ms, cell-stages per pass, launches per pass)."""
        ms, cells, nl = C.c_float(0.0), C.c_int64(0), C.c_int(0)
        self._check(self._lib.eu_stage_time(self._ctx, reps, C.byref(ms), C.byref(cells), C.byref(nl)),
                    "eu_stage_time")
        return ms.value, cells.value, nl.value

    def set_variant(self, variant: int):
        self._check(self._lib.eu_set_variant(self._ctx, variant), "eu_set_variant")

    def status(self):
        return self._lib.eu_status(self._ctx)

    def clear_status(self):
        self._check(self._lib.eu_clear_status(self._ctx), "eu_clear_status")
