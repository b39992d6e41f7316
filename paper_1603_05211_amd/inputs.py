"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module only draws numbers; it holds none of the method's arithmetic.
Every draw uses ``numpy.random.default_rng(seed)`` (PCG64) in a fixed order, so
the oracle and the GPU library consume identical doubles.

Workloads stand in for the paper's two test problems (the Lax-Liu #6
four-quadrant Riemann problem of Sec. 4.1 and the ellipsoidal shock of
Sec. 4.2): same geometry and structure, seeded states.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


def quadrant_states(seed: int) -> np.ndarray:
    """(4, 4) primitive states, rows = quadrants I, II, III, IV, columns
    (rho, v1, v2, p); rho ~ U[0.5, 2], v1, v2 ~ U[-1, 1], p ~ U[0.2, 2]."""
    rng = np.random.default_rng(seed)
    out = np.empty((4, 4))
    for q in range(4):
        out[q, 0] = rng.uniform(0.5, 2.0)
        out[q, 1] = rng.uniform(-1.0, 1.0)
        out[q, 2] = rng.uniform(-1.0, 1.0)
        out[q, 3] = rng.uniform(0.2, 2.0)
    return out


def lax_liu_6() -> np.ndarray:
    """The paper's Table 1 (Lax-Liu configuration #6): rows I..IV, columns
    (rho, v1, v2, p)."""
    return np.array([[1.0, 0.75, -0.5, 1.0],
                     [2.0, 0.75, 0.5, 1.0],
                     [1.0, -0.75, 0.5, 1.0],
                     [3.0, -0.75, -0.5, 1.0]])


@dataclass
class Ellipsoid:
    a: float
    b: float
    c: float
    theta: float = math.pi / 3.0
    phi: float = math.pi / 4.0
    rc: float = 1.0
    states: tuple = (1.0, 10.0, 0.125, 0.1)   # rho_in, p_in, rho_out, p_out


def ellipsoid(seed: int) -> Ellipsoid:
    """Semi-axes a, b, c ~ U[0.2, 0.4] (drawn in that order); the paper's
    rotation angles theta = pi/3, phi = pi/4; inside rho = 1, p = 10, outside
    rho = 0.125, p = 0.1, zero velocity; centre at the origin."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.2, 0.4)
    b = rng.uniform(0.2, 0.4)
    c = rng.uniform(0.2, 0.4)
    return Ellipsoid(a, b, c)


def paper_ellipsoid() -> Ellipsoid:
    """Sec. 4.2 as printed: r_c = 3/5, a = 1/3, b = 1, c = 3, theta = pi/3,
    phi = pi/4, rho = 0.125 / rho e = 0.25 inside, rho = 1 / rho e = 2.5
    outside (p = (gamma - 1) rho e)."""
    return Ellipsoid(1.0 / 3.0, 1.0, 3.0, math.pi / 3.0, math.pi / 4.0, 0.6,
                     (0.125, 0.4 * 0.25, 1.0, 0.4 * 2.5))


def riemann_1d(seed: int):
    """Seeded 1D Riemann data (rho, u, p) left and right."""
    rng = np.random.default_rng(seed)
    left = (rng.uniform(0.5, 2.0), rng.uniform(-1.0, 1.0), rng.uniform(0.2, 2.0))
    right = (rng.uniform(0.5, 2.0), rng.uniform(-1.0, 1.0), rng.uniform(0.2, 2.0))
    return left, right


@dataclass
class Batch:
    sides: np.ndarray            # (n,) int, multiples of 32 in [32, 512]
    states: np.ndarray           # (n, 4, 4) quadrant states


def batch(seed: int, n_instances: int = 512, side_step: int = 32, side_max_mult: int = 16) -> Batch:
    """Per instance in order: side = 32 * integers(1, 17), then its 16
    quadrant state draws (as quadrant_states)."""
    rng = np.random.default_rng(seed)
    sides = np.empty(n_instances, dtype=np.int64)
    states = np.empty((n_instances, 4, 4))
    for i in range(n_instances):
        sides[i] = side_step * int(rng.integers(1, side_max_mult + 1))
        for q in range(4):
            states[i, q, 0] = rng.uniform(0.5, 2.0)
            states[i, q, 1] = rng.uniform(-1.0, 1.0)
            states[i, q, 2] = rng.uniform(-1.0, 1.0)
            states[i, q, 3] = rng.uniform(0.2, 2.0)
    return Batch(sides, states)


@dataclass
class Workload:
    """A named configuration of the method (sizes from the paper's workloads)."""
    name: str
    dim: int
    levels: int
    n0: int
    lo: float
    hi: float
    cfl: float
    eps: float = 1e-3
    eta: float = 0.8
    pmin: int = 8
    pmax: int = 32
    steps: int = 0               # fixed step count (0: run to t_end)
    t_end: float = math.inf
    lts: bool = False
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # 2D uniform 128^2, FP64, 100 steps at CFL 0.45
    "quad2d_uniform128": Workload("quad2d_uniform128", 2, 1, 128, 0.0, 1.0, 0.45, steps=100),
    # 2D adaptive, 5 levels 32^2 .. 512^2, eps 1e-3 on density, global dt, t = 0.25
    "quad2d_adaptive5": Workload("quad2d_adaptive5", 2, 5, 32, 0.0, 1.0, 0.45, t_end=0.25),
    # 3D uniform 256^3 ellipsoid on [-1,1]^3, 200 steps at CFL 0.4
    "ellip3d_uniform256": Workload("ellip3d_uniform256", 3, 1, 256, -1.0, 1.0, 0.4, steps=200),
    # 512 independent 2D instances, sides 32..512, 100 steps each
    "quad2d_batch512": Workload("quad2d_batch512", 2, 1, 0, 0.0, 1.0, 0.45, steps=100),
    # 3D adaptive, 4 levels 32^3 .. 256^3, local time stepping, t = 0.2
    "ellip3d_adaptive4_lts": Workload("ellip3d_adaptive4_lts", 3, 4, 32, -1.0, 1.0, 0.4,
                                      t_end=0.2, lts=True),
}
