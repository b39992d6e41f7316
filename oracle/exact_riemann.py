"""Exact solution of the 1D Riemann problem of the ideal-gas Euler equations.

TEST INFRASTRUCTURE ONLY (used to pin the oracle's finite-volume scheme).

Standard construction from the Rankine-Hugoniot conditions and the isentropic
rarefaction relations: the star pressure p* solves f_L(p) + f_R(p) + (u_R -
u_L) = 0 with the wave functions

  f_K(p) = (p - p_K) sqrt(A_K / (p + B_K))          p >  p_K  (shock)
  f_K(p) = 2 c_K / (g - 1) ((p / p_K)^((g-1)/(2g)) - 1)   p <= p_K  (rarefaction)

A_K = 2 / ((g+1) rho_K), B_K = (g-1)/(g+1) p_K; solved by safeguarded Newton
iteration.  u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.  The self-similar
solution is then sampled at x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rK, pK, g):
    cK = math.sqrt(g * pK / rK)
    if p > pK:
        A = 2.0 / ((g + 1.0) * rK)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        f = (p - pK) * s
        df = s * (1.0 - 0.5 * (p - pK) / (p + B))
    else:
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * cK / (g - 1.0) * ((p / pK) ** e - 1.0)
        df = 1.0 / (rK * cK) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g=1.4, tol=1e-14):
    """left/right = (rho, u, p).  Returns (p*, u*)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    if 2.0 * (cL + cR) / (g - 1.0) <= uR - uL:
        raise ValueError("vacuum is generated")
    # two-rarefaction guess
    e = (g - 1.0) / (2.0 * g)
    p = ((cL + cR - 0.5 * (g - 1.0) * (uR - uL)) /
         (cL / pL ** e + cR / pR ** e)) ** (1.0 / e)
    p = max(p, 1e-12)
    for _ in range(200):
        fL, dL = _fK(p, rL, pL, g)
        fR, dR = _fK(p, rR, pR, g)
        fn = fL + fR + (uR - uL)
        pn = p - fn / (dL + dR)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, g)
    fR, _ = _fK(p, rR, pR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rL, uL, pL = left
    rR, uR, pR = right
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for side in ("L", "R"):
        if side == "L":
            rK, uK, pK, sgn = rL, uL, pL, -1.0
            m = xi <= us
        else:
            rK, uK, pK, sgn = rR, uR, pR, 1.0
            m = xi > us
        cK = math.sqrt(g * pK / rK)
        x = xi[m]
        rr = np.empty_like(x)
        uu = np.empty_like(x)
        pp = np.empty_like(x)
        if ps > pK:  # shock
            rs = rK * ((ps / pK + gm) / (gm * ps / pK + 1.0))
            S = uK + sgn * cK * math.sqrt((g + 1.0) / (2.0 * g) * ps / pK + (g - 1.0) / (2.0 * g))
            outside = (x < S) if sgn < 0 else (x > S)
            rr[:] = np.where(outside, rK, rs)
            uu[:] = np.where(outside, uK, us)
            pp[:] = np.where(outside, pK, ps)
        else:  # rarefaction
            rs = rK * (ps / pK) ** (1.0 / g)
            cs = cK * (ps / pK) ** ((g - 1.0) / (2.0 * g))
            head = uK + sgn * cK
            tail = us + sgn * cs
            if sgn < 0:
                outside = x < head
                star = x > tail
            else:
                outside = x > head
                star = x < tail
            fan = ~outside & ~star
            # inside the fan
            uf = 2.0 / (g + 1.0) * (-sgn * cK + (g - 1.0) / 2.0 * uK + x)
            cf = 2.0 / (g + 1.0) * (cK - sgn * (g - 1.0) / 2.0 * (uK - x))
            cf = np.maximum(cf, 0.0)
            rf = rK * (cf / cK) ** (2.0 / (g - 1.0))
            pf = pK * (cf / cK) ** (2.0 * g / (g - 1.0))
            rr[:] = np.where(outside, rK, np.where(star, rs, rf))
            uu[:] = np.where(outside, uK, np.where(star, us, uf))
            pp[:] = np.where(outside, pK, np.where(star, ps, pf))
        rho[m], u[m], p[m] = rr, uu, pp
    return rho, u, p


def cell_averages(left, right, n, t, x0=0.5, lo=0.0, hi=1.0, g=1.4, sub=64):
    """Cell averages of (rho, rho u, E) on n uniform cells by a midpoint rule
    with ``sub`` points per cell (exact where the solution is constant)."""
    dx = (hi - lo) / n
    xs = lo + (np.arange(n * sub) + 0.5) * (dx / sub)
    rho, u, p = sample(left, right, (xs - x0) / t, g)
    E = p / (g - 1.0) + 0.5 * rho * u * u
    avg = lambda a: a.reshape(n, sub).mean(axis=1)
    return avg(rho), avg(rho * u), avg(E)
