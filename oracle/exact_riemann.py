"""Exact solution of the B = 0 (gas-dynamic) Riemann problem -- TEST
INFRASTRUCTURE ONLY, used to pin the oracle's normal-pair Riemann solver and
its 1D sweep in the hydrodynamic limit.

Written independently of the oracle from the textbook construction (Toro,
"Riemann Solvers and Numerical Methods for Fluid Dynamics", Ch. 4): the star
pressure is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, found here by
plain bisection (no Newton step, no shared formula with the two-shock
iteration), and the similarity solution is sampled wave by wave.
"""
from __future__ import annotations

import math


def _f_side(p, rho, pk, gamma):
    """Velocity change across one wave as a function of the star pressure."""
    a = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(rhoL, uL, pL, rhoR, uR, pR, gamma=5.0 / 3.0, iters=200):
    """Return (p*, u*) by bisection on the pressure function."""
    def F(p):
        return _f_side(p, rhoL, pL, gamma) + _f_side(p, rhoR, pR, gamma) + (uR - uL)

    lo, hi = 1e-14 * min(pL, pR), 10.0 * max(pL, pR)
    while F(hi) < 0.0:
        hi *= 10.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    u = 0.5 * (uL + uR) + 0.5 * (_f_side(p, rhoR, pR, gamma) - _f_side(p, rhoL, pL, gamma))
    return p, u


def sample(s, rhoL, uL, pL, rhoR, uR, pR, gamma=5.0 / 3.0):
    """Exact (rho, u, p) at similarity coordinate s = x / t."""
    ps, us = star_state(rhoL, uL, pL, rhoR, uR, pR, gamma)
    g = gamma
    if s <= us:  # left of contact
        aL = math.sqrt(g * pL / rhoL)
        if ps > pL:  # left shock
            rs = rhoL * ((ps / pL + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pL + 1))
            S = uL - aL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
            return (rhoL, uL, pL) if s <= S else (rs, us, ps)
        # left rarefaction
        rs = rhoL * (ps / pL) ** (1.0 / g)
        ast = aL * (ps / pL) ** ((g - 1) / (2 * g))
        head, tail = uL - aL, us - ast
        if s <= head:
            return rhoL, uL, pL
        if s >= tail:
            return rs, us, ps
        c = 2.0 / (g + 1) + (g - 1) / ((g + 1) * aL) * (uL - s)
        rho = rhoL * c ** (2.0 / (g - 1))
        u = 2.0 / (g + 1) * (aL + (g - 1) / 2.0 * uL + s)
        p = pL * c ** (2.0 * g / (g - 1))
        return rho, u, p
    aR = math.sqrt(g * pR / rhoR)
    if ps > pR:  # right shock
        rs = rhoR * ((ps / pR + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pR + 1))
        S = uR + aR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
        return (rhoR, uR, pR) if s >= S else (rs, us, ps)
    rs = rhoR * (ps / pR) ** (1.0 / g)
    ast = aR * (ps / pR) ** ((g - 1) / (2 * g))
    head, tail = uR + aR, us + ast
    if s >= head:
        return rhoR, uR, pR
    if s <= tail:
        return rs, us, ps
    c = 2.0 / (g + 1) - (g - 1) / ((g + 1) * aR) * (uR - s)
    rho = rhoR * c ** (2.0 / (g - 1))
    u = 2.0 / (g + 1) * (-aR + (g - 1) / 2.0 * uR + s)
    p = pR * c ** (2.0 * g / (g - 1))
    return rho, u, p
