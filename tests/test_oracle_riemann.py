"""Pins of the oracle's interface Riemann solvers.

Normal pair: Colella & Woodward (1984) Section 2 two-shock Newton iteration on
the total transverse pressure.  In the B = 0 limit with two shocks it must
reach the exact gas-dynamic star state (checked against an independent
bisection on the textbook pressure function); with identical states it must
return them bitwise after zero iterations; symmetric collisions give u* = 0;
small jumps give the linear acoustic solution.
Transverse pair: closed-form linear Alfven problem, checked against a
numerical eigen-decomposition of the linear system.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import exact_riemann as X

G = 5.0 / 3.0


def _hydro(rhoL, uL, pL, rhoR, uR, pR, tol=1e-12):
    CL = math.sqrt(G * pL * rhoL)
    CR = math.sqrt(G * pR * rhoR)
    return O.riemann_normal(pL, pR, 0.0, uL, uR, CL, CR, G, G, tol=tol, max_iter=50)


@pytest.mark.parametrize("state", [
    (1.0, 0.3, 1.0, 1.0, 0.3, 1.0),
    (2.5, -1.7, 0.04, 2.5, -1.7, 0.04),
    (1e-3, 40.0, 7e5, 1e-3, 40.0, 7e5),
])
def test_identical_states_exact_and_zero_iterations(state):
    P, u, it, conv = _hydro(*state)
    assert it == 0 and conv
    assert P == state[2] and u == state[1]


@pytest.mark.parametrize("state", [
    (1.0, 1.0, 1.0, 1.0, -1.0, 1.0),          # colliding streams
    (1.0, 2.0, 1.0, 0.5, 0.0, 0.3),           # moving piston
    (5.0, 0.0, 8.7, 20.0, -18.0, 8.7),        # solar wind into plasma at rest
    (0.125, 3.0, 0.1, 1.0, 0.0, 1.0),
])
def test_two_shock_problems_match_exact_solution(state):
    ps_ex, us_ex = X.star_state(*state, gamma=G)
    # both waves must indeed be shocks for the two-shock form to be exact
    assert ps_ex > state[2] and ps_ex > state[5]
    P, u, it, conv = _hydro(*state)
    assert conv
    assert abs(P - ps_ex) <= 1e-10 * ps_ex
    assert abs(u - us_ex) <= 1e-10 * (abs(us_ex) + math.sqrt(G * ps_ex))


def test_symmetric_collision_has_zero_star_velocity():
    P, u, it, conv = _hydro(1.3, 2.2, 0.7, 1.3, -2.2, 0.7)
    assert conv and abs(u) <= 1e-15
    ps_ex, _ = X.star_state(1.3, 2.2, 0.7, 1.3, -2.2, 0.7, gamma=G)
    assert abs(P - ps_ex) <= 1e-10 * ps_ex


def test_rarefaction_error_is_small_and_reported():
    # two-shock form is approximate for rarefactions: the error is second
    # order in the jump (documented reading); weak rarefactions -> tiny error
    for eps, bound in ((0.01, 1e-6), (0.1, 1e-3)):
        st = (1.0, -eps, 1.0, 1.0, eps, 1.0)
        ps_ex, us_ex = X.star_state(*st, gamma=G)
        P, u, it, conv = _hydro(*st)
        assert conv
        assert abs(P - ps_ex) / ps_ex < bound


def test_small_jumps_follow_linear_acoustics():
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho, p = rng.uniform(0.5, 2), rng.uniform(0.5, 2)
        eps = 1e-6
        dp, du = eps * rng.normal(), eps * rng.normal()
        pL, pR = p, p + dp
        uL, uR = 0.1, 0.1 + du
        C = math.sqrt(G * p * rho)
        P, u, it, conv = _hydro(rho, uL, pL, rho, uR, pR)
        P_lin = 0.5 * (pL + pR) + 0.5 * C * (uL - uR)
        u_lin = 0.5 * (uL + uR) + 0.5 * (pL - pR) / C
        assert abs(P - P_lin) < 1e-11
        assert abs(u - u_lin) < 1e-11


def test_newton_nonconvergence_is_reported():
    P, u, it, conv = O.riemann_normal(1.0, 1e4, 0.0, 50.0, -50.0, math.sqrt(G), math.sqrt(G * 1e4),
                                      G, G, tol=1e-14, max_iter=1)
    assert not conv and it == 1


def test_dipole_offset_only_shifts_pressure():
    # the common dipole pressure Pd enters only the absolute level: jumps
    # are unchanged, so the star state relative to it is that of a problem
    # with pressures P = Pt + Pd and gamma_e adjusted accordingly
    rhoL, uL, pL, rhoR, uR, pR = 1.0, 1.0, 2.0, 1.0, -1.0, 2.0
    Pd = 3.0
    CL = math.sqrt(rhoL * (G * pL + 2 * Pd))
    CR = math.sqrt(rhoR * (G * pR + 2 * Pd))
    gL = CL * CL / (rhoL * (pL + Pd))
    gR = CR * CR / (rhoR * (pR + Pd))
    P1, u1, _, _ = O.riemann_normal(pL, pR, Pd, uL, uR, CL, CR, gL, gR)
    P2, u2, _, _ = O.riemann_normal(pL + Pd, pR + Pd, 0.0, uL, uR, CL, CR, gL, gR)
    assert abs((P1 + Pd) - P2) < 1e-12 * P2 and abs(u1 - u2) < 1e-12


@pytest.mark.parametrize("sigma", [1.0, -1.0])
def test_alfven_pair_matches_linear_eigen_solution(sigma):
    rng = np.random.default_rng(9)
    for _ in range(10):
        rho = rng.uniform(0.3, 3.0)
        Bn = sigma * rng.uniform(0.2, 2.0)
        vL, vR, bL, bR = rng.normal(size=4)
        # linear Lagrangian system d/dt (v, B) + A d/dm (v, B) = 0
        A = np.array([[0.0, -Bn], [-rho * Bn, 0.0]])
        lam, R = np.linalg.eig(A)
        Linv = np.linalg.inv(R)
        wL = Linv @ np.array([vL, bL])
        wR = Linv @ np.array([vR, bR])
        # the star state takes right-moving components from L, left-moving from R
        w = np.where(lam > 0, wL, wR)
        v_ex, b_ex = R @ w
        r = math.sqrt(rho)
        v, b = O.riemann_alfven(r, r, math.copysign(1.0, Bn), vL, vR, bL, bR)
        assert abs(v - v_ex) < 1e-12 and abs(b - b_ex) < 1e-12


def test_alfven_pair_identical_states_bitwise():
    v, b = O.riemann_alfven(1.7, 1.7, 1.0, 0.3, 0.3, -2.1, -2.1)
    assert v == 0.3 and b == -2.1
