"""The characteristic mode of the oracle (tracing of the seven waves of
Lagrangian 1D MHD and the linearised seven-wave Riemann problem), pinned
against what the mathematics fixes:
- its eigen-structure against a numerical eigen-decomposition of the
  Lagrangian Jacobian written from the equations (rho times the primitive
  ideal-MHD matrix), at generic and degenerate states (no transverse field,
  no normal field, c_f = c_s, the sonic point a = c_A);
- the traced face states of a zone whose parabolas hold a single wave: a
  wave that reaches the face carries the average of its own profile over its
  own domain of dependence, the others the average over the fast wave's
  (the reference state);
- the face state of the linearised Riemann problem between two states that
  differ by a few small waves: the left state plus the waves of negative
  speed, eigenvectors from the numerical decomposition;
- second-order convergence of fast, Alfven and slow eigenmodes, along an
  axis and oblique, beside the two-family mode's error on the same runs;
- the Sod shock tube (B = 0) converging to the exact solution;
- uniform states kept bitwise and mass, momentum and energy conserved on a
  periodic box;
- the split multi-D terms (B_n varying along the pencil) on a pencil whose
  primitive variables are uniform: the thermal pressure and density of both
  face states stay exactly the zone values (the Lagrangian equations of rho
  and p have no term in dB_n/dm), while the transverse field and velocity
  take the time-centring terms, so the magnetic-pressure change reaches the
  total pressure through the field alone;
- the inflow/dipole set-up (strong background field near the inner
  boundary) kept finite with positive density and pressure;
- a normal field at rounding level (a background field cancelled by the
  deviation field) decides nothing: the traced states and the interface
  state at B_n = 0 and at B_n = +-1e-14 agree, while a normal field well
  above the noise moves them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_02214_amd import inputs as I

import oracle_cases as OC

G = 5.0 / 3.0

STATES = [
    # rho, p, Bn, Bt1, Bt2
    (1.0, 1.0, 1.0, 1.2, 0.9),          # generic oblique
    (2.0, 0.5, -0.7, 0.3, -1.1),        # negative normal field
    (1.0, 1.0, 1.3, 0.0, 0.0),          # no transverse field
    (1.0, 1.0, 0.0, 0.8, 0.6),          # no normal field
    (1.0, 0.6, 1.0, 0.0, 0.0),          # a^2 = c_A^2 with no transverse field: c_f = c_s = c_A
    (0.5, 2.0, 0.4, 1e-9, 0.0),         # transverse field at rounding level
]


def _lagrangian_jacobian(rho, p, Bn, Bt1, Bt2):
    return rho * OC.mhd_jacobian(rho, p, Bn, Bt1, Bt2, G)


@pytest.mark.parametrize("st", STATES)
def test_eigen_structure_against_the_lagrangian_jacobian(st):
    rho, p, Bn, Bt1, Bt2 = st
    lam, R = O.mhd7_eigen(rho, p, G, Bn, Bt1, Bt2)
    A = _lagrangian_jacobian(rho, p, Bn, Bt1, Bt2)
    ref = np.sort(np.linalg.eigvals(A).real)
    assert np.allclose(np.sort(lam), ref, rtol=1e-10, atol=1e-10 * np.max(np.abs(ref)))
    assert np.all(np.diff(lam) >= -1e-12 * np.max(np.abs(lam)))          # -f, -A, -s, 0, +s, +A, +f
    scale = np.max(np.abs(A)) * np.max(np.abs(R))
    assert np.max(np.abs(A @ R - R * lam[None, :])) <= 1e-12 * scale
    assert np.linalg.cond(R) < 1e6                                        # complete at degeneracies


def _quad_parabola(c):
    """PPM parabola (aL, dA, a6) of q(xi) = c0 + c1 xi + c2 xi^2 on [0, 1]."""
    c0, c1, c2 = c
    return c0, c1 + c2, -c2


def _avg_right(c, y):       # mean of q over [1 - y, 1]
    c0, c1, c2 = c
    F = lambda x: c0 * x + c1 * x * x / 2 + c2 * x ** 3 / 3
    return (F(1.0) - F(1.0 - y)) / y


def _avg_left(c, y):        # mean of q over [0, y]
    c0, c1, c2 = c
    F = lambda x: c0 * x + c1 * x * x / 2 + c2 * x ** 3 / 3
    return F(y) / y


@pytest.mark.parametrize("st", STATES[:2])
@pytest.mark.parametrize("k", range(7))
def test_single_wave_traces_to_its_own_domain_average(st, k):
    rho, p, Bn, Bt1, Bt2 = st
    A = _lagrangian_jacobian(rho, p, Bn, Bt1, Bt2)
    lam, V = np.linalg.eig(A)
    order = np.argsort(lam.real)
    lam, V = lam.real[order], V.real[:, order]
    W0 = np.array([rho, 0.3, -0.2, 0.1, Bt1, Bt2, p])
    eps = 1e-6
    c = (0.4, 1.3, -0.8)                    # the profile in the zone's mass coordinate
    r = V[:, k] / np.max(np.abs(V[:, k]))
    par = np.zeros((7, 3))
    for v in range(7):
        aL, dA, a6 = _quad_parabola(c)
        par[v] = (W0[v] + eps * r[v] * aL, eps * r[v] * dA, eps * r[v] * a6)
    Wbar = W0 + eps * r * (c[0] + c[1] / 2 + c[2] / 3)
    dt, dm = 0.31, 1.0
    WL, WR = O.trace7(Wbar[0], Wbar[6], G, Bn, Wbar[4], Wbar[5], par, dt, dm)
    lamb = np.sort(np.linalg.eigvals(_lagrangian_jacobian(Wbar[0], Wbar[6], Bn, Wbar[4], Wbar[5])).real)
    yf = min(1.0, lamb[6] * dt / dm)
    yk = min(1.0, abs(lamb[k]) * dt / dm)
    # right face: waves 4, 5, 6 arrive with their own averages, the others
    # keep the fast wave's
    exp_L = W0 + eps * r * (_avg_right(c, yk) if k >= 4 and lamb[k] > 0 else _avg_right(c, yf))
    exp_R = W0 + eps * r * (_avg_left(c, yk) if k <= 2 and lamb[k] < 0 else _avg_left(c, yf))
    # O(eps^2): the eigenvectors are taken at the zone average
    assert np.max(np.abs(WL - exp_L)) <= 1e-4 * eps, (WL - exp_L) / eps
    assert np.max(np.abs(WR - exp_R)) <= 1e-4 * eps, (WR - exp_R) / eps


@pytest.mark.parametrize("st", STATES[:4])
def test_linear_riemann_problem_takes_the_left_going_waves(st):
    rho, p, Bn, Bt1, Bt2 = st
    rng = np.random.default_rng(11)
    WL = np.array([rho, 0.2, -0.1, 0.3, Bt1, Bt2, p])
    eps = 1e-7
    c = rng.uniform(-1.0, 1.0, 7)
    for _ in range(2):          # the mean state fixes the eigenvectors: iterate to it
        Wm = WL if _ == 0 else 0.5 * (WL + WR)
        lam, V = np.linalg.eig(_lagrangian_jacobian(Wm[0], Wm[6], Bn, Wm[4], Wm[5]))
        order = np.argsort(lam.real)
        lam, V = lam.real[order], V.real[:, order]
        WR = WL + eps * V @ c
    Ws = O.riemann7(WL, WR, G, Bn)
    expect = WL + eps * V[:, lam < -1e-12 * np.max(np.abs(lam))] @ c[lam < -1e-12 * np.max(np.abs(lam))]
    # the entropy wave (speed 0) carries density only, which no flux reads
    assert np.max(np.abs((Ws - expect)[1:])) <= 1e-4 * eps, (Ws - expect) / eps


def test_sod_shock_tube_converges_in_the_characteristic_mode():
    from oracle import exact_riemann as X
    errs = []
    for N in (100, 200, 400):
        f = I.uniform_faces(N)
        xc = I.centres(f)
        z = 0 * xc
        rho = np.where(xc < 0.5, 1.0, 0.125)
        p = np.where(xc < 0.5, 1.0, 0.1)
        U0 = I.conserved(rho, z, z, z, z, z, z, p).reshape(8, 1, 1, N)
        prob = O.OracleProblem([f, I.uniform_faces(1), I.uniform_faces(1)], bc_lo=(1, 0, 0), bc_hi=(1, 0, 0),
                               tracing=1)
        U, _ = OC.run_to(prob, U0, 0.2)
        ex = np.array([X.sample((x - 0.5) / 0.2, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1) for x in xc])
        errs.append(np.sum(np.abs(U[0, 0, 0] - ex[:, 0])) / N)
    errs = np.array(errs)
    print(f"sod, characteristic mode: density L1 errors {errs}")
    assert errs[0] < 8e-3
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 0.8), orders


def _order(errs):
    return np.log2(np.array(errs[:-1]) / np.array(errs[1:]))


@pytest.mark.parametrize("kind", ["fast", "alfven", "slow"])
def test_linear_eigenmodes_along_axis_converge_second_order(kind):
    errs = {0: [], 1: []}
    for N in (32, 64, 128):
        U0, faces, lam = OC.wave_state_1d(N, kind, B=(1.0, 1.2, 0.9))
        for tr in (0, 1):
            prob = O.OracleProblem(faces, tracing=tr)
            U, _ = OC.run_to(prob, U0, 1.0 / lam)
            errs[tr].append(np.sum(np.abs(U - U0)) / N)
    o7 = _order(errs[1])
    print(f"{kind}: seven-wave errors {errs[1]} orders {o7}; two-family errors {errs[0]}")
    assert np.all(o7 >= 1.8), o7
    # the same size of error as the two-family mode on the same runs
    assert errs[1][-1] <= 2.0 * errs[0][-1], (errs[1], errs[0])


@pytest.mark.parametrize("kind", ["fast", "alfven", "slow"])
def test_oblique_eigenmodes_converge_second_order(kind):
    errs = {0: [], 1: []}
    for N in (16, 32, 64):
        U0, faces, lam, T = OC.oblique_wave_state(N, kind)
        for tr in (0, 1):
            prob = O.OracleProblem(faces, tracing=tr)
            U, _ = OC.run_to(prob, U0, T)
            errs[tr].append(np.sum(np.abs(U - U0)) / N ** 2)
    o7 = _order(errs[1])
    print(f"{kind} oblique: seven-wave errors {errs[1]} orders {o7}; two-family errors {errs[0]}")
    assert np.mean(o7) >= 1.8 and o7[-1] >= 1.7, o7
    assert errs[1][-1] <= 2.0 * errs[0][-1], (errs[1], errs[0])


def test_uniform_state_bitwise_and_periodic_conservation():
    rng = np.random.default_rng(7)
    faces = [np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 1.5, n))]) for n in (12, 10, 9)]
    U = I.conserved(1.3 + 0 * np.ones((9, 10, 12)), 0.2, -0.1, 0.3, 0.7, -0.4, 1.1, 0.9, G)
    prob = O.OracleProblem(faces, tracing=1)
    dt = prob.cfl_dt(U, 0.4)
    out = prob.step(U, dt, 0)
    assert np.array_equal(out, U)
    Uc, faces_c = I.c1_state(n=16)
    prob = O.OracleProblem(faces_c, tracing=1)
    U1 = Uc.copy()
    for s in range(5):
        U1 = prob.step(U1, prob.cfl_dt(U1, 0.4), s)
    t0, t1 = prob.totals(Uc), prob.totals(U1)
    for q in (0, 1, 2, 3, 7):
        assert abs(t1[q] - t0[q]) <= 1e-13 * max(abs(t0[q]), 1.0), (q, t0[q], t1[q])


def test_split_multid_terms_leave_rho_and_p_and_move_the_field():
    N = 24
    faces = [I.uniform_faces(N), I.uniform_faces(1), I.uniform_faces(1)]
    xc = I.centres(faces[0])
    rho, p = 1.3, 0.9
    vt, bt = (0.4, -0.3), (0.7, 0.5)
    # B'_x varies along the pencil (as it does in a split multi-D step)
    bx = 0.8 + 0.2 * np.sin(2 * np.pi * xc)
    one = np.ones(N)
    U = I.conserved(rho * one, 0 * one, vt[0] * one, vt[1] * one, bx, bt[0] * one, bt[1] * one, p * one,
                    G)[:, None, None, :]
    prob = O.OracleProblem(faces, tracing=1)
    dt = prob.cfl_dt(U, 0.4)
    WL, WR = prob.face_states(U, dt, 0, 0, 0)
    for W in (WL, WR):
        # (the zone values themselves are recovered from the conserved
        # energy, so they sit within a few ulps of p)
        assert np.max(np.abs(W[:, 0] - rho)) <= 1e-14, W[:, 0] - rho
        assert np.max(np.abs(W[:, 6] - p)) <= 1e-14, W[:, 6] - p
        assert np.all(W[:, 1] != 0.0)                 # u takes B_n dB_n/dm
        # the field moves with the time-centring terms (rho v_t dB_n/dm)
        assert np.max(np.abs(W[:, 4] - bt[0])) > 1e-3
        assert np.max(np.abs(W[:, 5] - bt[1])) > 1e-3
    with pytest.raises(ValueError):
        O.OracleProblem(faces, tracing=0).face_states(U, dt, 0, 0, 0)


def test_inflow_dipole_stays_finite_and_positive():
    import gpu_cases as GC
    case = GC.dipole_case()
    case.tracing = 1
    prob = case.oracle()
    U = case.U.copy()
    for s in range(3):
        U = prob.step(U, prob.cfl_dt(U, 0.4), s)
    assert np.all(np.isfinite(U))
    rho = U[0]
    p = (G - 1) * (U[7] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho - 0.5 * (U[4] ** 2 + U[5] ** 2 + U[6] ** 2))
    assert rho.min() > 0 and p.min() > 0


def test_rounding_level_normal_field_decides_nothing():
    rng = np.random.default_rng(11)
    rho, p, Bt1, Bt2 = 1.2, 0.9, 0.7, -0.4
    # parabolas with gradients in every primitive (v_t and B_t included)
    base = np.array([rho, 0.1, 0.3, -0.2, 0.0, 0.0, p])
    par = np.zeros((7, 3))
    par[:, 0] = base + 0.05 * rng.standard_normal(7)      # left edge
    par[:, 1] = 0.1 * rng.standard_normal(7)              # aR - aL
    par[:, 2] = 0.02 * rng.standard_normal(7)             # a6
    dt, dm = 0.05, 1.0
    tr0 = O.trace7(rho, p, G, 0.0, Bt1, Bt2, par, dt, dm)
    WL0, WR0 = tr0
    WRn = WR0 + 0.03 * rng.standard_normal(7)
    rs0 = O.riemann7(WL0, WRn, G, 0.0, 0.2, -0.1)
    for Bn in (1e-14, -1e-14):
        WL, WR = O.trace7(rho, p, G, Bn, Bt1, Bt2, par, dt, dm)
        assert np.max(np.abs(WL - WL0)) <= 1e-12 and np.max(np.abs(WR - WR0)) <= 1e-12, (Bn, WL - WL0, WR - WR0)
        rs = O.riemann7(WL0, WRn, G, Bn, 0.2, -0.1)
        assert np.max(np.abs(rs - rs0)) <= 1e-12, (Bn, rs - rs0)
    # a normal field well above the noise: the Alfven and slow waves take part
    WL, WR = O.trace7(rho, p, G, 0.05, Bt1, Bt2, par, dt, dm)
    assert np.max(np.abs(WL - WL0)) > 1e-4
    rs = O.riemann7(WL0, WRn, G, 0.05, 0.2, -0.1)
    assert np.max(np.abs(rs - rs0)) > 1e-4
