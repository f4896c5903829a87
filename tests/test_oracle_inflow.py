"""Oracle pins for time-dependent driving at the inflow face: the series'
interpolation against its closed forms, and its use by a split step (the
state at the step's mid-time)."""
import numpy as np
import pytest

from oracle import oracle as O


def _series(seed=0, n=7):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.uniform(0.2, 1.0, n)) - 0.5
    P = rng.uniform(0.5, 2.0, (n, 8))
    return t, P


def test_knots_are_reproduced_exactly_and_ends_are_held():
    t, P = _series()
    for k in range(len(t)):
        assert np.array_equal(O.inflow_series_at(t, P, t[k]), P[k])
    assert np.array_equal(O.inflow_series_at(t, P, t[0] - 5.0), P[0])
    assert np.array_equal(O.inflow_series_at(t, P, t[-1] + 5.0), P[-1])


def test_linear_series_is_reproduced_between_knots():
    # knots sampled from a + b t: the interpolant is that line everywhere
    # inside (a wrong weight, index or sign fails this)
    rng = np.random.default_rng(1)
    t = np.sort(rng.uniform(-3.0, 3.0, 9))
    a, b = rng.normal(size=8), rng.normal(size=8)
    P = a[None, :] + t[:, None] * b[None, :]
    for tq in rng.uniform(t[0], t[-1], 50):
        assert np.allclose(O.inflow_series_at(t, P, tq), a + b * tq, rtol=0, atol=1e-13)
    mid = 0.5 * (t[3] + t[4])
    assert np.allclose(O.inflow_series_at(t, P, mid), 0.5 * (P[3] + P[4]), rtol=0, atol=1e-14)


def _inflow_box():
    # uniform flow entering through the x-max face; y and z periodic
    faces = [np.linspace(0.0, 1.0, 17), np.linspace(0.0, 0.25, 5), np.linspace(0.0, 0.25, 5)]
    prim0 = [1.0, -0.5, 0.0, 0.0, 0.0, 0.0, 0.5, 1.0]
    prob = O.OracleProblem(faces, bc_lo=(O.BC_OUTFLOW, O.BC_PERIODIC, O.BC_PERIODIC),
                           bc_hi=(O.BC_INFLOW, O.BC_PERIODIC, O.BC_PERIODIC), inflow=prim0)
    rho, v, B, p = prim0[0], np.array(prim0[1:4]), np.array(prim0[4:7]), prim0[7]
    U = np.zeros(prob.shape)
    U[0], U[1:4] = rho, (rho * v)[:, None, None, None]
    U[4:7] = B[:, None, None, None]
    U[7] = p / (2.0 / 3.0) + 0.5 * rho * v @ v + 0.5 * B @ B
    return prob, U, np.array(prim0)


def test_constant_series_steps_like_the_constant_inflow():
    prob, U, prim0 = _inflow_box()
    dt = prob.cfl_dt(U, 0.4)
    ref = prob.step(U, dt, 0)
    got = O.step_with_series(prob, U, dt, 0, 0.0, [0.0, 1.0], [prim0, prim0])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("jump,first", [(2.3, 2), (2.7, 3)])
def test_a_jump_enters_at_the_first_step_whose_mid_time_passes_it(jump, first):
    # mid-times 0.5, 1.5, 2.5, 3.5 dt: a jump at 2.3 dt enters at step 2 and
    # one at 2.7 dt at step 3 (start times would give 3 and 3, end times 2
    # and 2)
    prob, U, prim0 = _inflow_box()
    dt = prob.cfl_dt(U, 0.4)
    prim1 = prim0.copy()
    prim1[0] = 2.0                              # denser wind after the jump
    t_jump = jump * dt
    times = [0.0, t_jump, t_jump + 1e-9 * dt]
    prims = [prim0, prim0, prim1]
    t = 0.0
    for s in range(first + 1):
        Un = O.step_with_series(prob, U, dt, s, t, times, prims)
        if s < first:
            assert np.array_equal(Un, U), s     # uniform state: still the first knot's inflow
        else:
            assert Un[0, :, :, -1].min() > 1.0 + 1e-6     # the zone next to the face sees the denser wind
            assert np.array_equal(Un[:, :, :, :8], U[:, :, :, :8])
        U, t = Un, t + dt
