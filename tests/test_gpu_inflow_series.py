"""Time-dependent driving at the inflow face through the C ABI: the series'
inflow at each step's mid-time, against the FP64 oracle stepped with the same
states (host-given dt and the device-resident dt loop); a constant series is
bitwise the constant inflow; argument checks."""
import numpy as np
import pytest

from paper_1607_02214_amd import inputs as I

import gpu_cases as GC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_02214_amd import ppmlr
    ppmlr.lib()


def _dev(U, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype).contiguous()


def _host(u):
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


def test_host_steps_with_series_match_oracle_fp64():
    from oracle import oracle as O
    case = GC.dipole_case()
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.3)
    times, prims = I.solar_wind_series(6 * dt, n_knots=5, seed=3)
    ctx = case.context()
    ctx.set_inflow_series(times, prims)
    u = _dev(case.U)
    # a lone sweep takes the series at t + dt/2 without advancing the time
    ref = ora
    ref.set_inflow(O.inflow_series_at(times, prims, 0.5 * dt))
    w = _dev(case.U)
    ctx.sweep(w, dt, 0)
    err = GC.normwise_errors(_host(w), ref.sweep(case.U, dt, 0))
    assert np.all(err <= 1e-12), err
    assert ctx.time(w) == 0.0
    U, t = case.U, 0.0
    for s in range(6):
        ctx.step(u, dt)
        U = O.step_with_series(ora, U, dt, s, t, times, prims)
        t += dt
    err = GC.normwise_errors(_host(u), U)
    GC.log(f"[series] 6 host-driven FP64 steps vs oracle: {err}")
    assert np.all(err <= 1e-10), err
    assert ctx.time(u) == pytest.approx(6 * dt, rel=1e-14)
    # the series changes the run (it is not the constant inflow)
    plain = case.context()
    v = _dev(case.U)
    for s in range(6):
        plain.step(v, dt)
    assert float((u - v).abs().max()) > 1e-6


def test_device_dt_loop_with_series_matches_oracle_fp64():
    from oracle import oracle as O
    case = GC.dipole_case()
    ora = case.oracle()
    dt0 = ora.cfl_dt(case.U, 0.3)
    times, prims = I.solar_wind_series(5 * dt0, n_knots=6, seed=4)
    ctx = case.context()
    ctx.set_inflow_series(times, prims)
    u = _dev(case.U)
    U, t_prev = case.U, 0.0
    for s in range(4):
        ctx.advance(u, 1, 0.3)
        t_now = ctx.time(u)
        U = O.step_with_series(ora, U, t_now - t_prev, s, t_prev, times, prims)
        t_prev = t_now
    err = GC.normwise_errors(_host(u), U)
    GC.log(f"[series] 4 device-dt FP64 steps vs oracle: {err}")
    assert np.all(err <= 1e-10), err


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_constant_series_is_bitwise_the_constant_inflow(dtype):
    case = GC.dipole_case()
    prim = np.array(case.inflow)
    res = []
    for series in (False, True):
        ctx = case.context()
        if series:
            ctx.set_inflow_series([0.0, 1.0, 2.0], [prim, prim, prim])
        u = _dev(case.U, dtype)
        ctx.advance(u, 3, 0.4)
        dt = ctx.cfl_dt(u, 0.4)
        ctx.step(u, dt)
        torch.cuda.synchronize()
        res.append((u, ctx.time(u)))
    assert torch.equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]


def test_series_arguments():
    from paper_1607_02214_amd import ppmlr
    case = GC.dipole_case()
    ctx = case.context()
    prim = np.array(case.inflow)
    bad = prim.copy()
    bad[0] = -1.0
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_inflow_series([0.0, 0.0], [prim, prim])         # not increasing
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_inflow_series([0.0, 1.0], [prim, bad])          # negative density
    nan = prim.copy()
    nan[3] = np.nan
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_inflow_series([0.0, 1.0], [prim, nan])
    ctx.set_inflow_series([0.0, 1.0], [prim, prim])
    ctx.set_inflow_series([], [])                               # back to the constant inflow
    # ensembles do not take series
    ctx.set_inflow_series([0.0, 1.0], [prim, prim])
    u = _dev(case.U, torch.float32)
    with pytest.raises(ppmlr.PPMLRError):
        ppmlr.ensemble_run([ctx], [u], 1, 0.4, block=256)
