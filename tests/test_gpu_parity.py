"""GPU-vs-oracle parity of the HIP sweep, through the C ABI.

Tolerances (FP64 path): 1e-12 normwise per conserved variable after one
sweep; 1e-10 after 20 split steps (both sides run the same algorithm; they
differ only in rounding order and FMA contraction, which near-tie branches of
the limiter can amplify locally).  Pointwise (each zone against its own
magnitude, floored at 1e-6 of the variable's largest value): 1e-7 after one
step, 1e-6 after 20 steps (momentum components cross zero, where the floor
sets the scale: a normwise 1e-12 shows there as up to 1e-6; an error local
to a small-valued region, such as the near-static magnetosphere, is measured
against its own values).  FP32 path: compared with the FP64 oracle
on the FP32-rounded input; bound stated per test (single-precision rounding
through ~10^3 operations per zone, relative ~1e-5).
"""
import numpy as np
import pytest

from paper_1607_02214_amd import inputs as I

import gpu_cases as GC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(U, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(U)).to(device="cuda", dtype=dtype).contiguous()


def _host(u):
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_02214_amd import ppmlr
    ppmlr.lib()  # raises if the library is not built


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c1_single_sweep_fp64(axis):
    case = GC.c1_case()
    GC.log(f"[parity] c1 32^3 fp64 sweep axis={axis}")
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    ref = ora.sweep(case.U, dt, axis)
    ctx = case.context()
    u = _dev(case.U)
    ctx.sweep(u, dt, axis)
    err = GC.normwise_errors(_host(u), ref)
    assert np.all(err <= 1e-12), err


def test_c1_twenty_steps_fp64_and_dt():
    case = GC.c1_case()
    GC.log("[parity] c1 32^3 fp64 20 steps")
    ora = case.oracle()
    ctx = case.context()
    u = _dev(case.U)
    U = case.U.copy()
    for s in range(20):
        dt_o = ora.cfl_dt(U, 0.4)
        dt_g = ctx.cfl_dt(u, 0.4)
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o
        U = ora.step(U, dt_o, s)
        ctx.step(u, dt_o)
        if s == 0:
            err1 = GC.normwise_errors(_host(u), U)
            assert np.all(err1 <= 1e-12), err1
    got = _host(u)
    err = GC.normwise_errors(got, U)
    assert np.all(err <= 1e-10), err
    pw = GC.pointwise_errors(got, U)
    GC.log(f"[parity] c1 20 steps normwise {err.max():.2e} pointwise {pw}")
    assert np.all(pw <= 1e-6), pw
    st = ctx.stats()
    assert st["floor_hits"] == 0 and st["nonconverged"] == 0 and st["nonphys"] == 0


@pytest.mark.parametrize("maker", [GC.dipole_case, GC.blast_case, GC.smooth_case])
def test_one_step_fp64_stretched_dipole_shocks(maker):
    case = maker()
    GC.log(f"[parity] {case.name} fp64 one step shape={case.U.shape}")
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    from oracle import oracle as O
    st = O.Stats()
    ref = ora.step(case.U, dt, 0, st)
    ctx = case.context()
    u = _dev(case.U)
    ctx.step(u, dt)
    got = _host(u)
    err = GC.normwise_errors(got, ref)
    assert np.all(err <= 1e-11), err
    pw = GC.pointwise_errors(got, ref)
    GC.log(f"[parity] {case.name} one step normwise {err.max():.2e} pointwise {pw}")
    assert np.all(pw <= 1e-7), pw
    gst = ctx.stats()
    assert gst["floor_hits"] == st.floor_hits and gst["nonconverged"] == st.nonconverged
    # iteration histograms agree up to faces sitting exactly on the tolerance
    gh, oh = np.array(gst["iters_hist"]), np.array(st.iters_hist)
    assert gh.sum() == oh.sum()
    assert np.abs(gh - oh).sum() <= max(4, 1e-4 * oh.sum())


def test_background_field_and_odd_shapes_fp64():
    # uniform external field carried as B_d, ragged tiles, prime sizes
    case = GC.smooth_case(shape=(13, 11, 23), seed=8, bext=(0.3, -0.2, 0.5))
    GC.log(f"[parity] bext odd shapes {case.U.shape}")
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    for axis in range(3):
        ref = ora.sweep(case.U, dt, axis)
        for P in (1, 2, 3):
            ctx = case.context()
            ctx.set_tile(axis, P)
            u = _dev(case.U)
            ctx.sweep(u, dt, axis)
            err = GC.normwise_errors(_host(u), ref)
            assert np.all(err <= 1e-12), (axis, P, err)


def test_degenerate_one_zone_axes_and_minimum_pencils():
    # 1D problem: size-1 periodic axes; outflow axis at the 7-zone minimum
    N = 64
    f = I.uniform_faces(N)
    xc = I.centres(f)
    z = 0 * xc
    rho = np.where(xc < 0.5, 1.0, 0.125)
    p = np.where(xc < 0.5, 1.0, 0.1)
    U = I.conserved(rho, z, z, z, 0.75 + z, np.where(xc < 0.5, 1.0, -1.0), z, p).reshape(8, 1, 1, N)
    case = GC.Case("briowu-1d", [f, I.uniform_faces(1), I.uniform_faces(1)], U, bc_lo=(1, 0, 0), bc_hi=(1, 0, 0))
    GC.log("[parity] 1d brio-wu")
    ora = case.oracle()
    ctx = case.context()
    u = _dev(U)
    Uo = U.copy()
    for s in range(10):
        dt = ora.cfl_dt(Uo, 0.5)
        Uo = ora.step(Uo, dt, s)
        ctx.step(u, dt)
    err = GC.normwise_errors(_host(u), Uo)
    assert np.all(err <= 1e-11), err
    # the smallest non-periodic pencil (7 zones) along every axis
    U7 = I.random_smooth_state((7, 7, 7), seed=2)
    case7 = GC.Case("min7", [I.uniform_faces(7)] * 3, U7, bc_lo=(1, 1, 1), bc_hi=(1, 1, 1))
    ora = case7.oracle()
    dt = ora.cfl_dt(U7, 0.4)
    ref = ora.step(U7, dt, 0)
    ctx = case7.context()
    u = _dev(U7)
    ctx.step(u, dt)
    err = GC.normwise_errors(_host(u), ref)
    assert np.all(err <= 1e-12), err


def test_fp32_against_fp64_oracle():
    for case in (GC.c1_case(), GC.dipole_case()):
        GC.log(f"[parity] fp32 {case.name}")
        U32 = case.U.astype(np.float32).astype(np.float64)
        ora = case.oracle()
        dt = ora.cfl_dt(U32, 0.4)
        ref = ora.step(U32, dt, 0)
        ctx = case.context()
        u = _dev(U32, torch.float32)
        ctx.step(u, dt)
        err = GC.fp32_errors(_host(u), ref)
        GC.log(f"[parity] fp32 {case.name} errors {err}")
        # single-precision rounding through ~10^3 operations per zone
        assert all(v <= 2e-5 for v in err.values()), (case.name, err)
        tot_g = ctx.totals(u)
        tot_o = ora.totals(ref)
        for q in (0, 7):
            assert abs(tot_g[q] - tot_o[q]) <= 1e-5 * abs(tot_o[q]), (q, tot_g[q], tot_o[q])


@pytest.mark.parametrize("maker", [GC.dipole_case, GC.c1_case])
def test_fp32_fused_dt_matches_oracle_cfl_dt(maker):
    # The device-resident step loop takes the first dt from the FP64 CFL
    # kernel and every later one from the signal-speed maximum fused into the
    # previous step's last FP32 sweep.  Runs of k and k + 1 steps from one
    # start agree bitwise over their first k steps, so dt_k = t_{k+1} - t_k
    # belongs to the state after k steps, which the oracle's FP64 CFL dt
    # takes as its input.
    case = maker()
    ora = case.oracle()
    U32 = case.U.astype(np.float32)

    def run(k):
        ctx = case.context()
        u = _dev(U32, torch.float32)
        if k:
            ctx.advance(u, k, 0.4)
        return _host(u), ctx.time(u)

    runs = [run(k) for k in range(5)]
    for k in range(4):
        S, t_k = runs[k]
        dt_g = runs[k + 1][1] - t_k
        dt_o = ora.cfl_dt(S, 0.4)
        rel = abs(dt_g - dt_o) / dt_o
        GC.log(f"[parity] {case.name} fp32 dt of step {k} ({'fused' if k else 'fp64 kernel'}): gpu {dt_g:.12e} "
               f"oracle {dt_o:.12e} rel {rel:.2e}")
        # the fast speeds are evaluated in FP32 (a few roundings each)
        assert rel <= 2e-6, (k, dt_g, dt_o)


def test_totals_deterministic_and_match_oracle():
    case = GC.smooth_case(shape=(20, 24, 28), seed=1)
    ora = case.oracle()
    ctx = case.context()
    u = _dev(case.U)
    t1 = ctx.totals(u)
    t2 = ctx.totals(u)
    assert np.array_equal(t1, t2)
    to = ora.totals(case.U)
    assert np.all(np.abs(t1 - to) <= 1e-13 * np.maximum(np.abs(to), 1e-12))


def test_sweeps_are_deterministic():
    case = GC.blast_case()
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    outs = []
    for _ in range(2):
        ctx = case.context()
        u = _dev(case.U, torch.float32)
        for k in range(3):
            ctx.step(u, dt)
        outs.append(_host(u))
    assert np.array_equal(outs[0], outs[1])


def test_advance_matches_host_driven_steps():
    case = GC.dipole_case()
    GC.log("[parity] advance vs step")
    ctx_a = case.context()
    ctx_b = case.context()
    ua = _dev(case.U)
    ub = _dev(case.U)
    ctx_a.advance(ua, 4, 0.4)
    t = 0.0
    for s in range(4):
        dt = ctx_b.cfl_dt(ub, 0.4)
        ctx_b.step(ub, dt)
        t += dt
    assert abs(ctx_a.time(ua) - t) <= 1e-12 * t
    err = GC.normwise_errors(_host(ua), _host(ub))
    assert np.all(err <= 1e-12), err


def test_error_paths():
    from paper_1607_02214_amd import ppmlr
    case = GC.smooth_case(shape=(9, 10, 11))
    ctx = case.context()
    u = _dev(case.U)
    with pytest.raises(ppmlr.PPMLRError) as e:
        ctx.sweep(u, 1e-3, 3)
    assert e.value.status == ppmlr.PPMLR_EINVAL
    with pytest.raises(ppmlr.PPMLRError) as e:
        ctx.sweep(u, -1.0, 0)
    assert e.value.status == ppmlr.PPMLR_EINVAL
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_inflow([1, 0, 0, 0, 0, 0, 0, -1])
    # non-physical zone -> ENONPHYS through the status check
    Ub = case.U.copy()
    Ub[0, 3, 4, 5] = -1.0
    ctx.reset_stats()
    ub = _dev(Ub)
    ctx.sweep(ub, 1e-4, 0)
    assert ctx.status_check() == ppmlr.PPMLR_ENONPHYS
    # NaN in the input -> ENONPHYS through the status check
    Un = case.U.copy()
    Un[7, 2, 3, 4] = np.nan
    ctx.reset_stats()
    ctx.sweep(_dev(Un), 1e-4, 1)
    assert ctx.status_check() == ppmlr.PPMLR_ENONPHYS
    assert ctx.stats()["nonphys"] >= 1
    # Newton limit reached -> ERIEMANN
    blast = GC.blast_case()
    ctx2 = blast.context(max_iter=1, tol_f64=1e-15)
    ub = _dev(blast.U)
    dt = blast.oracle().cfl_dt(blast.U, 0.4)
    ctx2.step(ub, dt)
    assert ctx2.status_check() == ppmlr.PPMLR_ERIEMANN
    # bad grid
    with pytest.raises(ppmlr.PPMLRError):
        ppmlr.Context([I.uniform_faces(5)] * 3, (1, 1, 1), (1, 1, 1))
    # debug CFL check
    ctx3 = case.context(debug_cfl=1)
    lim = ctx3.cfl_dt(u, 1.0)
    with pytest.raises(ppmlr.PPMLRError) as e:
        ctx3.step(u, 2.0 * lim)
    assert e.value.status == ppmlr.PPMLR_ECFL
