"""GPU-vs-oracle parity of the characteristic mode (ppmlr_options.tracing =
PPMLR_TRACE_CHARACTERISTIC: the seven waves traced one by one and the
interface problem of all seven waves in its linearisation), through the C
ABI, against the oracle's characteristic mode on the same inputs.

Both sides run the same algorithm and differ only in rounding order and FMA
contraction, so the bounds are those of the default mode, with each
variable measured against the largest value of its family (mass, momentum,
field, energy: the transverse momentum of the blast, zero in exact
arithmetic, carries only rounding noise): FP64 1e-12 after one sweep,
1e-11 after one split step on shocks, stretched grids and the dipole, 1e-10
after 20 steps; pointwise (each zone against its own magnitude, floored at
1e-6 of its family's largest) 1e-7 after one step.  FP32 against the FP64 oracle on the
FP32-rounded input: 2e-5 (single-precision rounding through ~10^3 operations
per zone).  The counters: every face of the solve counts in bin 0 of the
iteration histogram (no iteration), floor hits as in the oracle."""
import numpy as np
import pytest

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


def _char(maker, **kw):
    case = maker(**kw)
    case.tracing = 1
    return case


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c1_single_sweep_fp64(axis):
    case = _char(GC.c1_case)
    GC.log(f"[char] c1 32^3 fp64 sweep axis={axis}")
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    ref = ora.sweep(case.U, dt, axis)
    ctx = case.context()
    u = _dev(case.U)
    ctx.sweep(u, dt, axis)
    err = GC.familywise_errors(_host(u), ref)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("maker", [GC.dipole_case, GC.blast_case, GC.smooth_case])
def test_one_step_fp64_dipole_shocks_stretched(maker):
    case = _char(maker)
    GC.log(f"[char] {case.name} fp64 one step shape={case.U.shape}")
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    from oracle import oracle as O
    st = O.Stats()
    ref = ora.step(case.U, dt, 0, st)
    assert np.all(np.isfinite(ref))
    ctx = case.context()
    u = _dev(case.U)
    ctx.step(u, dt)
    got = _host(u)
    err = GC.familywise_errors(got, ref)
    pw = GC.pointwise_errors(got, ref, by_family=True)
    GC.log(f"[char] {case.name} one step normwise {err.max():.2e} pointwise {pw.max():.2e}")
    assert np.all(err <= 1e-11), err
    assert np.all(pw <= 1e-7), pw
    gst = ctx.stats()
    assert gst["floor_hits"] == st.floor_hits and gst["nonconverged"] == 0 == st.nonconverged
    gh, oh = np.array(gst["iters_hist"]), np.array(st.iters_hist)
    assert np.array_equal(gh, oh), (gh, oh)
    assert gh[0] == gh.sum() > 0


def test_c1_twenty_steps_fp64():
    case = _char(GC.c1_case)
    GC.log("[char] c1 32^3 fp64 20 steps")
    ora = case.oracle()
    ctx = case.context()
    u = _dev(case.U)
    U = case.U.copy()
    for s in range(20):
        dt = ora.cfl_dt(U, 0.4)
        U = ora.step(U, dt, s)
        ctx.step(u, dt)
    got = _host(u)
    err = GC.familywise_errors(got, U)
    GC.log(f"[char] c1 20 steps normwise {err.max():.2e}")
    assert np.all(err <= 1e-10), err


def test_background_field_odd_shapes_and_tiles_fp64():
    case = _char(GC.smooth_case, shape=(13, 11, 23), seed=8, bext=(0.3, -0.2, 0.5))
    GC.log(f"[char] bext odd shapes {case.U.shape}")
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    for axis in range(3):
        ref = ora.sweep(case.U, dt, axis)
        for P in (1, 2, 3):
            ctx = case.context()
            ctx.set_tile(axis, P)
            u = _dev(case.U)
            ctx.sweep(u, dt, axis)
            err = GC.familywise_errors(_host(u), ref)
            assert np.all(err <= 1e-12), (axis, P, err)


def test_fp32_against_fp64_oracle():
    for case in (_char(GC.c1_case), _char(GC.dipole_case)):
        GC.log(f"[char] fp32 {case.name}")
        U32 = case.U.astype(np.float32).astype(np.float64)
        ora = case.oracle()
        dt = ora.cfl_dt(U32, 0.4)
        ref = ora.step(U32, dt, 0)
        ctx = case.context()
        u = _dev(U32, torch.float32)
        ctx.step(u, dt)
        err = GC.fp32_errors(_host(u), ref)
        GC.log(f"[char] fp32 {case.name} errors {err}")
        assert all(v <= 2e-5 for v in err.values()), (case.name, err)


def test_modes_that_do_not_take_the_characteristic_mode_are_refused():
    from paper_1607_02214_amd import inputs as I
    from paper_1607_02214_amd import ppmlr
    case = _char(GC.smooth_case, shape=(9, 10, 11))
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    # an unknown tracing value is refused at creation
    with pytest.raises(ppmlr.PPMLRError) as ei:
        case.context(tracing=2)
    assert ei.value.status == ppmlr.PPMLR_EINVAL
    # the learned initial guess belongs to the two-shock Newton solve
    ctx = case.context()
    u = _dev(case.U, torch.float32)
    before = u.clone()
    ctx.set_guess(ppmlr.GUESS_LEARNED, torch.from_numpy(I.mlp_init(1)).cuda())
    with pytest.raises(ppmlr.PPMLRError) as ei:
        ctx.sweep(u, dt, 0)
    assert ei.value.status == ppmlr.PPMLR_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(u, before)
    # ensembles run the two-family tracing only
    ctx2 = case.context()
    with pytest.raises(ppmlr.PPMLRError) as ei:
        ppmlr.ensemble_run([ctx2], [u], 1, 0.4, block=512)
    assert ei.value.status == ppmlr.PPMLR_EINVAL and "two-family" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
