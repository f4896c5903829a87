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



@pytest.mark.timeout(600)
def test_bench_workload_sampled_pencils_fp32():
    # The benchmark's inflow-dipole grid (256 x 192 x 192, FP32, automatic
    # tiles, device dt loop) in the characteristic mode: 5 steps, then one
    # sweep per axis; sampled pencils (and the pencils through the middle:
    # dipole, inner boundary, bow shock) against the oracle's characteristic
    # mode on the same FP32-rounded input, pencil by pencil.
    from oracle import oracle as O
    from paper_1607_02214_amd import inputs as I
    from paper_1607_02214_amd import ppmlr
    setup = I.c2_setup()
    n = [len(f) - 1 for f in setup.faces]
    GC.log(f"[char] inflow-dipole {n} fp32: 5 steps, one sweep per axis")
    ctx = ppmlr.Context(setup.faces, setup.bc_lo, setup.bc_hi, r_inner=setup.r_inner, p_floor=setup.p_floor,
                        tracing=1)
    ctx.set_dipole(setup.moment, setup.direction)
    ctx.set_inflow(setup.inflow)
    ctx.set_inner(setup.inner_rho, setup.inner_p)
    u = _dev(setup.U, torch.float32)
    ctx.advance(u, 5, 0.4)
    ora = O.OracleProblem(setup.faces, bc_lo=setup.bc_lo, bc_hi=setup.bc_hi, dip_moment=setup.moment,
                          dip_dir=setup.direction, inflow=setup.inflow, r_inner=setup.r_inner,
                          inner_rho=setup.inner_rho, inner_p=setup.inner_p, p_floor=setup.p_floor, tracing=1)
    rng = np.random.default_rng(77)
    for axis in range(3):
        Uin = _host(u)
        dt = ctx.cfl_dt(u, 0.4)
        ctx.sweep(u, dt, axis)
        out = _host(u)
        n1, n2 = n[(axis + 1) % 3], n[(axis + 2) % 3]
        j1 = np.concatenate([rng.integers(0, n1, 32), [n1 // 2, n1 // 2 - 1, n1 // 2]])
        j2 = np.concatenate([rng.integers(0, n2, 32), [n2 // 2, n2 // 2, n2 // 2 - 1]])
        ref = ora.sweep_pencils(Uin, dt, axis, j1, j2)
        got = np.empty_like(ref)
        for q in range(len(j1)):
            idx = [slice(None)] * 3
            idx[2 - (axis + 1) % 3] = j1[q]
            idx[2 - (axis + 2) % 3] = j2[q]
            got[q] = out[(slice(None),) + tuple(idx)]
        err = GC.fp32_errors(got.transpose(1, 0, 2).reshape(8, -1), ref.transpose(1, 0, 2).reshape(8, -1))
        GC.log(f"[char] bench workload axis {axis} fp32 vs oracle on {len(j1)} pencils: {err}")
        assert all(v <= 2e-5 for v in err.values()), (axis, err)

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
