"""GPU-vs-oracle parity of the ionosphere shell coupling (ppmlr_ionosphere_couple,
paper Section II: the shell at 1.017 R_E, its potential, and the drift it
gives the zones inside the inner boundary), through the C ABI, against the
oracle's coupling (oracle/ionosphere.py) on the same state.

Bounds: the shell current takes the same FP64 arithmetic on both sides
(the FP32 state is read exactly), 1e-12 of its largest value; the
potential comes from two direct solves of the same finite-volume system
(Fourier transform in longitude and tridiagonal elimination on the GPU, a
sparse LU factorisation in the oracle), 1e-11 of its largest value; the
drift and the sweeps that take it: 1e-10, family-scaled, after a coupled
sweep and after three coupled steps (the drift takes differences of the
mapped potential)."""
import numpy as np
import pytest

from paper_1607_02214_amd import inputs as I

import gpu_cases as GC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

M_EARTH = 30936.214602350923


@pytest.fixture(scope="module", autouse=True)
def _gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_02214_amd import ppmlr
    ppmlr.lib()


def _case(n=32, L=8.0, seed=2, stretch=False):
    if stretch:
        rng = np.random.default_rng(seed)
        faces = []
        for _ in range(3):
            w = rng.uniform(0.8, 1.2, n)
            f = np.concatenate([[0.0], np.cumsum(w)])
            faces.append(-L + 2 * L * f / f[-1])
    else:
        faces = [np.linspace(-L, L, n + 1)] * 3
    U = I.random_smooth_state((n, n, n), seed=seed, amp=0.2)
    # the zones inside the inner boundary start in the inner state (rest,
    # B' = 0, rho = p = 1), as the sweeps leave them
    xc, yc, zc = (0.5 * (f[1:] + f[:-1]) for f in faces)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    inside = X * X + Y * Y + Z * Z < 9.0
    U[:, inside] = 0.0
    U[0, inside] = 1.0
    U[7, inside] = 1.0 / (5.0 / 3.0 - 1.0)
    return GC.Case("iono-smooth", faces, U, bc_lo=(1, 1, 1), bc_hi=(1, 1, 1), dip_moment=M_EARTH,
                   dip_dir=(0.0, 0.0, -1.0), r_inner=3.0, inner_rho=1.0, inner_p=1.0)


def _oracle_couple(case, prob, U, prm):
    from oracle import ionosphere as IO
    grid = IO.ShellGrid(prm.n_theta, prm.n_phi, r_shell=prm.r_shell, r_fac=prm.r_fac)
    return IO.couple(prob, U, grid, prm.sigma)


def _dev(U, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype).contiguous()


def _host(u):
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


@pytest.mark.parametrize("stretch", [False, True])
def test_shell_current_potential_and_coupled_sweep_fp64(stretch):
    from paper_1607_02214_amd import ppmlr
    case = _case(stretch=stretch)
    GC.log(f"[iono] fp64 stretch={stretch}")
    prm = ppmlr.iono_default_params()
    prm.n_theta, prm.n_phi = 24, 48
    ctx = case.context()
    u = _dev(case.U)
    jr = torch.zeros((2, 24, 48), dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(jr)
    ctx.ionosphere_couple(u, prm, jr=jr, phi=phi)
    prob = case.oracle()
    jr_o, phi_o, box, v_o = _oracle_couple(case, prob, case.U, prm)
    jr_g, phi_g = _host(jr), _host(phi)
    e_jr = float(np.max(np.abs(jr_g - jr_o)) / np.max(np.abs(jr_o)))
    e_phi = float(np.max(np.abs(phi_g - phi_o)) / np.max(np.abs(phi_o)))
    GC.log(f"[iono] jr {e_jr:.2e} phi {e_phi:.2e} max|jr| {np.max(np.abs(jr_o)):.3e}")
    assert np.max(np.abs(jr_o)) > 0 and np.max(np.abs(v_o)) > 0
    assert e_jr <= 1e-12, e_jr
    assert e_phi <= 1e-11, e_phi
    # a sweep with the drift in the reset zones, on both sides
    dt = prob.cfl_dt(case.U, 0.4)
    for axis in range(3):
        ref = prob.sweep(case.U, dt, axis)
        w = _dev(case.U)
        ctx.sweep(w, dt, axis)
        got = _host(w)
        err = GC.familywise_errors(got, ref)
        assert np.all(err <= 1e-10), (axis, err)
    # the reset zones carry rho v (inner rho = 1) with the oracle's drift
    i0, i1, j0, j1, k0, k1 = box
    xc, yc, zc = (0.5 * (f[1:] + f[:-1]) for f in case.faces)
    Z, Y, X = np.meshgrid(zc[k0:k1], yc[j0:j1], xc[i0:i1], indexing="ij")
    inside = X * X + Y * Y + Z * Z < 9.0
    m = got[1:4, k0:k1, j0:j1, i0:i1]
    assert inside.sum() > 0
    assert np.max(np.abs(m[:, inside] - v_o[:, inside])) <= 1e-10 * np.max(np.abs(v_o))


def test_fp32_state_reads_exactly():
    from paper_1607_02214_amd import ppmlr
    case = _case(seed=5)
    U32 = case.U.astype(np.float32).astype(np.float64)
    prm = ppmlr.iono_default_params()
    ctx = case.context()
    u = _dev(U32, torch.float32)
    jr = torch.zeros((2, prm.n_theta, prm.n_phi), dtype=torch.float64, device="cuda")
    ctx.ionosphere_couple(u, prm, jr=jr)
    prob = case.oracle()
    jr_o, _, _, _ = _oracle_couple(case, prob, U32, prm)
    e = float(np.max(np.abs(_host(jr) - jr_o)) / np.max(np.abs(jr_o)))
    GC.log(f"[iono] fp32 state jr {e:.2e}")
    assert e <= 1e-12, e


def test_three_coupled_steps_fp64_and_detach():
    from paper_1607_02214_amd import ppmlr
    case = _case(n=28, seed=7, stretch=True)
    prm = ppmlr.iono_default_params()
    prm.n_theta, prm.n_phi = 16, 32
    ctx = case.context()
    u = _dev(case.U)
    prob = case.oracle()
    U = case.U.copy()
    for s in range(3):
        ctx.ionosphere_couple(u, prm)
        _oracle_couple(case, prob, U, prm)
        dt = prob.cfl_dt(U, 0.4)
        U = prob.step(U, dt, s)
        ctx.step(u, dt)
    err = GC.familywise_errors(_host(u), U)
    GC.log(f"[iono] three coupled steps {err.max():.2e}")
    assert np.all(err <= 1e-10), err
    # detached: the reset zones are at rest again, as in the oracle without a drift
    ctx.ionosphere_detach()
    prob.set_inner_velocity(None)
    dt = prob.cfl_dt(U, 0.4)
    ref = prob.sweep(U, dt, 0)
    ctx.sweep(u, dt, 0)
    err = GC.familywise_errors(_host(u), ref)
    assert np.all(err <= 1e-10), err


def test_refusals():
    from paper_1607_02214_amd import ppmlr
    case = _case(n=16)
    u = _dev(case.U)
    ctx = case.context()
    for over in ({"n_theta": 128, "n_phi": 64}, {"r_fac": 9.0}, {"sigma": 0.0}, {"r_fac": 1.0},
                 {"n_theta": 1}, {"n_phi": 2}):
        with pytest.raises(ppmlr.PPMLRError) as ei:
            ctx.ionosphere_couple(u, **over)
        assert ei.value.status == ppmlr.PPMLR_EINVAL, over
    # no dipole
    c2 = GC.Case("no-dipole", case.faces, case.U, bc_lo=(1, 1, 1), bc_hi=(1, 1, 1), r_inner=3.0).context()
    with pytest.raises(ppmlr.PPMLRError) as ei:
        c2.ionosphere_couple(u)
    assert ei.value.status == ppmlr.PPMLR_EINVAL and "dipole" in str(ei.value)


@pytest.mark.timeout(600)
def test_coupling_on_the_bench_workload():
    # The benchmark's inflow-dipole run (256 x 192 x 192, FP32, device dt
    # loop) after 10 steps: the shell current and potential at the default
    # shell against the oracle on the same FP32 state, then one x sweep of
    # pencils through the reset zones against the oracle's sweep with the
    # oracle's drift.  The oracle's coupling reads the block of zones that
    # holds every zone the current's stencils touch around the r_fac sphere
    # (3 zones of margin): its differences are zone-local, so the block gives
    # the whole grid's values there.
    from oracle import oracle as O
    from oracle import ionosphere as IO
    from paper_1607_02214_amd import ppmlr
    setup = I.c2_setup()
    n = [len(f) - 1 for f in setup.faces]
    GC.log(f"[iono] bench workload {n} fp32: 10 steps, coupling, one x sweep")
    ctx = ppmlr.Context(setup.faces, setup.bc_lo, setup.bc_hi, r_inner=setup.r_inner, p_floor=setup.p_floor)
    ctx.set_dipole(setup.moment, setup.direction)
    ctx.set_inflow(setup.inflow)
    ctx.set_inner(setup.inner_rho, setup.inner_p)
    u = _dev(setup.U, torch.float32)
    ctx.advance(u, 10, 0.4)
    prm = ppmlr.iono_default_params()
    jr = torch.zeros((2, prm.n_theta, prm.n_phi), dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(jr)
    ctx.ionosphere_couple(u, prm, jr=jr, phi=phi)
    U = _host(u)
    cs = IO.centres(setup.faces)
    lo = [max(0, int(np.searchsorted(c, -prm.r_fac)) - 3) for c in cs]
    hi = [min(len(c), int(np.searchsorted(c, prm.r_fac)) + 3) for c in cs]
    sub = [np.asarray(setup.faces[a])[lo[a]:hi[a] + 1] for a in range(3)]
    Us = np.ascontiguousarray(U[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
    grid = IO.ShellGrid(prm.n_theta, prm.n_phi, r_shell=prm.r_shell, r_fac=prm.r_fac)
    jr_o = IO.shell_current(sub, Us, setup.moment, list(setup.direction), grid)
    phi_o = IO.solve_potential(grid, jr_o, prm.sigma)
    box, v_o = IO.inner_drift(sub, setup.r_inner, setup.moment, list(setup.direction), grid, phi_o)
    e_jr = float(np.max(np.abs(_host(jr) - jr_o)) / np.max(np.abs(jr_o)))
    e_phi = float(np.max(np.abs(_host(phi) - phi_o)) / np.max(np.abs(phi_o)))
    GC.log(f"[iono] bench workload: max|jr| {np.max(np.abs(jr_o)):.3e}, jr {e_jr:.2e}, phi {e_phi:.2e}")
    assert np.max(np.abs(jr_o)) > 0 and np.max(np.abs(v_o)) > 0
    assert e_jr <= 1e-12, e_jr
    assert e_phi <= 1e-11, e_phi
    ora = O.OracleProblem(setup.faces, bc_lo=setup.bc_lo, bc_hi=setup.bc_hi, dip_moment=setup.moment,
                          dip_dir=setup.direction, inflow=setup.inflow, r_inner=setup.r_inner,
                          inner_rho=setup.inner_rho, inner_p=setup.inner_p, p_floor=setup.p_floor)
    full = (box[0] + lo[0], box[1] + lo[0], box[2] + lo[1], box[3] + lo[1], box[4] + lo[2], box[5] + lo[2])
    ora.set_inner_velocity(full, v_o)
    dt = ctx.cfl_dt(u, 0.4)
    ctx.sweep(u, dt, 0)
    out = _host(u)
    ys = np.linspace(full[2], full[3] - 1, 5).astype(int)
    zs = np.linspace(full[4], full[5] - 1, 5).astype(int)
    j1 = np.repeat(ys, len(zs))
    j2 = np.tile(zs, len(ys))
    ref = ora.sweep_pencils(U, dt, 0, j1, j2)
    got = np.stack([out[:, j2[p], j1[p], :] for p in range(len(j1))])
    err = GC.fp32_errors(got.transpose(1, 0, 2).reshape(8, -1), ref.transpose(1, 0, 2).reshape(8, -1))
    GC.log(f"[iono] bench workload: coupled x sweep of {len(j1)} pencils through the reset zones: {err}")
    assert all(val <= 2e-5 for val in err.values()), err
