"""GPU-vs-oracle parity, through the C ABI, on the two states that pin the
traced interface states' coupling terms in the oracle (paper, Section II):

* a plasma at rest with uniform rho, p and B' = (b, 0, 0) on pencils through
  the dipole field, where one x sweep changes B'_t only through the
  time-centring of the forces B'_n dB_d/dx (both tracing modes).  Bound: the
  whole state at 1e-12 family-scaled, as every FP64 sweep; and the change of
  B'_t itself (O(dt^2), ~1e-5 of b) within 1e-8 of its largest value, since
  the two sides take the dipole's differences between faces in their own
  rounding order;
* a strong transverse shear in a low-beta plasma, where the lower bound on
  the traced total pressure is active: FP64 at 1e-12 family-scaled with
  every interface converged, and the FP32 sweep finite with positive
  pressure.
"""
import numpy as np
import pytest

import gpu_cases as GC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GAMMA = 5.0 / 3.0


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


def _pencils(n, lo, hi, h):
    # n periodic transverse zones of width h around the interval's middle
    c = 0.5 * (lo + hi)
    return c + h * (np.arange(n + 1) - 0.5 * n)


@pytest.mark.parametrize("tracing", [0, 1])
def test_time_centring_state_fp64(tracing):
    N, L, b = 80, 2.0, 0.3
    fx = np.linspace(-L, L, N + 1)
    h = fx[1] - fx[0]
    fy = _pencils(3, 0.3, 0.5, h)
    fz = _pencils(3, 1.2, 1.4, h)
    U = np.zeros((8, 3, 3, N))
    U[0] = 1.0
    U[4] = b
    U[7] = 1.0 / (GAMMA - 1.0) + 0.5 * b * b
    case = GC.Case("time-centring", [fx, fy, fz], U, bc_lo=(1, 0, 0), bc_hi=(1, 0, 0), dip_moment=2.0,
                   dip_dir=(0.0, 0.0, -1.0), tracing=tracing)
    GC.log(f"[coupling] time-centring pencils fp64 tracing={tracing}")
    ora = case.oracle()
    dt = ora.cfl_dt(U, 0.4)
    ref = ora.sweep(U, dt, 0)
    ctx = case.context()
    u = _dev(U)
    ctx.sweep(u, dt, 0)
    got = _host(u)
    err = GC.familywise_errors(got, ref)
    assert np.all(err <= 1e-12), err
    dref = ref[5:7]
    assert np.max(np.abs(dref)) > 1e-6 * b
    e = float(np.max(np.abs(got[5:7] - dref)) / np.max(np.abs(dref)))
    GC.log(f"[coupling] change of B'_t {np.max(np.abs(dref)):.3e}, GPU error {e:.2e}")
    assert e <= 1e-8, e


def _shear_case(dtype_tag):
    N, Bn, Bt, p, slope, ramp = 64, 1.0, -0.1, 1e-3, 0.25, 12
    fx = np.linspace(0.0, 1.0, N + 1)
    h = fx[1] - fx[0]
    i = np.arange(N)
    v1 = slope * np.clip(i - (N // 2 - ramp // 2), 0, ramp)
    U = np.zeros((8, 2, 2, N))
    U[0] = 1.0
    U[2] = v1
    U[4] = Bn
    U[5] = Bt
    U[7] = p / (GAMMA - 1.0) + 0.5 * v1 ** 2 + 0.5 * (Bn ** 2 + Bt ** 2)
    dt = 0.8 * h / np.sqrt(GAMMA * p + Bn ** 2 + Bt ** 2)
    faces = [fx, h * np.arange(3.0), h * np.arange(3.0)]
    return GC.Case(f"shear-{dtype_tag}", faces, U, bc_lo=(1, 0, 0), bc_hi=(1, 0, 0)), dt


def _pressure(U):
    rho, m, B = U[0], U[1:4], U[4:7]
    return (GAMMA - 1.0) * (U[7] - 0.5 * np.sum(m ** 2, 0) / rho - 0.5 * np.sum(B ** 2, 0))


def test_pressure_bound_state_fp64_and_fp32():
    case, dt = _shear_case("f64")
    GC.log("[coupling] low-beta shear fp64")
    ref = case.oracle().sweep(case.U, dt, 0)
    ctx = case.context()
    ctx.reset_stats()
    u = _dev(case.U)
    ctx.sweep(u, dt, 0)
    got = _host(u)
    err = GC.familywise_errors(got, ref)
    assert np.all(err <= 1e-12), err
    s = ctx.stats()
    assert s["nonconverged"] == 0 and s["nonphys"] == 0, s
    assert np.min(_pressure(got)) > 0.0
    GC.log("[coupling] low-beta shear fp32")
    case32, _ = _shear_case("f32")
    c32 = case32.context()
    u32 = _dev(case32.U, torch.float32)
    c32.sweep(u32, dt, 0)
    g32 = _host(u32)
    assert np.all(np.isfinite(g32)) and np.min(_pressure(g32)) > 0.0
