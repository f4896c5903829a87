"""Seeded synthetic inputs: grids, initial states and boundary states.

Both the GPU library and the CPU oracle consume these arrays; this module
holds none of the sweep's arithmetic (no reconstruction, no Riemann solve, no
remap), only the problem definitions.  Everything is NumPy/FP64 on the host.

Units are code units with mu0 = 1: length R_E, density m_p cm^-3, field nT,
velocity B0 / sqrt(mu0 rho0) = 21.81 km/s, pressure B0^2 / mu0 = 7.958e-13 Pa,
time R_E / v0 = 292.1 s.

Workloads (sizes and value distributions follow the paper's Section IV-A
set-up: stretched Cartesian grid with Earth at the origin, x sunward, y dusk,
z north, solar wind and IMF upstream, dipole obstacle):
  * ``c1``: 32^3 periodic unit box, rho = p = 1, B = (1, 0.5, 0), random
    Fourier perturbations (|k| <= 4, amplitude 1e-3) on rho, v and B, with
    div B = 0 through a vector potential; cell averages are analytic.
  * ``c2``: 256 x 192 x 192 stretched grid (0.25 .. 2 R_E, growth 1.03),
    solar-wind inflow at x_max (n = 5 cm^-3, v = -400 km/s, T = 1e5 K,
    IMF Bz = -5 nT), dipole of moment 8e15 T m^3 (30,936 nT R_E^3), fixed
    inner boundary r < 3.
  * ``c3``: every c2 cell split in two: 512 x 384 x 384.
  * ``c4``: 32 ensemble members with seeded sizes 96^3 .. 160^3 and seeded
    solar-wind inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 5.0 / 3.0

# physical constants and code units
M_P = 1.67262192e-27       # kg
K_B = 1.380649e-23         # J/K
MU0 = 4e-7 * math.pi
R_E = 6.371e6              # m
RHO0 = M_P * 1e6           # kg m^-3 (1 proton per cm^3)
B0 = 1e-9                  # T
V0 = B0 / math.sqrt(MU0 * RHO0)   # m/s
P0 = B0 * B0 / MU0         # Pa
T0 = R_E / V0              # s

# dipole: mu0 m / (4 pi) = 8e15 T m^3 -> nT R_E^3
DIPOLE_MOMENT_SI = 8e15
DIPOLE_MOMENT = DIPOLE_MOMENT_SI / (B0 * R_E ** 3)
DIPOLE_DIR = (0.0, 0.0, -1.0)   # moment points south: equatorial field northward

BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2


def solar_wind(n_cc: float, v_kms: float, T_K: float, bz_nT: float, bx_nT=0.0, by_nT=0.0):
    """Primitive solar-wind state (rho, vx, vy, vz, Bx, By, Bz, p) in code
    units; the wind moves toward -x (x points at the Sun)."""
    rho = n_cc
    vx = -abs(v_kms) * 1e3 / V0
    p = n_cc * 1e6 * K_B * T_K / P0
    return np.array([rho, vx, 0.0, 0.0, bx_nT, by_nT, bz_nT, p], dtype=np.float64)


def solar_wind_series(t_end: float, n_knots: int = 9, seed: int = 11):
    """Seeded synthetic upstream time series (no measured solar-wind data is
    available here): n_knots equally spaced knots on [0, t_end] (code time
    units) with n ~ logU[3, 10] cm^-3, v ~ U[350, 550] km/s, T = 1e5 K,
    Bz ~ U[-10, 5] nT, By ~ U[-3, 3] nT.  Returns (times, prims[n, 8])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    times = np.linspace(0.0, t_end, n_knots)
    n = np.exp(rng.uniform(math.log(3.0), math.log(10.0), n_knots))
    v = rng.uniform(350.0, 550.0, n_knots)
    bz = rng.uniform(-10.0, 5.0, n_knots)
    by = rng.uniform(-3.0, 3.0, n_knots)
    prims = np.stack([solar_wind(float(n[k]), float(v[k]), 1e5, float(bz[k]), by_nT=float(by[k]))
                      for k in range(n_knots)])
    return times, prims


# ----------------------------------------------------------------- grids

def uniform_faces(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return np.linspace(lo, hi, n + 1, dtype=np.float64)


def stretched_half_axis(count: int, w_min=0.25, growth=1.03, w_max=2.0, core=16) -> np.ndarray:
    """Widths outward from the origin: `core` cells of w_min, then
    w_k = min(w_max, w_min * growth**(k - core + 1))."""
    k = np.arange(count)
    w = np.where(k < core, w_min, np.minimum(w_max, w_min * growth ** (k - core + 1.0)))
    return w.astype(np.float64)


def stretched_faces(n_neg: int, n_pos: int, **kw) -> np.ndarray:
    wn = stretched_half_axis(n_neg, **kw)
    wp = stretched_half_axis(n_pos, **kw)
    neg = -np.cumsum(wn)[::-1]
    pos = np.cumsum(wp)
    return np.concatenate([neg, [0.0], pos]).astype(np.float64)


def split_faces(f: np.ndarray) -> np.ndarray:
    """Split every cell in two (same domain, half widths)."""
    mid = 0.5 * (f[:-1] + f[1:])
    out = np.empty(2 * len(f) - 1)
    out[0::2] = f
    out[1::2] = mid
    return out


def c2_faces():
    fx = stretched_faces(192, 64)
    fy = stretched_faces(96, 96)
    fz = stretched_faces(96, 96)
    return [fx, fy, fz]


def c3_faces():
    return [split_faces(f) for f in c2_faces()]


def member_faces(N: int):
    """Coarsened c2 rule for an N^3 ensemble member: x gets N/4 cells sunward
    and 3N/4 tailward, y and z N/2 per side; widths scale with 192/N."""
    s = 192.0 / N
    core = int(round(N / 12))
    kw = dict(w_min=0.25 * s, w_max=2.0 * s, growth=1.03, core=core)
    fx = stretched_faces(3 * N // 4, N // 4, **kw)
    fy = stretched_faces(N // 2, N // 2, **kw)
    fz = stretched_faces(N // 2, N // 2, **kw)
    return [fx, fy, fz]


def centres(f: np.ndarray) -> np.ndarray:
    return 0.5 * (f[:-1] + f[1:])


# ---------------------------------------------------------------- states

def conserved(rho, vx, vy, vz, bx, by, bz, p, gamma=GAMMA) -> np.ndarray:
    """Conserved SoA array [8, nz, ny, nx] from primitive fields (B is B')."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast(rho, vx, vy, vz, bx, by, bz, p).shape
    U = np.empty((8,) + shape, dtype=np.float64)
    U[0] = rho
    U[1] = rho * vx
    U[2] = rho * vy
    U[3] = rho * vz
    U[4] = bx
    U[5] = by
    U[6] = bz
    U[7] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bx * bx + by * by + bz * bz)
    return U


def uniform_state(shape, rho=1.0, v=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0), p=1.0, gamma=GAMMA):
    z = np.zeros(shape)
    return conserved(rho + z, v[0] + z, v[1] + z, v[2] + z, B[0] + z, B[1] + z, B[2] + z, p + z, gamma)


def _fourier_modes(kmax: int):
    r = range(-kmax, kmax + 1)
    modes = [(a, b, c) for a in r for b in r for c in r if 0 < a * a + b * b + c * c <= kmax * kmax]
    return np.array(modes, dtype=np.float64)


def c1_state(n: int = 32, seed: int = 1607, amp: float = 1e-3, kmax: int = 4,
             B0vec=(1.0, 0.5, 0.0), gamma=GAMMA):
    """Periodic unit box with random Fourier perturbations; returns (U, faces).

    Each mode n in Z^3, 0 < |n| <= kmax, has one random amplitude and phase
    per field (PCG64).  Cell averages of sin(2 pi n.x + phi) are the centre
    values times prod_d sinc(pi n_d dx); B = B0 + curl A with A from the same
    modes, so the cell-averaged B is the exact average of a solenoidal field.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = _fourier_modes(kmax)
    nm = len(modes)
    f = uniform_faces(n)
    xc = centres(f)
    dx = 1.0 / n
    X = xc[None, None, :]
    Y = xc[None, :, None]
    Z = xc[:, None, None]
    # sinc factor of each mode for cell averages (np.sinc(x) = sin(pi x)/(pi x))
    sinc = np.sinc(modes[:, 0] * dx) * np.sinc(modes[:, 1] * dx) * np.sinc(modes[:, 2] * dx)

    def field_from(amps, phases, deriv=None):
        out = np.zeros((n, n, n))
        for m in range(nm):
            kx, ky, kz = modes[m]
            arg = 2 * np.pi * (kx * X + ky * Y + kz * Z) + phases[m]
            if deriv is None:
                out += amps[m] * sinc[m] * np.sin(arg)
            else:
                out += amps[m] * sinc[m] * 2 * np.pi * modes[m][deriv] * np.cos(arg)
        return out

    pert = {}
    for name in ("rho", "vx", "vy", "vz"):
        a = rng.uniform(-1.0, 1.0, nm)
        ph = rng.uniform(0.0, 2 * np.pi, nm)
        fld = field_from(a, ph)
        pert[name] = fld * (amp / np.max(np.abs(fld)))
    Aa = [rng.uniform(-1.0, 1.0, nm) for _ in range(3)]
    Ap = [rng.uniform(0.0, 2 * np.pi, nm) for _ in range(3)]
    # curl A: Bx = dAz/dy - dAy/dz, By = dAx/dz - dAz/dx, Bz = dAy/dx - dAx/dy
    dB = [field_from(Aa[2], Ap[2], 1) - field_from(Aa[1], Ap[1], 2),
          field_from(Aa[0], Ap[0], 2) - field_from(Aa[2], Ap[2], 0),
          field_from(Aa[1], Ap[1], 0) - field_from(Aa[0], Ap[0], 1)]
    s = amp / max(np.max(np.abs(c)) for c in dB)
    dB = [c * s for c in dB]
    rho = 1.0 + pert["rho"]
    U = conserved(rho, pert["vx"], pert["vy"], pert["vz"],
                  B0vec[0] + dB[0], B0vec[1] + dB[1], B0vec[2] + dB[2], 1.0 + 0.0 * rho, gamma)
    return U, [f, f.copy(), f.copy()]


def dipole_point(xyz, moment=DIPOLE_MOMENT, direction=DIPOLE_DIR, origin=(0.0, 0.0, 0.0)):
    """Point-dipole field (used only to build initial and inflow states)."""
    x = xyz[0] - origin[0]
    y = xyz[1] - origin[1]
    z = xyz[2] - origin[2]
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    mr = direction[0] * x + direction[1] * y + direction[2] * z
    r3 = r2 * r
    r5 = r3 * r2
    return [moment * (3 * mr * c / r5 - d / r3) for c, d in zip((x, y, z), direction)]


@dataclass
class DipoleSetup:
    faces: list
    U: np.ndarray
    inflow: np.ndarray                    # primitive, total B
    r_inner: float = 3.0
    inner_rho: float = 5.0
    inner_p: float = 0.0
    bc_lo: tuple = (BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW)
    bc_hi: tuple = (BC_INFLOW, BC_OUTFLOW, BC_OUTFLOW)
    moment: float = DIPOLE_MOMENT
    direction: tuple = DIPOLE_DIR
    p_floor: float = 0.0
    meta: dict = field(default_factory=dict)


def dipole_initial_state(faces, sw, x_switch=15.0, r_inner=3.0, image_x=30.0, gamma=GAMMA,
                         dtype=np.float64) -> np.ndarray:
    """Section IV-A style start: for x <= 15 the deviation field is that of an
    image dipole at (30, 0, 0) and the plasma is at rest with solar-wind
    density and pressure; for x > 15 uniform solar wind and IMF (B' = IMF -
    B_d); inside r < r_inner the fixed inner state (rest, B' = 0)."""
    xc, yc, zc = (centres(f) for f in faces)
    nz, ny, nx = len(zc), len(yc), len(xc)
    U = np.empty((8, nz, ny, nx), dtype=dtype)
    Y2, X2 = np.meshgrid(yc, xc, indexing="ij")
    rho, vx, p = sw[0], sw[1], sw[7]
    imf = sw[4:7]
    for k in range(nz):   # slab by slab to bound memory on large grids
        Z2 = np.full_like(X2, zc[k])
        bd = dipole_point((X2, Y2, Z2))
        bi = dipole_point((X2, Y2, Z2), origin=(image_x, 0.0, 0.0))
        up = X2 > x_switch
        bxp = np.where(up, imf[0] - bd[0], bi[0])
        byp = np.where(up, imf[1] - bd[1], bi[1])
        bzp = np.where(up, imf[2] - bd[2], bi[2])
        vxx = np.where(up, vx, 0.0)
        r = np.sqrt(X2 * X2 + Y2 * Y2 + Z2 * Z2)
        inner = r < r_inner
        bxp = np.where(inner, 0.0, bxp)
        byp = np.where(inner, 0.0, byp)
        bzp = np.where(inner, 0.0, bzp)
        vxx = np.where(inner, 0.0, vxx)
        slab = conserved(rho + 0 * X2, vxx, 0 * X2, 0 * X2, bxp, byp, bzp, p + 0 * X2, gamma)
        U[:, k] = slab.astype(dtype)
    return U


def c2_setup(faces=None, dtype=np.float64) -> DipoleSetup:
    faces = faces if faces is not None else c2_faces()
    sw = solar_wind(5.0, 400.0, 1e5, -5.0)
    U = dipole_initial_state(faces, sw, dtype=dtype)
    return DipoleSetup(faces=faces, U=U, inflow=sw, inner_rho=sw[0], inner_p=sw[7],
                       p_floor=1e-8 * sw[7],
                       meta={"workload": "inflow-dipole", "n": [len(f) - 1 for f in faces]})


def c3_setup(dtype=np.float32) -> DipoleSetup:
    return c2_setup(c3_faces(), dtype=dtype)


def ensemble_members(count: int = 32, seed: int = 4):
    """Seeded sizes N in {96, 104, ..., 160} and solar-wind inputs:
    v ~ U[300, 800] km/s, n ~ logU[1, 20] cm^-3, Bz ~ U[-20, 10] nT,
    T = 1e5 K, Bx = By = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.choice(np.arange(96, 161, 8), size=count)
    v = rng.uniform(300.0, 800.0, count)
    n = np.exp(rng.uniform(math.log(1.0), math.log(20.0), count))
    bz = rng.uniform(-20.0, 10.0, count)
    out = []
    for m in range(count):
        sw = solar_wind(float(n[m]), float(v[m]), 1e5, float(bz[m]))
        out.append({"N": int(sizes[m]), "sw": sw})
    return out


def random_smooth_state(shape, seed=0, amp=0.2, B0vec=(0.8, -0.4, 0.3), rho0=1.0, p0=1.0, gamma=GAMMA):
    """Smooth random state with O(amp) variations (parity tests that exercise
    every branch of the limiter and the Newton iteration)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) / max(nz, 1), np.arange(ny) / max(ny, 1),
                          np.arange(nx) / max(nx, 1), indexing="ij")

    def smooth():
        out = np.zeros(shape)
        for _ in range(4):
            k = rng.integers(1, 4, 3)
            ph = rng.uniform(0, 2 * np.pi)
            out += rng.uniform(-1, 1) * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return out / 4.0

    rho = rho0 * (1.0 + amp * smooth())
    p = p0 * (1.0 + amp * smooth())
    v = [amp * smooth() for _ in range(3)]
    B = [B0vec[i] + amp * smooth() for i in range(3)]
    return conserved(rho, v[0], v[1], v[2], B[0], B[1], B[2], p, gamma)


def blast_state(faces, seed=0, gamma=GAMMA, B0vec=(0.5, 0.3, -0.2)):
    """Off-centre overpressure sphere: strong shocks in every direction
    (exercises flattening and multi-iteration Newton solves)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xc, yc, zc = (centres(f) for f in faces)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    c = [rng.uniform(f[0] + 0.3 * (f[-1] - f[0]), f[-1] - 0.3 * (f[-1] - f[0])) for f in faces]
    L = min(f[-1] - f[0] for f in faces)
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    inside = r < 0.2 * L
    p = np.where(inside, 20.0, 1.0)
    rho = np.where(inside, 2.0, 1.0)
    z0 = 0 * X
    return conserved(rho, z0, z0, z0, B0vec[0] + z0, B0vec[1] + z0, B0vec[2] + z0, p, gamma)


# ---------------------------------------------------------------------------
# Learned Riemann guess: initial parameters and synthetic samples

MLP_SHAPES = ((14, 64), (64,), (64, 64), (64,), (64, 2), (2,))


def mlp_init(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Initial parameters of the 14-64-64-2 network as one FP32 vector
    (W1, b1, W2, b2, W3, b3, row-major, input index first): weights drawn
    uniformly on +-scale*sqrt(6 / (fan_in + fan_out)) (Glorot & Bengio 2010),
    biases zero.  PCG64(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            lim = scale * np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def mlp_samples(n: int, seed: int = 0, spread: float = 1.0):
    """n synthetic network inputs of the guess's feature ranges: densities and
    pressures near 1 (ratios up to e^spread), velocities and fields O(spread)."""
    rng = np.random.default_rng(seed)
    X = np.empty((n, 14), dtype=np.float32)
    for base in (0, 7):
        X[:, base + 0] = np.exp(rng.uniform(-spread, spread, n))
        X[:, base + 1:base + 4] = rng.normal(0.0, 0.5 * spread, (n, 3))
        X[:, base + 4:base + 6] = rng.normal(0.0, 0.5 * spread, (n, 2))
        X[:, base + 6] = np.exp(rng.uniform(-spread, spread, n))
    return X
