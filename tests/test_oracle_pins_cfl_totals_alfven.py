"""Pins of oracle functions that the scheme-level pins do not reach.

* `cfl_dt` (the split step's time step: dt = CFL / max over unmasked zones
  of max_a (|v_a| + c_f,a) / dx_a with the total field) against the largest
  eigenvalue magnitude of the 1D ideal-MHD Jacobian along each axis, taken
  numerically with `numpy.linalg.eigvals`, on anisotropic states on
  stretched grids, with a background field and an inner mask;
* `totals` (volume integrals of the conserved variables) against closed-form
  integrals of uniform and linear fields on stretched grids (cell averages of
  a linear field are its centre values);
* the transverse (Alfven) Riemann pair with unequal densities on the two
  sides, against the star state solved from the two-medium jump conditions
  (continuous v_t and B_t, the outgoing characteristic invariant carried
  across each wave) as a 2x2 linear system;
* the factor 2 of the CW84 Eq. 1.8 limiter: where the limiter clips, the
  zone's linear profile a_j -+ da_j/2 reaches the neighbouring average
  exactly.
Test infrastructure only; every expected value below is computed here from
the mathematics, not from the oracle's own formulas.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_02214_amd import inputs as I

import oracle_cases as OC

G = 5.0 / 3.0


def _stretched(n, lo, hi, rng):
    w = rng.uniform(0.4, 1.6, n)
    f = np.concatenate([[0.0], np.cumsum(w)])
    return lo + (hi - lo) * f / f[-1]


def _random_state(shape, rng, vscale=(3.0, 1.0, 2.0), bscale=(0.5, 1.5, 1.0)):
    nz, ny, nx = shape
    rho = rng.uniform(0.5, 2.0, shape)
    v = [rng.uniform(-s, s, shape) for s in vscale]
    b = [rng.uniform(-s, s, shape) for s in bscale]
    p = rng.uniform(0.2, 2.0, shape)
    U = I.conserved(rho, v[0], v[1], v[2], b[0], b[1], b[2], p, G)
    return U.reshape((8,) + shape), rho, v, b, p


def _fast_speeds(rho, p, B, gamma=G):
    """Per zone and axis: the largest |eigenvalue| of the primitive MHD
    Jacobian with the normal field B[a] (rho, p, B flattened arrays)."""
    out = np.zeros((3, rho.size))
    for a in range(3):
        A = np.stack([OC.mhd_jacobian(r, q, B[a][k], B[(a + 1) % 3][k], B[(a + 2) % 3][k], gamma)
                      for k, (r, q) in enumerate(zip(rho, p))])
        out[a] = np.max(np.abs(np.linalg.eigvals(A).real), axis=1)
    return out


def _expected_dt(faces, rho, v, bprime, p, Bd, cfl, r_inner):
    nz, ny, nx = rho.shape
    w = [np.diff(f) for f in faces]
    c = [0.5 * (f[1:] + f[:-1]) for f in faces]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    WZ, WY, WX = np.meshgrid(w[2], w[1], w[0], indexing="ij")
    B = [(bprime[a] + Bd[a]).ravel() for a in range(3)]
    cf = _fast_speeds(rho.ravel(), p.ravel(), B)
    widths = [WX.ravel(), WY.ravel(), WZ.ravel()]
    s = np.max(np.stack([(np.abs(v[a].ravel()) + cf[a]) / widths[a] for a in range(3)]), axis=0)
    keep = np.sqrt(X.ravel() ** 2 + Y.ravel() ** 2 + Z.ravel() ** 2) >= r_inner if r_inner > 0 else np.ones(s.size, bool)
    return cfl / np.max(s[keep]), s, keep


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cfl_dt_matches_jacobian_fast_speeds_on_stretched_grid(seed):
    rng = np.random.default_rng(100 + seed)
    shape = (7, 8, 9)
    faces = [_stretched(9, -4.0, 5.0, rng), _stretched(8, -3.0, 3.5, rng), _stretched(7, -2.5, 4.0, rng)]
    U, rho, v, b, p = _random_state(shape, rng)
    bext = (0.7, -1.1, 0.4)
    prob = O.OracleProblem(faces, bext=bext)
    dt = prob.cfl_dt(U, 0.4)
    Bd = [np.full(shape, x) for x in bext]
    want, _, _ = _expected_dt(faces, rho, v, b, p, Bd, 0.4, 0.0)
    assert abs(dt - want) <= 1e-12 * want, (dt, want)


def test_cfl_dt_excludes_masked_zones_and_uses_total_field():
    rng = np.random.default_rng(7)
    shape = (8, 8, 8)
    faces = [_stretched(8, -4.0, 4.5, rng), _stretched(8, -4.2, 4.0, rng), _stretched(8, -3.8, 4.1, rng)]
    U, rho, v, b, p = _random_state(shape, rng)
    c = [0.5 * (f[1:] + f[:-1]) for f in faces]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    r_in = 2.0
    inside = r < r_in
    assert inside.any() and (~inside).any()
    # the fastest zone of the whole box sits inside the mask
    v0 = v[0].copy()
    v0[inside] = 50.0
    U = I.conserved(rho, v0, v[1], v[2], b[0], b[1], b[2], p, G).reshape((8,) + shape)
    moment, mdir = 3.0, (0.2, -0.3, -0.93)
    prob = O.OracleProblem(faces, dip_moment=moment, dip_dir=mdir, r_inner=r_in)
    dt = prob.cfl_dt(U, 0.4)
    Bd = np.zeros((3,) + shape)
    for idx in np.ndindex(shape):
        Bd[(slice(None),) + idx] = prob.dipole(np.array([X[idx], Y[idx], Z[idx]]))
    want, s, keep = _expected_dt(faces, rho, [v0, v[1], v[2]], b, p, Bd, 0.4, r_in)
    assert abs(dt - want) <= 1e-12 * want, (dt, want)
    # a reading that ignored the mask or the background field would differ
    assert 0.4 / np.max(s) < 0.5 * want
    alt, _, _ = _expected_dt(faces, rho, [v0, v[1], v[2]], b, p, np.zeros_like(Bd), 0.4, r_in)
    assert abs(alt - want) > 1e-3 * want


def test_cfl_dt_fast_speed_depends_on_direction():
    # strong field along x: the fast speed along x is max(a, b_x) and across
    # it sqrt(a^2 + b^2); widths differ per axis so that a mixed-up axis
    # changes the answer
    shape = (3, 4, 5)
    faces = [np.linspace(0, 5 * 0.3, 6), np.linspace(0, 4 * 0.7, 5), np.linspace(0, 3 * 1.1, 4)]
    rho, p = np.full(shape, 1.3), np.full(shape, 0.2)
    zero = np.zeros(shape)
    U = I.conserved(rho, zero + 0.4, zero - 0.1, zero + 0.25, zero + 3.0, zero + 0.5, zero, p, G).reshape((8,) + shape)
    prob = O.OracleProblem(faces)
    dt = prob.cfl_dt(U, 0.8)
    a2, bx2, b2 = G * 0.2 / 1.3, 9.0 / 1.3, 9.25 / 1.3
    cfx = np.sqrt(0.5 * (a2 + b2 + np.sqrt((a2 + b2) ** 2 - 4 * a2 * bx2)))
    cfy = np.sqrt(0.5 * (a2 + b2 + np.sqrt((a2 + b2) ** 2 - 4 * a2 * 0.25 / 1.3)))
    cfz = np.sqrt(a2 + b2)
    s = max((0.4 + cfx) / 0.3, (0.1 + cfy) / 0.7, (0.25 + cfz) / 1.1)
    assert abs(dt - 0.8 / s) <= 1e-13 * dt
    lam = _fast_speeds(np.array([1.3]), np.array([0.2]), [np.array([3.0]), np.array([0.5]), np.array([0.0])])
    assert np.allclose(lam[:, 0], [cfx, cfy, cfz], rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_totals_are_volume_integrals_of_linear_fields_on_stretched_grids(seed):
    rng = np.random.default_rng(300 + seed)
    faces = [_stretched(11, -3.0, 7.0, rng), _stretched(6, -1.0, 2.0, rng), _stretched(9, 0.5, 4.5, rng)]
    c = [0.5 * (f[1:] + f[:-1]) for f in faces]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    a = rng.uniform(-2, 2, 8)
    b = rng.uniform(-1, 1, (8, 3))
    U = np.stack([a[v] + b[v, 0] * X + b[v, 1] * Y + b[v, 2] * Z for v in range(8)])
    got = O.OracleProblem(faces).totals(U)
    (x0, x1), (y0, y1), (z0, z1) = [(f[0], f[-1]) for f in faces]
    V = (x1 - x0) * (y1 - y0) * (z1 - z0)
    ix = 0.5 * (x1 ** 2 - x0 ** 2) * (y1 - y0) * (z1 - z0)
    iy = 0.5 * (y1 ** 2 - y0 ** 2) * (x1 - x0) * (z1 - z0)
    iz = 0.5 * (z1 ** 2 - z0 ** 2) * (x1 - x0) * (y1 - y0)
    want = a * V + b[:, 0] * ix + b[:, 1] * iy + b[:, 2] * iz
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * V)


def test_totals_of_uniform_state_are_value_times_volume():
    rng = np.random.default_rng(9)
    faces = [_stretched(5, 0.0, 2.0, rng), _stretched(7, -1.0, 1.0, rng), _stretched(4, 3.0, 3.5, rng)]
    vals = rng.uniform(-3, 3, 8)
    U = np.broadcast_to(vals[:, None, None, None], (8, 4, 7, 5)).copy()
    got = O.OracleProblem(faces).totals(U)
    V = 2.0 * 2.0 * 0.5
    assert np.allclose(got, vals * V, rtol=1e-14)


def _alfven_star_from_jump_conditions(rhoL, rhoR, sigma, vL, vR, bL, bR):
    """v*, b* with v and b continuous at the contact; across the left-moving
    wave (in the left medium) the right-moving invariant v - sigma b / sqrt(rho_L)
    is unchanged, across the right-moving wave the left-moving invariant
    v + sigma b / sqrt(rho_R)."""
    rL, rR = np.sqrt(rhoL), np.sqrt(rhoR)
    A = np.array([[1.0, -sigma / rL], [1.0, sigma / rR]])
    rhs = np.array([vL - sigma * bL / rL, vR + sigma * bR / rR])
    return np.linalg.solve(A, rhs)


@pytest.mark.parametrize("seed", range(4))
def test_alfven_pair_with_unequal_densities_matches_jump_conditions(seed):
    rng = np.random.default_rng(400 + seed)
    for _ in range(50):
        rhoL = 10 ** rng.uniform(-1, 1)
        rhoR = 10 ** rng.uniform(-1, 1)
        sigma = rng.choice([-1.0, 1.0])
        vL, vR, bL, bR = rng.uniform(-2, 2, 4)
        want = _alfven_star_from_jump_conditions(rhoL, rhoR, sigma, vL, vR, bL, bR)
        got = O.riemann_alfven(np.sqrt(rhoL), np.sqrt(rhoR), sigma, vL, vR, bL, bR)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12), (rhoL, rhoR, sigma, got, want)


def test_alfven_pair_star_state_is_the_evolved_linear_solution():
    # the same star state from a direct evolution of the linear two-medium
    # system d_t v = B_n d_m b, d_t b = rho B_n d_m v (upwind characteristic
    # solver on a fine mass grid; the interface zone holds the star state)
    rhoL, rhoR, Bn = 4.0, 0.25, -1.3
    vL, vR, bL, bR = 0.3, -0.7, 1.1, -0.4
    sigma = np.sign(Bn)
    n = 400
    rho = np.where(np.arange(2 * n) < n, rhoL, rhoR)
    c = np.sqrt(rho) * abs(Bn)                       # Lagrangian wave speeds
    v = np.where(np.arange(2 * n) < n, vL, vR).astype(float)
    b = np.where(np.arange(2 * n) < n, bL, bR).astype(float)
    dm = 1.0
    dt = 0.4 * dm / c.max()
    for _ in range(200):
        # characteristic variables w+- = v -+ sigma b / sqrt(rho) travel at +-c;
        # at a face the upwind values of each invariant fix (v, b) there
        wp = v - sigma * b / np.sqrt(rho)
        wm = v + sigma * b / np.sqrt(rho)
        vf = np.empty(2 * n + 1)
        bf = np.empty(2 * n + 1)
        rl, rr = np.sqrt(rho[:-1]), np.sqrt(rho[1:])
        A11, A12, A21, A22 = 1.0, -sigma / rl, 1.0, sigma / rr
        det = A11 * A22 - A12 * A21
        vf[1:-1] = (A22 * wp[:-1] - A12 * wm[1:]) / det
        bf[1:-1] = (-A21 * wp[:-1] + A11 * wm[1:]) / det
        vf[0], bf[0], vf[-1], bf[-1] = v[0], b[0], v[-1], b[-1]
        v = v + dt / dm * Bn * (bf[1:] - bf[:-1])
        b = b + dt / dm * rho * Bn * (vf[1:] - vf[:-1])
    got = O.riemann_alfven(np.sqrt(rhoL), np.sqrt(rhoR), sigma, vL, vR, bL, bR)
    assert abs(vf[n] - got[0]) < 1e-10 and abs(bf[n] - got[1]) < 1e-10, (vf[n], bf[n], got)


@pytest.mark.parametrize("seed", range(4))
def test_limiter_clip_reaches_the_neighbouring_average(seed):
    rng = np.random.default_rng(500 + seed)
    for _ in range(40):
        w = rng.uniform(0.3, 3.0, 3)
        s = rng.choice([-1.0, 1.0])
        base = rng.uniform(-1, 1)
        small, big = rng.uniform(0.01, 0.05), rng.uniform(0.8, 1.2)
        # clip on the left difference: a_0 -> a_1 small step, a_1 -> a_2 big
        a = base + s * np.array([0.0, small, small + big])
        da = O.ppm_slopes(a, w, limit=True)[1]
        assert abs((a[1] - 0.5 * da) - a[0]) <= 1e-14 * (1 + abs(a[0])), (a, w, da)
        # clip on the right difference
        a = base + s * np.array([0.0, big, big + small])
        da = O.ppm_slopes(a, w, limit=True)[1]
        assert abs((a[1] + 0.5 * da) - a[2]) <= 1e-14 * (1 + abs(a[2])), (a, w, da)
        # no clip when both one-sided differences are comparable: the
        # unlimited Eq. 1.7 slope is kept
        a = base + s * np.array([0.0, 1.0, 2.0 + rng.uniform(-0.2, 0.2)])
        assert O.ppm_slopes(a, w, limit=True)[1] == O.ppm_slopes(a, w, limit=False)[1]
