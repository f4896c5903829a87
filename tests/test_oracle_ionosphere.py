"""Pins of the oracle's ionosphere coupling (paper, Section II: the shell at
1.017 R_E, its electrostatic potential, the mapping along dipole field lines
to the inner boundary), against what the mathematics fixes:
- the potential of a uniform radial current on a cap against its closed
  form, 2 kappa ln(cos(theta_c / 2) / cos(theta / 2)), converging at second
  order;
- a potential ~ cos(phi) against the exact operator applied to it
  (manufactured solution), second order;
- discrete conservation: the current into the cap equals the flux through
  its edge;
- the field-aligned current of a uniform current density J = alpha z
  (B' = alpha (-y, x, 0) / 2, exact under central differences), mapped to
  the shell, against the dipole written in spherical components;
- the mapped points lie on dipole field lines (field line integrated with
  RK4 from the shell cell to r_fac);
- the drift of an axisymmetric potential is azimuthal with the magnitude
  of the analytic E x B;
- the sweep's inner reset takes the drift: reset zones hold rho v and the
  kinetic energy."""
import math

import numpy as np
import pytest

from oracle import ionosphere as IO
from oracle import oracle as O
from paper_1607_02214_amd import inputs as I

G = 5.0 / 3.0


def _cap_error(n_theta, jr_fn, exact_fn, n_phi=16, sigma=0.7):
    grid = IO.ShellGrid(n_theta, n_phi, r_shell=1.017, r_fac=3.0)
    TH, PH = np.meshgrid(grid.th, grid.ph, indexing="ij")
    jr = np.stack([jr_fn(grid, TH, PH)] * 2)
    phi = IO.solve_potential(grid, jr, sigma)
    ex = exact_fn(grid, TH, PH, sigma)
    return max(float(np.max(np.abs(phi[h] - ex))) for h in range(2)) / float(np.max(np.abs(ex))), grid, phi, jr


def test_uniform_current_closed_form_second_order():
    c = -0.3

    def jr_fn(grid, TH, PH):
        return c + 0.0 * TH

    def exact(grid, TH, PH, sigma):
        kappa = c * grid.r_shell ** 2 / sigma
        return 2.0 * kappa * np.log(math.cos(grid.theta_c / 2.0) / np.cos(TH / 2.0))

    errs = [_cap_error(n, jr_fn, exact)[0] for n in (8, 16, 32)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 2e-3 and np.all(orders > 1.8), (errs, orders)


def test_manufactured_cos_phi_second_order():
    # Phi = f(theta) cos(phi), f = sin(theta) (cos(theta) - cos(theta_c)):
    # zero on the edge, regular at the pole; the operator in closed form
    def f(tc, t):
        return np.sin(t) * (np.cos(t) - math.cos(tc))

    def lap(tc, t):
        fp = np.cos(2 * t) - math.cos(tc) * np.cos(t)
        fpp = -2.0 * np.sin(2 * t) + math.cos(tc) * np.sin(t)
        return (np.cos(t) * fp + np.sin(t) * fpp) / np.sin(t) - f(tc, t) / np.sin(t) ** 2

    def jr_fn(grid, TH, PH):
        return 0.7 * lap(grid.theta_c, TH) * np.cos(PH) / grid.r_shell ** 2

    def exact(grid, TH, PH, sigma):
        return f(grid.theta_c, TH) * np.cos(PH)

    errs = [_cap_error(n, jr_fn, exact, n_phi=4 * n)[0] for n in (8, 16, 32)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 5e-3 and np.all(orders > 1.8), (errs, orders)


def test_current_into_the_cap_leaves_through_its_edge():
    rng = np.random.default_rng(3)
    grid = IO.ShellGrid(12, 20, r_shell=1.017, r_fac=3.5)
    jr = rng.standard_normal((2, 12, 20))
    sigma = 0.4
    phi = IO.solve_potential(grid, jr, sigma)
    for h in range(2):
        into = sum(float(np.sum(jr[h, k])) * grid.area(k) for k in range(12))
        edge = sigma * math.sin(grid.theta_c) * grid.dph * float(np.sum(0.0 - phi[h, -1])) / (0.5 * grid.dth)
        assert abs(into - edge) <= 1e-10 * max(1.0, abs(into)), (into, edge)


def _box_grid(n=20, L=6.0, seed=1):
    rng = np.random.default_rng(seed)
    faces = []
    for _ in range(3):
        w = rng.uniform(0.8, 1.2, n)
        f = np.concatenate([[0.0], np.cumsum(w)])
        faces.append(-L + 2 * L * f / f[-1])
    return faces


def test_fac_of_a_uniform_current_maps_as_the_dipole_fixes():
    alpha, M = 0.02, 30.0
    faces = _box_grid(n=22, L=5.0)
    xc, yc, zc = IO.centres(faces)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    U = np.zeros((8, len(zc), len(yc), len(xc)))
    U[4] = -0.5 * alpha * Y
    U[5] = 0.5 * alpha * X
    grid = IO.ShellGrid(6, 8, r_shell=1.017, r_fac=3.5)
    jr = IO.shell_current(faces, U, M, (0.0, 0.0, -1.0), grid)
    # dipole of moment M along -z in spherical components: B_r = -2 M cos / r^3,
    # B_theta = -M sin / r^3 (theta from +z); J = alpha z: J_r = alpha cos,
    # J_theta = -alpha sin
    for h in range(2):
        for k in range(6):
            th_s = grid.th[k] if h == 0 else math.pi - grid.th[k]
            s_f = math.sin(grid.th[k]) * math.sqrt(3.5 / 1.017)
            th_f = math.asin(s_f) if h == 0 else math.pi - math.asin(s_f)

            def bsph(r, t):
                return np.array([-2 * M * math.cos(t) / r ** 3, -M * math.sin(t) / r ** 3])

            bf, bs = bsph(3.5, th_f), bsph(1.017, th_s)
            jpar = float(np.dot([alpha * math.cos(th_f), -alpha * math.sin(th_f)], bf)) / np.linalg.norm(bf)
            want = jpar * np.linalg.norm(bs) / np.linalg.norm(bf) * bs[0] / np.linalg.norm(bs)
            assert np.allclose(jr[h, k], want, rtol=1e-10, atol=1e-14), (h, k, jr[h, k], want)


def test_mapped_points_lie_on_dipole_field_lines():
    M, mdir = 30.0, (0.2, -0.1, -1.0)
    frame = IO.magnetic_frame(mdir)
    grid = IO.ShellGrid(5, 7, r_shell=1.017, r_fac=3.5)

    def rhs(p):
        b = IO.dipole(M, mdir, p)
        return b / np.linalg.norm(b)

    for h in range(2):
        for k in range(5):
            for j in (0, 3, 6):
                p = grid.r_shell * grid.shell_point(frame, h, k, j)
                target = grid.fac_point(frame, h, k, j)
                # integrate along the field line (either direction) until r = r_fac
                sgn = 1.0 if np.dot(IO.dipole(M, mdir, p), p) > 0 else -1.0
                ds = 1e-3
                while np.linalg.norm(p) < grid.r_fac:
                    k1 = rhs(p)
                    k2 = rhs(p + 0.5 * ds * sgn * k1)
                    k3 = rhs(p + 0.5 * ds * sgn * k2)
                    k4 = rhs(p + ds * sgn * k3)
                    q = p + ds * sgn * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
                    if np.linalg.norm(q) >= grid.r_fac:
                        # last partial step to the sphere (linear in the step)
                        a = (grid.r_fac - np.linalg.norm(p)) / (np.linalg.norm(q) - np.linalg.norm(p))
                        q = p + a * (q - p)
                    p = q
                assert np.linalg.norm(p - target) < 1e-5, (h, k, j, p, target)


def _drift_error(n, M=30.0, cs=(-0.2, 0.35), sigma=0.5):
    # a different uniform current on each cap (north cs[0], south cs[1])
    faces = [np.linspace(-4.0, 4.0, n + 1)] * 3
    grid = IO.ShellGrid(64, 16, r_shell=1.017, r_fac=3.5)
    jr = np.stack([np.full((64, 16), cs[0]), np.full((64, 16), cs[1])])
    phi = IO.solve_potential(grid, jr, sigma)
    box, v = IO.inner_drift(faces, 3.0, M, (0.0, 0.0, -1.0), grid, phi)
    xc = IO.centres(faces)[0]
    i0, i1, j0, j1, k0, k1 = box
    worst, radial, checked = 0.0, 0.0, 0
    for k in range(k0, k1):
        for j in range(j0, j1):
            for i in range(i0, i1):
                pos = np.array([xc[i], xc[j], xc[k]])
                r = np.linalg.norm(pos)
                if r >= 3.0 or r < 2.0 or abs(pos[2]) < 0.5:
                    continue
                t = math.acos(pos[2] / r)
                s2s = (1.017 / r) * math.sin(t) ** 2
                if s2s > 0.8 * math.sin(grid.theta_c) ** 2:
                    continue
                ts = math.asin(math.sqrt(s2s))
                kappa = cs[0 if pos[2] > 0 else 1] * grid.r_shell ** 2 / sigma
                dphi_dts = kappa * math.tan(ts / 2.0)
                # (in the south cos t < 0: theta_s, counted from the south
                # pole, falls as t grows)
                dts_dt = math.sqrt(1.017 / r) * math.cos(t) / math.cos(ts)
                dts_dr = -0.5 * math.sqrt(1.017 / r) * math.sin(t) / (r * math.cos(ts))
                Eth = -dphi_dts * dts_dt / r
                Er = -dphi_dts * dts_dr
                rho = math.hypot(pos[0], pos[1])
                that = np.array([math.cos(t) * pos[0] / rho, math.cos(t) * pos[1] / rho, -math.sin(t)])
                B = IO.dipole(M, (0.0, 0.0, -1.0), pos)
                want = np.cross(Eth * that + Er * pos / r, B) / np.dot(B, B)
                got = v[:, k - k0, j - j0, i - i0]
                worst = max(worst, float(np.linalg.norm(got - want) / np.linalg.norm(want)))
                radial = max(radial, abs(float(np.dot(got, pos))) / (float(np.linalg.norm(got)) * r))
                checked += 1
    return worst, radial, checked


def test_drift_of_an_axisymmetric_potential():
    # a uniform current on each cap -> Phi(theta_s) in closed form, carried to
    # (r, theta) by sin^2 theta_s = (r_s / r) sin^2 theta; E = -grad Phi
    # (theta and r parts through theta_s) and v = E x B / B^2 is azimuthal;
    # the central differences of the mapped potential converge to it at
    # second order
    e1, r1, n1 = _drift_error(24)
    e2, r2, n2 = _drift_error(48)
    assert n1 > 20 and n2 > 100
    assert e2 < 0.05 and e2 < e1 / 3.0, (e1, e2)
    assert r2 < 0.02, r2


def test_inner_reset_takes_the_drift():
    n = 16
    faces = [np.linspace(-4.0, 4.0, n + 1)] * 3
    U = I.conserved(np.ones((n, n, n)), 0.1, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, G)
    prob = O.OracleProblem(faces, r_inner=2.5, inner_rho=2.0, inner_p=0.5, dip_moment=0.0)
    box = IO.inner_box(faces, 2.5)
    i0, i1, j0, j1, k0, k1 = box
    rng = np.random.default_rng(0)
    v = rng.standard_normal((3, k1 - k0, j1 - j0, i1 - i0)) * 0.1
    prob.set_inner_velocity(box, v)
    out = prob.sweep(U, 0.01, 0)
    xc = IO.centres(faces)[0]
    for k in range(k0, k1):
        for j in range(j0, j1):
            for i in range(i0, i1):
                r2 = xc[i] ** 2 + xc[j] ** 2 + xc[k] ** 2
                if r2 >= 2.5 ** 2:
                    continue
                vv = v[:, k - k0, j - j0, i - i0]
                assert np.allclose(out[1:4, k, j, i], 2.0 * vv, rtol=0, atol=1e-15)
                assert np.all(out[4:7, k, j, i] == 0.0)
                assert abs(out[7, k, j, i] - (0.5 / (G - 1) + 0.5 * 2.0 * np.dot(vv, vv))) <= 1e-15
    prob.set_inner_velocity(None)
    out0 = prob.sweep(U, 0.01, 0)
    mask = np.zeros(out0.shape[1:], bool)
    for k in range(n):
        for j in range(n):
            for i in range(n):
                mask[k, j, i] = xc[i] ** 2 + xc[j] ** 2 + xc[k] ** 2 < 2.5 ** 2
    assert np.all(out0[1:4][:, mask] == 0.0)
