"""Ionosphere shell coupling of the oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package's smoke check and the benchmark's CPU baseline use
this module; the HIP path has its own implementation and shares nothing with
it.  Plain FP64 numpy (and one sparse direct solve) written for checking by
eye, with loops where they make the steps plain.

Paper, Section II (the ionosphere paragraph): a thin shell at r = 1.017 R_E
closes the field-aligned currents under the electrostatic assumption; an
electrostatic potential equation is solved on it, and the potential is
carried along dipole field lines to the magnetospheric inner boundary at
r = 3 R_E, where it sets the flow.  The paper states the coupling in words
only; the readings taken here:

* Field-aligned current.  J = curl B' (the background field is curl-free),
  at zone centres by central differences ((f[i+1] - f[i-1]) /
  (x[i+1] - x[i-1]) per axis; zero in the outermost layer of zones), taken
  at the point where the field line of a shell cell crosses the sphere
  r_fac (trilinear interpolation between zone centres) and projected on the
  dipole direction.  Along a flux tube J_par / |B| is constant (div J = 0,
  J parallel to B), so the current density at the shell is J_par(r_fac) *
  |B(shell)| / |B(r_fac)|, and its radial component j_r (outward positive)
  feeds the shell.
* Shell.  Height-integrated Pedersen conductance Sigma, uniform, no Hall
  term; the shell's horizontal current K = -Sigma grad Phi carries away what
  the field-aligned current brings (div_h K = -j_r), so
  div_h(Sigma grad_h Phi) = j_r.  Each hemisphere is solved on the polar cap
  whose field lines cross r_fac (sin^2 theta <= r_shell / r_fac) with
  Phi = 0 at the cap's edge.
* Discretisation: finite volumes on cells uniform in magnetic colatitude
  (n_theta over the cap) and longitude (n_phi), Phi at cell centres; fluxes
  Sigma * (difference of Phi) / (distance) times face length; no flux
  through the pole; the edge value 0 half a cell outside the last ring.
* Mapping back.  Phi is constant along a dipole field line (r = L sin^2
  theta), so a point (r, theta, phi) takes the shell potential at
  sin^2 theta_s = (r_shell / r) sin^2 theta, same longitude and hemisphere
  (0 equatorward of the cap), by bilinear interpolation in (theta, phi)
  (towards the pole: the mean of the first ring; towards the edge: 0).
* Drift of the reset zones (r < r_inner): E = -grad Phi by central
  differences of the mapped potential at the neighbouring zone centres,
  v = E x B_d / |B_d|^2 (the dipole alone); zero where the zone or a
  neighbour lies inside the shell (r <= r_shell).
* Magnetic frame: z_m opposite to the dipole moment (the dipole points from
  north to south), x_m the x axis projected off z_m (the y axis if x is
  along z_m), y_m = z_m x x_m.  Hemisphere 0 has z_m > 0.
* Units: code units with mu_0 = 1, so Sigma[code] = Sigma[S] * mu_0 * v_0
  (v_0 = 21.81 km/s: 5 S -> 0.137).
"""
from __future__ import annotations

import math

import numpy as np

MU0 = 4.0e-7 * math.pi
V0 = 21.81e3                       # code velocity unit, m/s


def sigma_code(sigma_siemens: float) -> float:
    """Height-integrated conductance in code units (mu_0 = 1)."""
    return sigma_siemens * MU0 * V0


def magnetic_frame(dip_dir):
    m = np.asarray(dip_dir, dtype=np.float64)
    m = m / np.linalg.norm(m)
    zm = -m
    x = np.array([1.0, 0.0, 0.0])
    xm = x - np.dot(x, zm) * zm
    if np.linalg.norm(xm) < 1e-6:
        y = np.array([0.0, 1.0, 0.0])
        xm = y - np.dot(y, zm) * zm
    xm = xm / np.linalg.norm(xm)
    ym = np.cross(zm, xm)
    return xm, ym, zm


def dipole(moment, dip_dir, pos):
    """B_d = M [3 (m.r) r / r^5 - m / r^3] (the dipole alone)."""
    m = np.asarray(dip_dir, dtype=np.float64)
    m = m / np.linalg.norm(m)
    r = np.asarray(pos, dtype=np.float64)
    r2 = float(np.dot(r, r))
    rr = math.sqrt(r2)
    return moment * (3.0 * np.dot(m, r) * r / (r2 * r2 * rr) - m / (r2 * rr))


class ShellGrid:
    """Cells of the two polar caps of the shell."""

    def __init__(self, n_theta=32, n_phi=64, r_shell=1.017, r_fac=3.5):
        if not (r_fac > r_shell > 0.0):
            raise ValueError("need r_fac > r_shell > 0")
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        self.r_shell, self.r_fac = float(r_shell), float(r_fac)
        self.theta_c = math.asin(math.sqrt(self.r_shell / self.r_fac))
        self.dth = self.theta_c / self.n_theta
        self.dph = 2.0 * math.pi / self.n_phi
        self.th = (np.arange(self.n_theta) + 0.5) * self.dth
        self.ph = (np.arange(self.n_phi) + 0.5) * self.dph

    def area(self, k):
        """Area of a cell of ring k on the sphere r_shell."""
        return self.r_shell ** 2 * (math.cos(k * self.dth) - math.cos((k + 1) * self.dth)) * self.dph

    def shell_point(self, frame, h, k, j):
        """Unit vector of cell (hemisphere h, ring k, column j)."""
        xm, ym, zm = frame
        s, c = math.sin(self.th[k]), math.cos(self.th[k])
        sgn = 1.0 if h == 0 else -1.0
        return s * math.cos(self.ph[j]) * xm + s * math.sin(self.ph[j]) * ym + sgn * c * zm

    def fac_point(self, frame, h, k, j):
        """Where the field line of cell (h, k, j) crosses r_fac."""
        xm, ym, zm = frame
        sf = math.sin(self.th[k]) * math.sqrt(self.r_fac / self.r_shell)
        cf = math.sqrt(max(0.0, 1.0 - sf * sf))
        sgn = 1.0 if h == 0 else -1.0
        return self.r_fac * (sf * math.cos(self.ph[j]) * xm + sf * math.sin(self.ph[j]) * ym + sgn * cf * zm)


def centres(faces):
    return [0.5 * (np.asarray(f)[1:] + np.asarray(f)[:-1]) for f in faces]


def zone_curl(faces, Bp):
    """curl B' at zone centres: Bp[3, nz, ny, nx] -> J[3, nz, ny, nx];
    central differences per axis, zero in the outermost layer."""
    xc, yc, zc = centres(faces)
    nz, ny, nx = Bp.shape[1:]
    J = np.zeros_like(Bp)

    def d(f, axis, c, idx):
        i, j, k = idx
        if axis == 0:
            return (f[k, j, i + 1] - f[k, j, i - 1]) / (c[i + 1] - c[i - 1])
        if axis == 1:
            return (f[k, j + 1, i] - f[k, j - 1, i]) / (c[j + 1] - c[j - 1])
        return (f[k + 1, j, i] - f[k - 1, j, i]) / (c[k + 1] - c[k - 1])

    Bx, By, Bz = Bp
    for k in range(1, nz - 1):
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                idx = (i, j, k)
                J[0, k, j, i] = d(Bz, 1, yc, idx) - d(By, 2, zc, idx)
                J[1, k, j, i] = d(Bx, 2, zc, idx) - d(Bz, 0, xc, idx)
                J[2, k, j, i] = d(By, 0, xc, idx) - d(Bx, 1, yc, idx)
    return J


def trilinear(faces, F, pos):
    """Trilinear interpolation of F[c, nz, ny, nx] (zone-centred) at pos."""
    cs = centres(faces)
    idx, w = [], []
    for a in range(3):
        c = cs[a]
        if not (c[0] <= pos[a] <= c[-1]):
            raise ValueError("interpolation point outside the zone centres")
        i = int(np.searchsorted(c, pos[a], side="right")) - 1
        i = min(i, len(c) - 2)
        idx.append(i)
        w.append((pos[a] - c[i]) / (c[i + 1] - c[i]))
    i, j, k = idx
    wx, wy, wz = w
    out = np.zeros(F.shape[0])
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                wt = (wx if di else 1 - wx) * (wy if dj else 1 - wy) * (wz if dk else 1 - wz)
                out += wt * F[:, k + dk, j + dj, i + di]
    return out


def shell_current(faces, U, moment, dip_dir, grid: ShellGrid):
    """Radial current density j_r [2, n_theta, n_phi] entering the shell's
    cells from the field-aligned current at r_fac (outward positive)."""
    frame = magnetic_frame(dip_dir)
    J = zone_curl(faces, U[4:7])
    jr = np.zeros((2, grid.n_theta, grid.n_phi))
    for h in range(2):
        for k in range(grid.n_theta):
            for j in range(grid.n_phi):
                rs = grid.shell_point(frame, h, k, j)
                P = grid.fac_point(frame, h, k, j)
                BP = dipole(moment, dip_dir, P)
                Bs = dipole(moment, dip_dir, grid.r_shell * rs)
                nP, ns = np.linalg.norm(BP), np.linalg.norm(Bs)
                jpar = float(np.dot(trilinear(faces, J, P), BP)) / nP
                jr[h, k, j] = jpar * (ns / nP) * float(np.dot(Bs, rs)) / ns
    return jr


def shell_matrix(grid: ShellGrid):
    """Finite-volume operator of div_h(grad_h Phi) integrated over a cell
    (Sigma = 1), with Phi = 0 at the cap's edge: sparse [n, n], n = n_theta *
    n_phi, unknown q = k * n_phi + j."""
    import scipy.sparse as sp
    nt, nph, dth, dph = grid.n_theta, grid.n_phi, grid.dth, grid.dph
    rows, cols, vals = [], [], []

    def add(q, p, v):
        rows.append(q)
        cols.append(p)
        vals.append(v)

    for k in range(nt):
        sk = math.sin(grid.th[k])
        for j in range(nph):
            q = k * nph + j
            if k + 1 < nt:                        # face towards the edge
                a = math.sin((k + 1) * dth) * dph / dth
                add(q, q, -a)
                add(q, q + nph, a)
            else:                                 # the edge, Phi = 0 half a cell out
                a = math.sin(grid.theta_c) * dph / (0.5 * dth)
                add(q, q, -a)
            if k > 0:                             # face towards the pole
                a = math.sin(k * dth) * dph / dth
                add(q, q, -a)
                add(q, q - nph, a)
            b = dth / (sk * dph)                  # the two longitude faces
            for jj in ((j + 1) % nph, (j - 1) % nph):
                add(q, q, -b)
                add(q, k * nph + jj, b)
    n = nt * nph
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def solve_potential(grid: ShellGrid, jr, sigma):
    """Phi [2, n_theta, n_phi] with div_h(Sigma grad_h Phi) = j_r on each cap."""
    import scipy.sparse.linalg as spla
    L = shell_matrix(grid).tocsc()
    area = np.array([grid.area(k) for k in range(grid.n_theta)])
    phi = np.zeros_like(jr)
    for h in range(2):
        rhs = (jr[h] * area[:, None] / sigma).reshape(-1)
        phi[h] = spla.spsolve(L, rhs).reshape(grid.n_theta, grid.n_phi)
    return phi


def potential_at(grid: ShellGrid, phi, frame, pos):
    """Shell potential carried along the dipole field line through pos
    (None inside the shell)."""
    xm, ym, zm = frame
    r = float(np.linalg.norm(pos))
    if r <= grid.r_shell:
        return None
    x, y, z = float(np.dot(pos, xm)), float(np.dot(pos, ym)), float(np.dot(pos, zm))
    s2 = (grid.r_shell / r) * (x * x + y * y) / (r * r)
    if s2 > math.sin(grid.theta_c) ** 2:
        return 0.0
    th = math.asin(math.sqrt(s2))
    ph = math.atan2(y, x) % (2.0 * math.pi)
    h = 0 if z >= 0.0 else 1
    nt, nph = grid.n_theta, grid.n_phi

    def ring(k):
        s = ph / grid.dph - 0.5
        j0 = math.floor(s)
        wj = s - j0
        return (1.0 - wj) * phi[h, k, j0 % nph] + wj * phi[h, k, (j0 + 1) % nph]

    t = th / grid.dth - 0.5
    if t < 0.0:
        w = (t + 0.5) / 0.5
        return (1.0 - w) * float(np.mean(phi[h, 0])) + w * ring(0)
    if t > nt - 1:
        w = (t - (nt - 1)) / 0.5
        return (1.0 - w) * ring(nt - 1)
    k = int(math.floor(t))
    w = t - k
    return (1.0 - w) * ring(k) + w * ring(k + 1)


def inner_box(faces, r_inner):
    """Index box (i0, i1, j0, j1, k0, k1) (half-open) holding every zone whose
    centre lies inside r_inner."""
    box = []
    for c in centres(faces):
        inside = np.nonzero(c * c < r_inner * r_inner)[0]
        if len(inside) == 0:
            return None
        box += [int(inside[0]), int(inside[-1]) + 1]
    return tuple(box)


def inner_drift(faces, r_inner, moment, dip_dir, grid: ShellGrid, phi):
    """(box, v[3, nk, nj, ni]): the E x B drift of the reset zones."""
    box = inner_box(faces, r_inner)
    if box is None:
        return None, None
    frame = magnetic_frame(dip_dir)
    cs = centres(faces)
    i0, i1, j0, j1, k0, k1 = box
    v = np.zeros((3, k1 - k0, j1 - j0, i1 - i0))
    n = [len(c) for c in cs]
    for k in range(k0, k1):
        for j in range(j0, j1):
            for i in range(i0, i1):
                pos = np.array([cs[0][i], cs[1][j], cs[2][k]])
                if float(np.dot(pos, pos)) >= r_inner * r_inner:
                    continue
                idx = [i, j, k]
                E = np.zeros(3)
                ok = True
                for a in range(3):
                    if idx[a] == 0 or idx[a] == n[a] - 1:
                        ok = False
                        break
                    pp, pm = pos.copy(), pos.copy()
                    pp[a] = cs[a][idx[a] + 1]
                    pm[a] = cs[a][idx[a] - 1]
                    fp, fm = potential_at(grid, phi, frame, pp), potential_at(grid, phi, frame, pm)
                    if fp is None or fm is None or potential_at(grid, phi, frame, pos) is None:
                        ok = False
                        break
                    E[a] = -(fp - fm) / (pp[a] - pm[a])
                if not ok:
                    continue
                B = dipole(moment, dip_dir, pos)
                v[:, k - k0, j - j0, i - i0] = np.cross(E, B) / float(np.dot(B, B))
    return box, v


def couple(prob, U, grid: ShellGrid, sigma):
    """One coupling of an OracleProblem's state: shell current, potential,
    and the drift of the reset zones set on the problem.  Returns (j_r, Phi,
    box, v)."""
    faces = prob.faces
    moment = prob.p.dip_moment
    dip_dir = [prob.p.dip_dir[q] for q in range(3)]
    jr = shell_current(faces, U, moment, dip_dir, grid)
    phi = solve_potential(grid, jr, sigma)
    box, v = inner_drift(faces, prob.p.r_inner, moment, dip_dir, grid, phi)
    prob.set_inner_velocity(box, v)
    return jr, phi, box, v
