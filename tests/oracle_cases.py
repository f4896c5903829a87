"""Problem builders shared by the oracle pins and the GPU parity tests.

Only test infrastructure imports this module.  The linear eigenmodes come from
a numerical eigen-decomposition of the 1D ideal-MHD primitive system (no
formula of the scheme is involved)."""
from __future__ import annotations

import math

import numpy as np

from paper_1607_02214_amd import inputs as I

G = 5.0 / 3.0


def mhd_jacobian(rho, p, Bn, Bt1, Bt2, gamma=G):
    """Primitive 1D ideal-MHD Jacobian A (zero background velocity) for
    W = (rho, u, v1, v2, B1, B2, p):  dW/dt + A dW/dn = 0."""
    A = np.zeros((7, 7))
    A[0, 1] = rho
    A[1, 4] = Bt1 / rho
    A[1, 5] = Bt2 / rho
    A[1, 6] = 1.0 / rho
    A[2, 4] = -Bn / rho
    A[3, 5] = -Bn / rho
    A[4, 1] = Bt1
    A[4, 2] = -Bn
    A[5, 1] = Bt2
    A[5, 3] = -Bn
    A[6, 1] = gamma * p
    return A


def eigenmode(kind, rho, p, Bn, Bt1, Bt2, gamma=G):
    """(speed, right eigenvector) of the right-moving fast / alfven / slow
    wave, eigenvector normalised to unit 2-norm with a fixed sign."""
    lam, R = np.linalg.eig(mhd_jacobian(rho, p, Bn, Bt1, Bt2, gamma))
    lam = lam.real
    R = R.real
    pos = np.argsort(-lam)
    order = {"fast": 0, "alfven": 1, "slow": 2}[kind]
    k = pos[order]
    r = R[:, k] / np.linalg.norm(R[:, k])
    j = np.argmax(np.abs(r))
    r = r * np.sign(r[j])
    return lam[k], r


def wave_state_1d(N, kind, amp=1e-6, rho=1.0, p=1.0, B=(1.0, 1.5, 0.0), axis=0, gamma=G,
                  v0=(0.0, 0.0, 0.0), split_background=False):
    """Periodic N-zone pencil along `axis` (other axes size 1) holding a
    sinusoidal right-moving eigenmode on a background moving with v0 (the
    mode then travels at speed + v0[axis]); returns (U, faces, speed).  With
    split_background the uniform background field is left out of B' (it is
    to be carried as the static field B_d)."""
    Bn = B[axis]
    Bt1 = B[(axis + 1) % 3]
    Bt2 = B[(axis + 2) % 3]
    lam, r = eigenmode(kind, rho, p, Bn, Bt1, Bt2, gamma)
    f = I.uniform_faces(N)
    xc = I.centres(f)
    s = np.sin(2 * np.pi * xc) * np.sinc(1.0 / N)   # exact cell averages of sin
    W = [rho, 0.0, 0.0, 0.0, Bt1, Bt2, p]
    prim = [W[i] + amp * r[i] * s for i in range(7)]
    v = [None] * 3
    Bv = [None] * 3
    v[axis], v[(axis + 1) % 3], v[(axis + 2) % 3] = prim[1], prim[2], prim[3]
    v = [v[k] + v0[k] for k in range(3)]
    Bv[axis] = Bn + 0 * s
    Bv[(axis + 1) % 3], Bv[(axis + 2) % 3] = prim[4], prim[5]
    if split_background:
        Bv = [Bv[k] - B[(k - axis) % 3] for k in range(3)]
    U1 = I.conserved(prim[0], v[0], v[1], v[2], Bv[0], Bv[1], Bv[2], prim[6], gamma)  # [8, N]
    shape = [1, 1, 1]
    shape[2 - axis] = N
    U = U1.reshape((8,) + tuple(shape))
    faces = [I.uniform_faces(1), I.uniform_faces(1), I.uniform_faces(1)]
    faces[axis] = f
    return U, faces, lam + v0[axis]


def oblique_wave_state(N, kind, amp=1e-6, rho=1.0, p=1.0, B=(1.2, 0.4, 0.9), gamma=G):
    """2D periodic N x N x 1 box, wave vector (1, 1, 0) * 2 pi; B is given in
    the frame (n, t1, t2) with n along (1,1,0)/sqrt2, t1 = (-1,1,0)/sqrt2,
    t2 = z.  Returns (U, faces, speed, period)."""
    lam, r = eigenmode(kind, rho, p, B[0], B[1], B[2], gamma)
    f = I.uniform_faces(N)
    xc = I.centres(f)
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    # cell average of sin(2 pi (x + y)) on a square cell
    s = np.sin(2 * np.pi * (X + Y)) * np.sinc(1.0 / N) ** 2
    n = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    t1 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    t2 = np.array([0.0, 0.0, 1.0])
    rho_ = rho + amp * r[0] * s
    vn, v1, v2 = amp * r[1] * s, amp * r[2] * s, amp * r[3] * s
    b1, b2 = B[1] + amp * r[4] * s, B[2] + amp * r[5] * s
    p_ = p + amp * r[6] * s
    v = [vn * n[k] + v1 * t1[k] + v2 * t2[k] for k in range(3)]
    Bv = [B[0] * n[k] + b1 * t1[k] + b2 * t2[k] for k in range(3)]
    U = I.conserved(rho_, v[0], v[1], v[2], Bv[0], Bv[1], Bv[2], p_, gamma)[:, None, :, :]
    faces = [f, f.copy(), I.uniform_faces(1)]
    # wavelength along n is 1/sqrt2
    period = (1.0 / math.sqrt(2.0)) / lam
    return U, faces, lam, period


def run_to(prob, U, t_end, cfl=0.4, start_step=0):
    """Advance with the oracle to exactly t_end (last dt shortened)."""
    t = 0.0
    step = start_step
    while t < t_end - 1e-14 * t_end:
        dt = prob.cfl_dt(U, cfl)
        dt = min(dt, t_end - t)
        U = prob.step(U, dt, step)
        t += dt
        step += 1
    return U, step


def background_in_xyz(B, axis):
    """Field given in the pencil frame (n, t1, t2) of `axis`, in (x, y, z)."""
    out = [0.0, 0.0, 0.0]
    out[axis], out[(axis + 1) % 3], out[(axis + 2) % 3] = B
    return tuple(out)


def primitives(U, faces=None, bd=None, gamma=G):
    """(rho, v[3], B_total[3], p) from a conserved state; bd = B_d arrays."""
    rho = U[0]
    v = [U[1 + k] / rho for k in range(3)]
    bp = [U[4 + k] for k in range(3)]
    p = (gamma - 1) * (U[7] - 0.5 * rho * sum(x * x for x in v) - 0.5 * sum(x * x for x in bp))
    Bt = [bp[k] + (bd[k] if bd is not None else 0.0) for k in range(3)]
    return rho, v, Bt, p
