"""Paired problem definitions for GPU-vs-oracle parity tests: one description
builds both the HIP context (through the C ABI binding) and the oracle
problem, so that both sides see the same grid, boundaries, background field,
inflow and options.  Test infrastructure only."""
from __future__ import annotations

import sys
from dataclasses import dataclass, field

import numpy as np

from paper_1607_02214_amd import inputs as I


@dataclass
class Case:
    name: str
    faces: list
    U: np.ndarray                       # FP64 conserved state [8, nz, ny, nx]
    bc_lo: tuple = (0, 0, 0)
    bc_hi: tuple = (0, 0, 0)
    dip_moment: float = 0.0
    dip_dir: tuple = (0.0, 0.0, -1.0)
    bext: tuple = (0.0, 0.0, 0.0)
    inflow: tuple | None = None
    r_inner: float = 0.0
    inner_rho: float = 1.0
    inner_p: float = 1.0
    flatten: bool = True
    janhunen: bool = True
    max_iter: int = 20
    p_floor: float = 1e-8
    tol64: float = 1e-12
    tol32: float = 1e-6
    tracing: int = 0                    # 0: two-family tracing, 1: characteristic mode
    meta: dict = field(default_factory=dict)

    def oracle(self, tol=None):
        from oracle import oracle as O
        return O.OracleProblem(self.faces, bc_lo=self.bc_lo, bc_hi=self.bc_hi, dip_moment=self.dip_moment,
                               dip_dir=self.dip_dir, bext=self.bext, inflow=self.inflow,
                               r_inner=self.r_inner, inner_rho=self.inner_rho, inner_p=self.inner_p,
                               flatten=self.flatten, janhunen=self.janhunen, max_iter=self.max_iter,
                               tol=self.tol64 if tol is None else tol, p_floor=self.p_floor,
                               tracing=self.tracing)

    def context(self, **over):
        from paper_1607_02214_amd import ppmlr
        opt = dict(flatten=int(self.flatten), janhunen=int(self.janhunen), max_iter=self.max_iter,
                   tol_f64=self.tol64, tol_f32=self.tol32, p_floor=self.p_floor, tracing=self.tracing)
        opt.update(over)
        ctx = ppmlr.Context(self.faces, self.bc_lo, self.bc_hi, r_inner=self.r_inner, **opt)
        if self.dip_moment != 0.0:
            ctx.set_dipole(self.dip_moment, self.dip_dir)
        if any(b != 0.0 for b in self.bext):
            ctx.set_background(self.bext)
        if self.inflow is not None:
            ctx.set_inflow(self.inflow)
        if self.r_inner > 0:
            ctx.set_inner(self.inner_rho, self.inner_p)
        return ctx


def c1_case(n=32):
    U, faces = I.c1_state(n=n)
    return Case("c1-periodic", faces, U)


def dipole_case(nx=48, ny=28, nz=24, seed=0):
    """Inflow/dipole set-up of the paper's Section IV-A on a small stretched
    grid (coarsened widths so that the box still holds the bow-shock region)."""
    s = 192.0 / (2 * ny)
    kw = dict(w_min=0.25 * s * 2, w_max=2.0 * s * 2, growth=1.03, core=max(2, ny // 8))
    fx = I.stretched_faces(3 * nx // 4, nx - 3 * nx // 4, **kw)
    fy = I.stretched_faces(ny // 2, ny - ny // 2, **kw)
    fz = I.stretched_faces(nz // 2, nz - nz // 2, **kw)
    faces = [fx, fy, fz]
    st = I.c2_setup(faces)
    return Case("inflow-dipole", faces, st.U, bc_lo=st.bc_lo, bc_hi=st.bc_hi, dip_moment=st.moment,
                dip_dir=st.direction, inflow=tuple(st.inflow), r_inner=st.r_inner, inner_rho=st.inner_rho,
                inner_p=st.inner_p, p_floor=st.p_floor)


def blast_case(n=(40, 33, 30), seed=3):
    rng = np.random.default_rng(seed)
    faces = [np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 1.5, k))]) for k in n]
    faces = [f / f[-1] for f in faces]
    U = I.blast_state(faces, seed=seed)
    return Case("blast", faces, U, bc_lo=(1, 1, 1), bc_hi=(1, 1, 1))


def smooth_case(shape=(21, 18, 37), seed=5, bext=(0.0, 0.0, 0.0)):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    faces = [np.concatenate([[0.0], np.cumsum(rng.uniform(0.6, 1.4, k))]) for k in (nx, ny, nz)]
    faces = [f / f[-1] for f in faces]
    U = I.random_smooth_state(shape, seed=seed)
    return Case("smooth-stretched", faces, U, bext=bext)


def normwise_errors(gpu: np.ndarray, ref: np.ndarray):
    """Per conserved variable: max |gpu - ref| / max |ref| (FP64)."""
    g = gpu.reshape(8, -1).astype(np.float64)
    r = ref.reshape(8, -1).astype(np.float64)
    scale = np.maximum(np.max(np.abs(r), axis=1), 1e-300)
    return np.max(np.abs(g - r), axis=1) / scale


FAMILIES = ((0,), (1, 2, 3), (4, 5, 6), (7,))


def familywise_errors(gpu: np.ndarray, ref: np.ndarray):
    """Per conserved variable: max |gpu - ref| over the largest |ref| of its
    family (mass; the three momentum components; the three field components;
    energy), so that a component that vanishes in exact arithmetic (the
    transverse momentum of a blast at rest) is measured against its
    family's scale instead of its own rounding noise."""
    g = gpu.reshape(8, -1).astype(np.float64)
    r = ref.reshape(8, -1).astype(np.float64)
    out = np.zeros(8)
    for fam in FAMILIES:
        scale = max(float(np.max(np.abs(r[list(fam)]))), 1e-300)
        for q in fam:
            out[q] = float(np.max(np.abs(g[q] - r[q]))) / scale
    return out


def pointwise_errors(gpu: np.ndarray, ref: np.ndarray, floor: float = 1e-6, by_family: bool = False):
    """Per conserved variable: max_i |gpu_i - ref_i| / max(|ref_i|, floor *
    max |ref|), the pointwise form of the error metric (each zone against its
    own magnitude, so that a small-valued region is not measured against the
    largest value elsewhere in the box).  by_family: the floor is taken from
    the largest |ref| of the variable's family (see familywise_errors)."""
    g = gpu.reshape(8, -1).astype(np.float64)
    r = ref.reshape(8, -1).astype(np.float64)
    scale = np.maximum(np.max(np.abs(r), axis=1), 1e-300)
    if by_family:
        for fam in FAMILIES:
            scale[list(fam)] = max(float(np.max(scale[list(fam)])), 1e-300)
    den = np.maximum(np.abs(r), floor * scale[:, None])
    return np.max(np.abs(g - r) / den, axis=1)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def fp32_errors(gpu: np.ndarray, ref: np.ndarray, gamma=5.0 / 3.0):
    """FP32-vs-FP64 error per result: normwise on the primitive fields rho,
    p and |B'| (max |f32 - f64| / max |f64|), and the momentum error measured
    against the flow's momentum scale max(rho * c) with c the magnetosonic
    speed sqrt((gamma p + |B'|^2) / rho)."""
    def prim(U):
        U = U.reshape(8, -1).astype(np.float64)
        rho = U[0]
        v2 = (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / (rho * rho)
        b2 = U[4] ** 2 + U[5] ** 2 + U[6] ** 2
        p = (gamma - 1) * (U[7] - 0.5 * rho * v2 - 0.5 * b2)
        return rho, p, np.sqrt(b2), U[1:4]
    rg, pg, bg, mg = prim(gpu)
    rr, pr, br, mr = prim(ref)
    out = {}
    for name, a, b in (("rho", rg, rr), ("p", pg, pr), ("|B'|", bg, br)):
        out[name] = float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
    mscale = np.max(np.sqrt(rr * (gamma * pr + br * br)))
    out["m"] = float(np.max(np.abs(mg - mr)) / mscale)
    return out
