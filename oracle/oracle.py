"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this module.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

The oracle follows the paper's Section II (zone-centred averages, parabolic
reconstruction, characteristic edge values, Lagrangian update, remap) and the
dimensional splitting of Section III-A; the scheme details follow Colella &
Woodward (1984).  See `oracle/ppmlr_oracle.c` for the function-by-function
citations.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(_HERE, "libppmlr_oracle.so")
SRC_PATH = os.path.join(_HERE, "ppmlr_oracle.c")
MLP_SRC_PATH = os.path.join(_HERE, "mlp_oracle.c")

BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= max(
            os.path.getmtime(SRC_PATH), os.path.getmtime(MLP_SRC_PATH)):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, SRC_PATH, MLP_SRC_PATH, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("faces", C.POINTER(C.c_double) * 3),
        ("bc_lo", C.c_int * 3),
        ("bc_hi", C.c_int * 3),
        ("gamma", C.c_double),
        ("dip_moment", C.c_double),
        ("dip_dir", C.c_double * 3),
        ("bext", C.c_double * 3),
        ("inflow", C.c_double * 8),
        ("r_inner", C.c_double),
        ("inner_rho", C.c_double),
        ("inner_p", C.c_double),
        ("inner_v", C.POINTER(C.c_double)),
        ("inner_box", C.c_int * 6),
        ("flatten", C.c_int),
        ("janhunen", C.c_int),
        ("max_iter", C.c_int),
        ("tol", C.c_double),
        ("p_floor", C.c_double),
        ("tracing", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iters_hist", C.c_longlong * 32),
        ("floor_hits", C.c_longlong),
        ("nonconverged", C.c_longlong),
        ("nonphys", C.c_longlong),
    ]

    def as_dict(self):
        return {
            "iters_hist": list(self.iters_hist),
            "floor_hits": self.floor_hits,
            "nonconverged": self.nonconverged,
            "nonphys": self.nonphys,
        }


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_get_threads.argtypes = []
        L.oracle_get_threads.restype = C.c_int
        L.oracle_sweep.argtypes = [C.POINTER(Problem), dp, C.c_double, C.c_int, C.POINTER(Stats)]
        L.oracle_sweep.restype = C.c_int
        L.oracle_sweep_pencils.argtypes = [C.POINTER(Problem), dp, C.c_double, C.c_int, C.c_int,
                                           ip, ip, dp, C.POINTER(Stats)]
        L.oracle_sweep_pencils.restype = C.c_int
        L.oracle_step.argtypes = [C.POINTER(Problem), dp, C.c_double, C.c_longlong, C.POINTER(Stats)]
        L.oracle_step.restype = C.c_int
        L.oracle_cfl_dt.argtypes = [C.POINTER(Problem), dp, C.c_double]
        L.oracle_cfl_dt.restype = C.c_double
        L.oracle_totals.argtypes = [C.POINTER(Problem), dp, dp]
        L.oracle_totals.restype = None
        L.oracle_ppm_edges.argtypes = [C.c_int, dp, dp, C.c_int, dp]
        L.oracle_ppm_slopes.argtypes = [C.c_int, dp, dp, C.c_int, dp]
        L.oracle_ppm_parabolas.argtypes = [C.c_int, dp, dp, dp, C.c_int, C.c_int, dp]
        L.oracle_par_avg.argtypes = [C.c_double] * 4 + [C.c_int]
        L.oracle_par_avg.restype = C.c_double
        L.oracle_flattening.argtypes = [C.c_int, dp, dp, dp, dp, dp]
        L.oracle_riemann_normal.argtypes = [C.c_double] * 9 + [C.c_double, C.c_int, dp, dp, ip]
        L.oracle_riemann_normal.restype = C.c_int
        L.oracle_riemann_alfven.argtypes = [C.c_double] * 7 + [dp, dp]
        L.oracle_dipole.argtypes = [C.POINTER(Problem), dp, dp]
        L.oracle_ghosts.restype = C.c_int
        L.oracle_mhd7_eigen.argtypes = [C.c_double] * 6 + [dp, dp]
        L.oracle_mhd7_eigen.restype = None
        L.oracle_trace7.argtypes = [C.c_double] * 6 + [dp, C.c_double, C.c_double, dp, dp]
        L.oracle_trace7.restype = C.c_int
        L.oracle_face_states.argtypes = [C.POINTER(Problem), dp, C.c_double, C.c_int, C.c_int, C.c_int, dp]
        L.oracle_face_states.restype = C.c_int
        L.oracle_riemann7.argtypes = [dp, dp] + [C.c_double] * 4 + [dp]
        L.oracle_riemann7.restype = C.c_int
        L.mlp_gelu.argtypes = [C.c_double]
        L.mlp_gelu.restype = C.c_double
        L.mlp_gelu_grad.argtypes = [C.c_double]
        L.mlp_gelu_grad.restype = C.c_double
        L.mlp_num_params.restype = C.c_int
        L.mlp_forward.argtypes = [dp, C.c_int, dp, dp, dp, dp]
        L.mlp_loss_grad.argtypes = [dp, C.c_int, dp, dp, dp]
        L.mlp_loss_grad.restype = C.c_double
        L.mlp_adam.argtypes = [dp, dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleProblem:
    """Holds a `Problem` struct and keeps its face arrays alive."""

    def __init__(self, faces, bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), gamma=5.0 / 3.0,
                 dip_moment=0.0, dip_dir=(0.0, 0.0, -1.0), bext=(0.0, 0.0, 0.0), inflow=None, r_inner=0.0,
                 inner_rho=1.0, inner_p=1.0, flatten=True, janhunen=True, max_iter=20,
                 tol=1e-12, p_floor=1e-8, tracing=0):
        self.faces = [np.ascontiguousarray(f, dtype=np.float64) for f in faces]
        p = Problem()
        for a in range(3):
            p.n[a] = len(self.faces[a]) - 1
            p.faces[a] = _dptr(self.faces[a])
            p.bc_lo[a] = int(bc_lo[a])
            p.bc_hi[a] = int(bc_hi[a])
        p.gamma = gamma
        p.dip_moment = dip_moment
        for k in range(3):
            p.dip_dir[k] = dip_dir[k]
            p.bext[k] = bext[k]
        inflow = inflow if inflow is not None else [1, 0, 0, 0, 0, 0, 0, 1]
        for k in range(8):
            p.inflow[k] = inflow[k]
        p.r_inner = r_inner
        p.inner_rho = inner_rho
        p.inner_p = inner_p
        p.flatten = int(bool(flatten))
        p.janhunen = int(bool(janhunen))
        p.max_iter = int(max_iter)
        p.tol = tol
        p.p_floor = p_floor
        p.tracing = int(tracing)
        self.p = p

    @property
    def shape(self):
        return (8, self.p.n[2], self.p.n[1], self.p.n[0])

    def set_inner_velocity(self, box=None, v=None):
        """Velocity of the zones the inner boundary resets (the ionosphere's
        drift): box = (i0, i1, j0, j1, k0, k1) zone-index ranges (half-open),
        v: [3, k1 - k0, j1 - j0, i1 - i0].  None: the reset zones are at rest."""
        if v is None:
            self._inner_v = None
            self.p.inner_v = None
            for q in range(6):
                self.p.inner_box[q] = 0
            return
        i0, i1, j0, j1, k0, k1 = (int(b) for b in box)
        v = np.ascontiguousarray(v, dtype=np.float64)
        if v.shape != (3, k1 - k0, j1 - j0, i1 - i0):
            raise ValueError("velocity box shape does not match the box")
        self._inner_v = v
        self.p.inner_v = _dptr(v)
        for q, b in enumerate((i0, i1, j0, j1, k0, k1)):
            self.p.inner_box[q] = b

    def sweep(self, U: np.ndarray, dt: float, axis: int, stats: Stats | None = None) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64).copy()
        assert U.shape == self.shape
        rc = lib().oracle_sweep(C.byref(self.p), _dptr(U), dt, axis, C.byref(stats) if stats else None)
        if rc != 0:
            raise ValueError("oracle_sweep rejected its arguments")
        return U

    def sweep_pencils(self, U: np.ndarray, dt: float, axis: int, j1, j2,
                      stats: Stats | None = None) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64)
        j1 = np.ascontiguousarray(j1, dtype=np.int32)
        j2 = np.ascontiguousarray(j2, dtype=np.int32)
        N = self.p.n[axis]
        out = np.zeros((len(j1), 8, N), dtype=np.float64)
        rc = lib().oracle_sweep_pencils(C.byref(self.p), _dptr(U), dt, axis, len(j1),
                                        j1.ctypes.data_as(C.POINTER(C.c_int)),
                                        j2.ctypes.data_as(C.POINTER(C.c_int)), _dptr(out),
                                        C.byref(stats) if stats else None)
        if rc != 0:
            raise ValueError("oracle_sweep_pencils rejected its arguments")
        return out

    def face_states(self, U: np.ndarray, dt: float, axis: int, j1: int, j2: int):
        """Characteristic mode only: the two primitive states (rho, u, v_t1,
        v_t2, B'_t1, B'_t2, p), after the split multi-D time-centring terms,
        of the linearised interface problem at the faces of pencil (j1, j2)
        of `axis`.  Returns (WL, WR), each [N + 1, 7], for the faces
        -1/2 .. N - 1/2 of the pencil's zones."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        N = self.p.n[axis]
        G = ghosts()
        out = np.zeros((N + 2 * G, 14), dtype=np.float64)
        if lib().oracle_face_states(C.byref(self.p), _dptr(U), dt, axis, j1, j2, _dptr(out)) != 0:
            raise ValueError("oracle_face_states rejected its arguments")
        f = out[G - 1:G + N]
        return f[:, :7].copy(), f[:, 7:].copy()

    def step(self, U: np.ndarray, dt: float, step_index: int, stats: Stats | None = None) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64).copy()
        rc = lib().oracle_step(C.byref(self.p), _dptr(U), dt, step_index, C.byref(stats) if stats else None)
        if rc != 0:
            raise ValueError("oracle_step rejected its arguments")
        return U

    def cfl_dt(self, U: np.ndarray, cfl: float) -> float:
        U = np.ascontiguousarray(U, dtype=np.float64)
        return lib().oracle_cfl_dt(C.byref(self.p), _dptr(U), cfl)

    def totals(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros(8)
        lib().oracle_totals(C.byref(self.p), _dptr(U), _dptr(out))
        return out

    def set_inflow(self, prim) -> None:
        """Fixed state of the inflow ghosts from now on: rho, vx, vy, vz,
        Bx, By, Bz (total field), p (Section IV-A upstream conditions)."""
        for k in range(8):
            self.p.inflow[k] = float(prim[k])

    def dipole(self, r) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(3)
        lib().oracle_dipole(C.byref(self.p), _dptr(r), _dptr(out))
        return out


def set_threads(n: int) -> None:
    """Host threads of the oracle's pencil loops (timing only)."""
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


# ------------------------------------------------- time-dependent driving

def inflow_series_at(times, prims, t):
    """Inflow state of a time series of upstream conditions at time t.

    The paper drives the upstream face with given solar-wind conditions
    (Section IV-A); conditions that vary in time are read here as linear in
    time between knots, held at the first / last knot outside them, and a
    step from t to t + dt takes the state at t + dt/2.
    Written out as that definition: find the knots around t, interpolate."""
    times = np.asarray(times, dtype=np.float64)
    prims = np.asarray(prims, dtype=np.float64).reshape(len(times), 8)
    if t <= times[0]:
        return prims[0].copy()
    if t >= times[-1]:
        return prims[-1].copy()
    k = int(np.searchsorted(times, t, side="right")) - 1
    w = (t - times[k]) / (times[k + 1] - times[k])
    return prims[k] + w * (prims[k + 1] - prims[k])


def step_with_series(prob, U, dt, step_index, t, times, prims, stats=None):
    """One split step from time t with the series' inflow at t + dt/2."""
    prob.set_inflow(inflow_series_at(times, prims, t + 0.5 * dt))
    return prob.step(U, dt, step_index, stats)


# ---------------------------------------------------------------- unit-level

def ppm_edges(a, w, limit=True):
    a = np.ascontiguousarray(a, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros_like(a)
    lib().oracle_ppm_edges(len(a), _dptr(a), _dptr(w), int(limit), _dptr(out))
    return out


def ppm_slopes(a, w, limit=True):
    a = np.ascontiguousarray(a, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros_like(a)
    lib().oracle_ppm_slopes(len(a), _dptr(a), _dptr(w), int(limit), _dptr(out))
    return out


def ppm_parabolas(a, w, flat=None, limit=True, monot=True):
    a = np.ascontiguousarray(a, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    M = len(a)
    out = np.zeros(3 * M)
    fp = None
    if flat is not None:
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        fp = _dptr(flat)
    lib().oracle_ppm_parabolas(M, _dptr(a), _dptr(w), fp, int(limit), int(monot), _dptr(out))
    return out.reshape(3, M)


def par_avg(aL, dA, a6, y, right_part):
    return lib().oracle_par_avg(aL, dA, a6, y, int(right_part))


def flattening(Pt, Pa, un, rho=None):
    """CW84 flattening coefficients of a pencil (rho: density, ones if not
    given; it sets the speed scale of the compression test's margin)."""
    Pt = np.ascontiguousarray(Pt, dtype=np.float64)
    Pa = np.ascontiguousarray(Pa, dtype=np.float64)
    un = np.ascontiguousarray(un, dtype=np.float64)
    rho = np.ones_like(Pt) if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    f = np.zeros_like(Pt)
    lib().oracle_flattening(len(Pt), _dptr(Pt), _dptr(Pa), _dptr(un), _dptr(rho), _dptr(f))
    return f


def mhd7_eigen(rho, p, gamma, Bn, Bt1, Bt2):
    """Eigenvalues (order -f, -A, -s, 0, +s, +A, +f) and right eigenvectors
    (columns) of the Lagrangian 1D MHD system in the primitive variables
    (rho, u, v_t1, v_t2, B_t1, B_t2, p) at a state (total field)."""
    lam = np.zeros(7)
    R = np.zeros(49)
    lib().oracle_mhd7_eigen(rho, p, gamma, Bn, Bt1, Bt2, _dptr(lam), _dptr(R))
    return lam, R.reshape(7, 7)


def trace7(rho, p, gamma, Bn, Bt1, Bt2, par, dt, dm):
    """Face states (right face, left face) of one zone by full
    characteristic tracing; par[7][3] = (aL, dA, a6) per primitive; the
    eigen-structure at (rho, p, Bn, Bt1, Bt2)."""
    par = np.ascontiguousarray(par, dtype=np.float64).reshape(21)
    WL = np.zeros(7)
    WR = np.zeros(7)
    if lib().oracle_trace7(rho, p, gamma, Bn, Bt1, Bt2, _dptr(par), dt, dm, _dptr(WL), _dptr(WR)) != 0:
        raise ValueError("singular eigenvector matrix")
    return WL, WR


def riemann7(WL, WR, gamma, Bn, Bd1=0.0, Bd2=0.0):
    """Face state of the linearised seven-wave Riemann problem (characteristic
    mode) between primitive states W_L, W_R (B'_t components)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    Ws = np.zeros(7)
    if lib().oracle_riemann7(_dptr(WL), _dptr(WR), gamma, Bn, Bd1, Bd2, _dptr(Ws)) != 0:
        raise ValueError("singular eigenvector matrix")
    return Ws


def riemann_normal(PtL, PtR, Pd, uL, uR, CL, CR, gL, gR, tol=1e-12, max_iter=20):
    P = C.c_double()
    u = C.c_double()
    conv = C.c_int()
    it = lib().oracle_riemann_normal(PtL, PtR, Pd, uL, uR, CL, CR, gL, gR, tol, max_iter,
                                     C.byref(P), C.byref(u), C.byref(conv))
    return P.value, u.value, it, bool(conv.value)


def riemann_alfven(rL, rR, sigma, vL, vR, bL, bR):
    v = C.c_double()
    b = C.c_double()
    lib().oracle_riemann_alfven(rL, rR, sigma, vL, vR, bL, bR, C.byref(v), C.byref(b))
    return v.value, b.value


def ghosts() -> int:
    return lib().oracle_ghosts()


# ------------------------------------------------------------ learned guess

MLP_IN, MLP_HID, MLP_OUT = 14, 64, 2


def mlp_num_params() -> int:
    return lib().mlp_num_params()


def mlp_gelu(x: float) -> float:
    return lib().mlp_gelu(float(x))


def mlp_gelu_grad(x: float) -> float:
    return lib().mlp_gelu_grad(float(x))


def mlp_forward(theta, X):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    out = np.zeros((n, MLP_OUT))
    lib().mlp_forward(_dptr(theta), n, _dptr(X), _dptr(out), None, None)
    return out


def mlp_loss_grad(theta, X, Y):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    g = np.zeros(mlp_num_params())
    loss = lib().mlp_loss_grad(_dptr(theta), X.shape[0], _dptr(X), _dptr(Y), _dptr(g))
    return loss, g


def mlp_adam(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on theta, m, v (float64 arrays)."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    lib().mlp_adam(_dptr(theta), _dptr(m), _dptr(v), _dptr(grad), int(t), lr, b1, b2, eps)


def mlp_unpack(theta):
    """Views (W1 [14,64], b1, W2 [64,64], b2, W3 [64,2], b3) into theta."""
    o = 0
    out = []
    for shape in ((MLP_IN, MLP_HID), (MLP_HID,), (MLP_HID, MLP_HID), (MLP_HID,), (MLP_HID, MLP_OUT), (MLP_OUT,)):
        n = int(np.prod(shape))
        out.append(theta[o:o + n].reshape(shape))
        o += n
    return out
