"""Python binding of the C ABI in include/ppmlr.h (ctypes; argument
marshalling only -- every step of the sweep runs in the HIP library).

PyTorch provides device memory and streams: a state is a contiguous CUDA
(HIP) tensor of shape [8, nz, ny, nx], dtype float32 or float64, holding
(rho, m_x, m_y, m_z, B'_x, B'_y, B'_z, E').

The library must be built (``python -m paper_1607_02214_amd.build`` or
``__graft_entry__.build()``); without it the first call into the library
raises ImportError (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PPMLR_LIB names another build of the same sources
LIB_PATH = os.environ.get("PPMLR_LIB") or os.path.join(_HERE, "libppmlr.so")

PPMLR_OK = 0
PPMLR_EINVAL = -1
PPMLR_ECFL = -2
PPMLR_ERIEMANN = -3
PPMLR_ENONPHYS = -4
PPMLR_EDEVICE = -5
PPMLR_ENOMEM = -6
PERIODIC, OUTFLOW, INFLOW = 0, 1, 2
F32, F64 = 0, 1
GHOSTS = 7
GUESS_PLAIN, GUESS_LEARNED, GUESS_HARVEST = 0, 1, 2
TRACE_TWO_FAMILY, TRACE_CHARACTERISTIC = 0, 1
MLP_PARAMS = 5250
RECORD_FLOATS = 28

_STATUS_NAMES = {0: "PPMLR_OK", -1: "PPMLR_EINVAL", -2: "PPMLR_ECFL", -3: "PPMLR_ERIEMANN",
                 -4: "PPMLR_ENONPHYS", -5: "PPMLR_EDEVICE", -6: "PPMLR_ENOMEM"}


class PPMLRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [
        ("flatten", C.c_int),
        ("janhunen", C.c_int),
        ("max_iter", C.c_int),
        ("tol_f64", C.c_double),
        ("tol_f32", C.c_double),
        ("p_floor", C.c_double),
        ("collect_stats", C.c_int),
        ("debug_cfl", C.c_int),
        ("tracing", C.c_int),
    ]


class Grid(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("bc_lo", C.c_int * 3),
        ("bc_hi", C.c_int * 3),
        ("r_inner", C.c_double),
    ]


class IonoParams(C.Structure):
    _fields_ = [
        ("n_theta", C.c_int),
        ("n_phi", C.c_int),
        ("r_shell", C.c_double),
        ("r_fac", C.c_double),
        ("sigma", C.c_double),
    ]


class Coords(C.Structure):
    _fields_ = [("faces", C.POINTER(C.c_double) * 3)]


class State(C.Structure):
    _fields_ = [("u", C.c_void_p), ("dtype", C.c_int), ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [
        ("iters_hist", C.c_longlong * 32),
        ("floor_hits", C.c_longlong),
        ("nonconverged", C.c_longlong),
        ("nonphys", C.c_longlong),
        ("guess_faces", C.c_longlong),
        ("guess_fallbacks", C.c_longlong),
    ]

    def as_dict(self):
        return {"iters_hist": list(self.iters_hist), "floor_hits": self.floor_hits,
                "nonconverged": self.nonconverged, "nonphys": self.nonphys,
                "guess_faces": self.guess_faces, "guess_fallbacks": self.guess_fallbacks}


# exported symbols and their signatures (mirrors include/ppmlr.h)
_P = C.c_void_p
_dp = C.POINTER(C.c_double)
SIGNATURES = {
    "ppmlr_default_options": (None, [C.POINTER(Options)]),
    "ppmlr_create": (C.c_int, [C.POINTER(Grid), C.c_double, C.POINTER(Coords), C.POINTER(Options), C.POINTER(_P)]),
    "ppmlr_destroy": (None, [_P]),
    "ppmlr_last_error": (C.c_char_p, [_P]),
    "ppmlr_set_dipole": (C.c_int, [_P, C.c_double, _dp]),
    "ppmlr_set_background": (C.c_int, [_P, _dp]),
    "ppmlr_set_inflow": (C.c_int, [_P, _dp]),
    "ppmlr_set_inner": (C.c_int, [_P, C.c_double, C.c_double]),
    "ppmlr_iono_default_params": (None, [C.POINTER(IonoParams)]),
    "ppmlr_ionosphere_couple": (C.c_int, [_P, C.POINTER(State), C.POINTER(IonoParams), C.c_void_p, C.c_void_p]),
    "ppmlr_ionosphere_detach": (C.c_int, [_P]),
    "ppmlr_sweep": (C.c_int, [_P, C.POINTER(State), C.c_double, C.c_int]),
    "ppmlr_step": (C.c_int, [_P, C.POINTER(State), C.c_double]),
    "ppmlr_set_step_index": (C.c_int, [_P, C.c_longlong]),
    "ppmlr_get_step_index": (C.c_int, [_P, C.POINTER(C.c_longlong)]),
    "ppmlr_cfl_dt": (C.c_int, [_P, C.POINTER(State), C.c_double, _dp]),
    "ppmlr_advance": (C.c_int, [_P, C.POINTER(State), C.c_int, C.c_double]),
    "ppmlr_time": (C.c_int, [_P, C.POINTER(State), _dp]),
    "ppmlr_totals": (C.c_int, [_P, C.POINTER(State), _dp]),
    "ppmlr_stats": (C.c_int, [_P, _P, C.POINTER(Stats)]),
    "ppmlr_reset_stats": (C.c_int, [_P, _P]),
    "ppmlr_status_check": (C.c_int, [_P, _P]),
    "ppmlr_set_profiling": (C.c_int, [_P, C.c_int]),
    "ppmlr_kernel_times": (C.c_int, [_P, _dp, C.POINTER(C.c_longlong)]),
    "ppmlr_set_tile": (C.c_int, [_P, C.c_int, C.c_int]),
    "ppmlr_get_tile": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "ppmlr_set_segments": (C.c_int, [_P, C.c_int, C.c_int]),
    "ppmlr_set_inflow_series": (C.c_int, [_P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ppmlr_set_segment_order": (C.c_int, [_P, C.c_int, C.c_int]),
    "ppmlr_get_segment_order": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int)]),
    "ppmlr_get_segments": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "ppmlr_autotune": (C.c_int, [_P, C.POINTER(State), C.c_int, C.POINTER(C.c_int)]),
    "ppmlr_ensemble_run": (C.c_int, [C.POINTER(_P), C.POINTER(C.POINTER(State)), C.c_int, C.c_int, C.c_double,
                                     C.c_int, C.POINTER(C.c_int)]),
    "ppmlr_ensemble_run_noalloc": (C.c_int, [C.POINTER(_P), C.POINTER(C.POINTER(State)), C.c_int, C.c_int,
                                             C.c_double, C.c_int, C.POINTER(C.c_int)]),
    "ppmlr_set_ensemble_launch": (C.c_int, [C.c_int]),
    "ppmlr_set_ensemble_barrier_limit": (C.c_int, [C.c_longlong]),
    "ppmlr_ensemble_autotune": (C.c_int, [C.POINTER(_P), C.POINTER(C.POINTER(State)), C.c_int, C.c_int, C.c_double,
                                          C.POINTER(C.c_int)]),
    "ppmlr_set_guess": (C.c_int, [_P, C.c_int, _P, _P]),
    "ppmlr_set_gate": (C.c_int, [_P, C.c_double, C.c_double]),
    "ppmlr_set_harvest": (C.c_int, [_P, _P, C.c_longlong, _P]),
    "ppmlr_mlp_create": (C.c_int, [C.c_int, C.POINTER(_P)]),
    "ppmlr_mlp_destroy": (None, [_P]),
    "ppmlr_mlp_last_error": (C.c_char_p, [_P]),
    "ppmlr_mlp_forward": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, _P, C.c_int, _P]),
    "ppmlr_mlp_grad": (C.c_int, [_P, _P, _P, C.c_int, _P, C.c_int, C.c_int, _P, _P, _P]),
    "ppmlr_mlp_train_step": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, _P, C.c_int, C.c_int, C.c_int, C.c_float,
                                       C.c_float, C.c_float, C.c_float, _P, _P]),
}

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def iono_default_params() -> IonoParams:
    p = IonoParams()
    lib().ppmlr_iono_default_params(C.byref(p))
    return p


def default_options() -> Options:
    o = Options()
    lib().ppmlr_default_options(C.byref(o))
    return o


def _d3(v):
    return (C.c_double * 3)(*[float(x) for x in v])


class Context:
    """Owns one ppmlr_ctx (grid tables, counters, device scalars)."""

    def __init__(self, faces, bc_lo=(PERIODIC,) * 3, bc_hi=(PERIODIC,) * 3, gamma=5.0 / 3.0,
                 r_inner=0.0, options: Options | None = None, **opt_overrides):
        self._faces = [np.ascontiguousarray(f, dtype=np.float64) for f in faces]
        g = Grid()
        cd = Coords()
        for a in range(3):
            g.n[a] = len(self._faces[a]) - 1
            g.bc_lo[a] = int(bc_lo[a])
            g.bc_hi[a] = int(bc_hi[a])
            cd.faces[a] = self._faces[a].ctypes.data_as(_dp)
        g.r_inner = float(r_inner)
        opt = options if options is not None else default_options()
        known = {f[0] for f in Options._fields_}
        for k, v in opt_overrides.items():
            if k not in known:
                raise TypeError(f"unknown option {k!r}")
            setattr(opt, k, v)
        self.options = opt
        self.n = tuple(g.n)
        h = _P()
        rc = lib().ppmlr_create(C.byref(g), float(gamma), C.byref(cd), C.byref(opt), C.byref(h))
        if rc != PPMLR_OK:
            raise PPMLRError(rc, "ppmlr_create rejected the grid or options")
        self.h = h

    # -- helpers
    def _chk(self, rc):
        if rc != PPMLR_OK:
            msg = lib().ppmlr_last_error(self.h)
            raise PPMLRError(rc, msg.decode() if msg else "")
        return rc

    @staticmethod
    def state(u, stream=None) -> State:
        import torch
        if not u.is_cuda or not u.is_contiguous():
            raise ValueError("state must be a contiguous device tensor")
        if u.dtype == torch.float32:
            dt = F32
        elif u.dtype == torch.float64:
            dt = F64
        else:
            raise ValueError("state dtype must be float32 or float64")
        if stream is None:
            stream = torch.cuda.current_stream(u.device).cuda_stream
        return State(C.c_void_p(u.data_ptr()), dt, C.c_void_p(stream))

    def _st(self, u, stream):
        if tuple(u.shape) != (8, self.n[2], self.n[1], self.n[0]):
            raise ValueError(f"state shape {tuple(u.shape)} does not match the grid {self.n}")
        return self.state(u, stream)

    # -- ABI wrappers (same names without the prefix)
    def set_dipole(self, moment, direction=(0.0, 0.0, -1.0)):
        return self._chk(lib().ppmlr_set_dipole(self.h, float(moment), _d3(direction)))

    def set_background(self, b):
        return self._chk(lib().ppmlr_set_background(self.h, _d3(b)))

    def set_inflow(self, prim):
        arr = (C.c_double * 8)(*[float(x) for x in prim])
        return self._chk(lib().ppmlr_set_inflow(self.h, arr))

    def set_inflow_series(self, times, prims):
        """Inflow state as a time series (knot times, [n, 8] primitive
        states); an empty series returns to the constant inflow."""
        import numpy as np
        t = np.ascontiguousarray(times, dtype=np.float64).ravel()
        p = np.ascontiguousarray(prims, dtype=np.float64).reshape(len(t), 8) if len(t) else np.zeros((0, 8))
        p = np.ascontiguousarray(p)
        dp = C.POINTER(C.c_double)
        return self._chk(lib().ppmlr_set_inflow_series(self.h, len(t), t.ctypes.data_as(dp) if len(t) else None,
                                                       p.ctypes.data_as(dp) if len(t) else None))

    def set_inner(self, rho, p):
        return self._chk(lib().ppmlr_set_inner(self.h, float(rho), float(p)))

    def ionosphere_couple(self, u, params: IonoParams | None = None, jr=None, phi=None, stream=None, **over):
        """One ionosphere coupling of state u (see ppmlr_ionosphere_couple):
        the context keeps the drift of the reset zones for later sweeps.  jr,
        phi: optional device float64 tensors [2, n_theta, n_phi] receiving the
        shell current and potential."""
        prm = params if params is not None else iono_default_params()
        known = {f[0] for f in IonoParams._fields_}
        for k, v in over.items():
            if k not in known:
                raise TypeError(f"unknown ionosphere parameter {k!r}")
            setattr(prm, k, v)
        shape = (2, prm.n_theta, prm.n_phi)
        ptrs = []
        for t in (jr, phi):
            if t is None:
                ptrs.append(None)
                continue
            import torch
            if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape:
                raise ValueError(f"ionosphere outputs are contiguous device float64 tensors {shape}")
            ptrs.append(C.c_void_p(t.data_ptr()))
        st = self._st(u, stream)
        return self._chk(lib().ppmlr_ionosphere_couple(self.h, C.byref(st), C.byref(prm), ptrs[0], ptrs[1]))

    def ionosphere_detach(self):
        return self._chk(lib().ppmlr_ionosphere_detach(self.h))

    def sweep(self, u, dt, axis, stream=None):
        st = self._st(u, stream)
        return self._chk(lib().ppmlr_sweep(self.h, C.byref(st), float(dt), int(axis)))

    def step(self, u, dt, stream=None):
        st = self._st(u, stream)
        return self._chk(lib().ppmlr_step(self.h, C.byref(st), float(dt)))

    def set_step_index(self, k):
        return self._chk(lib().ppmlr_set_step_index(self.h, int(k)))

    def get_step_index(self):
        v = C.c_longlong()
        self._chk(lib().ppmlr_get_step_index(self.h, C.byref(v)))
        return v.value

    def cfl_dt(self, u, cfl, stream=None):
        st = self._st(u, stream)
        out = C.c_double()
        self._chk(lib().ppmlr_cfl_dt(self.h, C.byref(st), float(cfl), C.byref(out)))
        return out.value

    def advance(self, u, nsteps, cfl, stream=None):
        st = self._st(u, stream)
        return self._chk(lib().ppmlr_advance(self.h, C.byref(st), int(nsteps), float(cfl)))

    def time(self, u=None, stream=None):
        out = C.c_double()
        st = self._st(u, stream) if u is not None else None
        self._chk(lib().ppmlr_time(self.h, C.byref(st) if st is not None else None, C.byref(out)))
        return out.value

    def totals(self, u, stream=None):
        st = self._st(u, stream)
        out = (C.c_double * 8)()
        self._chk(lib().ppmlr_totals(self.h, C.byref(st), out))
        return np.array(out[:])

    def stats(self, stream=None):
        s = Stats()
        self._chk(lib().ppmlr_stats(self.h, C.c_void_p(stream) if stream else None, C.byref(s)))
        return s.as_dict()

    def reset_stats(self, stream=None):
        return self._chk(lib().ppmlr_reset_stats(self.h, C.c_void_p(stream) if stream else None))

    def status_check(self, stream=None) -> int:
        """Returns the status code (does not raise)."""
        return lib().ppmlr_status_check(self.h, C.c_void_p(stream) if stream else None)

    def set_profiling(self, enable=True):
        return self._chk(lib().ppmlr_set_profiling(self.h, int(bool(enable))))

    def kernel_times(self):
        ms = (C.c_double * 3)()
        n = (C.c_longlong * 3)()
        self._chk(lib().ppmlr_kernel_times(self.h, ms, n))
        return list(ms), list(n)

    def set_tile(self, axis, pencils):
        return self._chk(lib().ppmlr_set_tile(self.h, int(axis), int(pencils)))

    def get_tile(self, axis, dtype=F32):
        v = C.c_int()
        self._chk(lib().ppmlr_get_tile(self.h, int(axis), int(dtype), C.byref(v)))
        return v.value

    def set_segments(self, axis, segments):
        return self._chk(lib().ppmlr_set_segments(self.h, int(axis), int(segments)))

    def set_segment_order(self, axis, order):
        return self._chk(lib().ppmlr_set_segment_order(self.h, int(axis), int(order)))

    def get_segment_order(self, axis):
        v = C.c_int()
        self._chk(lib().ppmlr_get_segment_order(self.h, int(axis), C.byref(v)))
        return v.value

    def get_segments(self, axis, dtype=F32):
        v = C.c_int()
        self._chk(lib().ppmlr_get_segments(self.h, int(axis), int(dtype), C.byref(v)))
        return v.value

    def autotune(self, u, reps=3, stream=None):
        st = self._st(u, stream)
        t = (C.c_int * 3)()
        self._chk(lib().ppmlr_autotune(self.h, C.byref(st), int(reps), t))
        return list(t)

    def set_guess(self, mode, theta=None, stream=None):
        """mode: GUESS_PLAIN, GUESS_LEARNED (theta: device float32 tensor of
        MLP_PARAMS values) or GUESS_HARVEST."""
        ptr = None
        if theta is not None:
            _check_f32(theta, (MLP_PARAMS,))
            ptr = C.c_void_p(theta.data_ptr())
        return self._chk(lib().ppmlr_set_guess(self.h, int(mode), ptr, _stream(theta, stream)))

    def set_gate(self, rel_p, rel_u):
        return self._chk(lib().ppmlr_set_gate(self.h, float(rel_p), float(rel_u)))

    def set_harvest(self, records=None, count=None):
        """records: device float32 tensor [capacity, RECORD_FLOATS]; count: device
        int64 tensor of one element (zeroed by the caller).  None detaches."""
        if records is None:
            return self._chk(lib().ppmlr_set_harvest(self.h, None, 0, None))
        import torch
        if records.dtype != torch.float32 or not records.is_cuda or not records.is_contiguous() \
                or records.dim() != 2 or records.shape[1] != RECORD_FLOATS:
            raise ValueError("records must be a contiguous device float32 tensor [capacity, 28]")
        if count is None or count.dtype != torch.int64 or not count.is_cuda or count.numel() != 1:
            raise ValueError("count must be a device int64 tensor of one element")
        return self._chk(lib().ppmlr_set_harvest(self.h, C.c_void_p(records.data_ptr()), int(records.shape[0]),
                                                 C.c_void_p(count.data_ptr())))

    def last_error(self):
        m = lib().ppmlr_last_error(self.h)
        return m.decode() if m else ""

    def close(self):
        if getattr(self, "h", None):
            lib().ppmlr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ensemble_args(ctxs, states, stream):
    n = len(ctxs)
    if n != len(states) or n == 0:
        raise ValueError("one state per context")
    hs = (_P * n)(*[c.h for c in ctxs])
    sts = [c._st(u, stream) for c, u in zip(ctxs, states)]
    sp = (C.POINTER(State) * n)(*[C.pointer(x) for x in sts])
    return n, hs, sts, sp


def ensemble_run(ctxs, states, steps, cfl, block=0, stream=None, noalloc=False):
    """Advance every member (context, state tensor) by `steps` split steps,
    all members in each launch (one launch per sweep, or one per call in the
    persistent form, see set_ensemble_launch); returns the per-member status
    codes.  noalloc: call ppmlr_ensemble_run_noalloc (work tables in the
    library's fixed device array; at most 64 members)."""
    n, hs, sts, sp = _ensemble_args(ctxs, states, stream)
    per = (C.c_int * n)()
    fn = lib().ppmlr_ensemble_run_noalloc if noalloc else lib().ppmlr_ensemble_run
    rc = fn(hs, sp, n, int(steps), float(cfl), int(block), per)
    if rc != PPMLR_OK:
        msg = lib().ppmlr_last_error(ctxs[0].h)
        raise PPMLRError(rc, msg.decode() if msg else "")
    return list(per)


ENSEMBLE_PERSISTENT, ENSEMBLE_PER_SWEEP = 0, 1


def set_ensemble_launch(mode):
    """Launch form of the ensemble calls: ENSEMBLE_PER_SWEEP (one launch per
    sweep, the default) or ENSEMBLE_PERSISTENT (one launch per call)."""
    rc = lib().ppmlr_set_ensemble_launch(int(mode))
    if rc != PPMLR_OK:
        raise PPMLRError(rc, "bad ensemble launch mode")


def set_ensemble_barrier_limit(polls):
    """Polls of a grid-barrier wait of the persistent ensemble launch before
    it gives up (default 4194304; 0: every wait gives up at once)."""
    rc = lib().ppmlr_set_ensemble_barrier_limit(int(polls))
    if rc != PPMLR_OK:
        raise PPMLRError(rc, "bad barrier poll limit")


def ensemble_autotune(ctxs, states, reps=1, cfl=0.4, stream=None):
    """Pick the ensemble workgroup size (256 / 512 / 1024) and segment length
    (whole pencils or about 96 / 64 / 48 / 32 interior zones) by timing `reps`
    steps on copies of the states; sets the members' segments and returns the
    workgroup size."""
    n, hs, sts, sp = _ensemble_args(ctxs, states, stream)
    b = C.c_int()
    rc = lib().ppmlr_ensemble_autotune(hs, sp, n, int(reps), float(cfl), C.byref(b))
    if rc != PPMLR_OK:
        msg = lib().ppmlr_last_error(ctxs[0].h)
        raise PPMLRError(rc, msg.decode() if msg else "")
    return b.value


def _stream(t, stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    dev = t.device if t is not None else torch.device("cuda")
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check_f32(t, shape=None, ld=None):
    """Device float32 tensor: a contiguous vector of the given shape, or (ld)
    a row-major matrix with at least ld columns (row stride free)."""
    import torch
    if t.dtype != torch.float32 or not t.is_cuda:
        raise ValueError("expected a device float32 tensor")
    if shape is not None and (tuple(t.shape) != tuple(shape) or not t.is_contiguous()):
        raise ValueError(f"expected a contiguous tensor of shape {shape}, got {tuple(t.shape)}")
    if ld is not None and (t.dim() != 2 or t.shape[1] < ld or t.stride(1) != 1):
        raise ValueError(f"expected a row-major 2-D tensor with at least {ld} columns")


class MLP:
    """Training workspace of the learned Riemann guess (ppmlr_mlp)."""

    def __init__(self, max_batch):
        h = _P()
        rc = lib().ppmlr_mlp_create(int(max_batch), C.byref(h))
        if rc != PPMLR_OK:
            raise PPMLRError(rc, "ppmlr_mlp_create failed")
        self.h = h
        self.max_batch = int(max_batch)

    def _chk(self, rc):
        if rc != PPMLR_OK:
            msg = lib().ppmlr_mlp_last_error(self.h)
            raise PPMLRError(rc, msg.decode() if msg else "")
        return rc

    def forward(self, theta, X, out=None, stream=None):
        """X: [n, >=14] device float32 -> [n, 2]."""
        import torch
        _check_f32(theta, (MLP_PARAMS,))
        _check_f32(X, ld=14)
        n = X.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device=X.device)
        _check_f32(out, ld=2)
        self._chk(lib().ppmlr_mlp_forward(self.h, C.c_void_p(theta.data_ptr()), C.c_void_p(X.data_ptr()),
                                          int(X.stride(0)), int(n), C.c_void_p(out.data_ptr()), int(out.stride(0)),
                                          _stream(X, stream)))
        return out

    def grad(self, theta, X, Y, stream=None):
        """Returns (gradient [MLP_PARAMS], loss [1]) device tensors."""
        import torch
        _check_f32(theta, (MLP_PARAMS,))
        _check_f32(X, ld=14)
        _check_f32(Y, ld=2)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        self._chk(lib().ppmlr_mlp_grad(self.h, C.c_void_p(theta.data_ptr()), C.c_void_p(X.data_ptr()),
                                       int(X.stride(0)), C.c_void_p(Y.data_ptr()), int(Y.stride(0)), int(X.shape[0]),
                                       C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr()), _stream(X, stream)))
        return g, loss

    def train_step(self, theta, m, v, X, Y, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss=None, stream=None):
        """One Adam step in place on theta, m, v (device float32); loss: optional
        device float32 tensor of one element receiving the batch loss."""
        for a in (theta, m, v):
            _check_f32(a, (MLP_PARAMS,))
        _check_f32(X, ld=14)
        _check_f32(Y, ld=2)
        lp = C.c_void_p(loss.data_ptr()) if loss is not None else None
        return self._chk(lib().ppmlr_mlp_train_step(
            self.h, C.c_void_p(theta.data_ptr()), C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()),
            C.c_void_p(X.data_ptr()), int(X.stride(0)), C.c_void_p(Y.data_ptr()), int(Y.stride(0)), int(X.shape[0]),
            int(t), float(lr), float(beta1), float(beta2), float(eps), lp, _stream(X, stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().ppmlr_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
