"""Operation count of the method per zone-sweep -- TEST INFRASTRUCTURE ONLY.

Builds `oracle/flop_count.cpp` (the oracle's own source compiled with a
counting FP64 value type; results unchanged) and runs the oracle's pencil
sweep on sampled pencils of the inflow-dipole start state (256 x 192 x 192
stretched grid, Section IV-A set-up) with the single-precision Newton
tolerance, one OpenMP thread.  Prints and returns the operations per
zone-sweep: additions and subtractions, multiplications, divisions, square
roots (their sum is the floating-point operation count), plus comparisons and
selections (min / max / |x|), which are not counted as floating-point
operations.  Ghost zones are part of what the oracle computes per pencil, so
the per-zone figure is the pencil's count divided by its interior zones.

    python oracle/flop_count.py            # writes nothing; prints the JSON line
"""
from __future__ import annotations

import ctypes as C
import json
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

LIB_PATH = os.path.join(_HERE, "libppmlr_oracle_count.so")
SRC = os.path.join(_HERE, "flop_count.cpp")
ORACLE_SRC = os.path.join(_HERE, "ppmlr_oracle.c")


def build() -> str:
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fpermissive", "-w", "-ffp-contract=off", "-fopenmp",
                           "-fPIC", "-shared", "-o", tmp, SRC])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(os.path.getmtime(SRC),
                                                                                os.path.getmtime(ORACLE_SRC)):
            build()
        from oracle import oracle as O
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.oracle_sweep_pencils.argtypes = [C.POINTER(O.Problem), dp, C.c_double, C.c_int, C.c_int,
                                           C.POINTER(C.c_int), C.POINTER(C.c_int), dp, C.POINTER(O.Stats)]
        L.oracle_sweep_pencils.restype = C.c_int
        L.oracle_cfl_dt.argtypes = [C.POINTER(O.Problem), dp, C.c_double]
        L.oracle_cfl_dt.restype = C.c_double
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_count_reset.argtypes = []
        L.oracle_count_get.argtypes = [C.POINTER(C.c_longlong)]
        _lib = L
    return _lib


def counted_sweep_pencils(prob, U, dt, axis, j1, j2):
    """The counting build's pencil sweep: (output like OracleProblem.sweep_pencils,
    the six operation counts)."""
    from oracle import oracle as O
    L = lib()
    L.oracle_set_threads(1)
    U = np.ascontiguousarray(U, dtype=np.float64)
    j1 = np.ascontiguousarray(j1, dtype=np.int32)
    j2 = np.ascontiguousarray(j2, dtype=np.int32)
    out = np.zeros((len(j1), 8, prob.p.n[axis]), dtype=np.float64)
    L.oracle_count_reset()
    rc = L.oracle_sweep_pencils(C.byref(prob.p), U.ctypes.data_as(C.POINTER(C.c_double)), dt, axis, len(j1),
                                j1.ctypes.data_as(C.POINTER(C.c_int)), j2.ctypes.data_as(C.POINTER(C.c_int)),
                                out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(O.Stats()))
    if rc != 0:
        raise ValueError("oracle_sweep_pencils rejected its arguments")
    cnt = (C.c_longlong * 6)()
    L.oracle_count_get(cnt)
    return out, list(cnt)


def count_inflow_dipole(pencils=64, seed=0, tol=1e-6, cfl=0.4):
    """Operations per zone-sweep on `pencils` random pencils per axis of the
    256 x 192 x 192 inflow-dipole start state, at the CFL dt."""
    from oracle import oracle as O
    from paper_1607_02214_amd import inputs as I
    setup = I.c2_setup()
    prob = O.OracleProblem(setup.faces, bc_lo=setup.bc_lo, bc_hi=setup.bc_hi, dip_moment=setup.moment,
                           dip_dir=setup.direction, inflow=setup.inflow, r_inner=setup.r_inner,
                           inner_rho=setup.inner_rho, inner_p=setup.inner_p, p_floor=setup.p_floor, tol=tol)
    dt = prob.cfl_dt(setup.U, cfl)
    n = [len(f) - 1 for f in setup.faces]
    rng = np.random.default_rng(seed)
    tot = np.zeros(6, dtype=np.int64)
    zs = 0
    for axis in range(3):
        n1, n2 = n[(axis + 1) % 3], n[(axis + 2) % 3]
        j1 = rng.integers(0, n1, pencils)
        j2 = rng.integers(0, n2, pencils)
        _, c = counted_sweep_pencils(prob, setup.U, dt, axis, j1, j2)
        tot += np.array(c, dtype=np.int64)
        zs += pencils * n[axis]
    per = tot / zs
    names = ["add_sub", "mul", "div", "sqrt", "cmp", "select"]
    res = {k: round(float(v), 1) for k, v in zip(names, per)}
    res["flops_per_zone_sweep"] = round(float(per[:4].sum()), 1)
    res["sample"] = (f"{pencils} random pencils per axis of the 256x192x192 inflow-dipole start state, "
                     f"Newton tol {tol:g}, CFL {cfl} dt ({zs} zone-sweeps)")
    return res


if __name__ == "__main__":
    print(json.dumps(count_inflow_dipole()))
