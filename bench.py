#!/usr/bin/env python3
"""Benchmark of the split PPMLR-MHD step on one MI355X.

Workload (the inflow/dipole run of the paper's Section IV-A set-up at the
configured size): 256 x 192 x 192 stretched Cartesian grid (cell sizes
0.25 .. 2 R_E, growth 1.03), solar wind n = 5 cm^-3, v = 400 km/s,
T = 1e5 K, IMF Bz = -5 nT entering at x_max, dipole of moment 8e15 T m^3,
fixed inner boundary r < 3 R_E, FP32 state with FP64 dt reduction.  One step
= dt from the fused signal-speed maximum + x, y, z sweeps (z, y, x on odd
steps); the state stays resident in HBM.

Prints one JSON line: zone-updates/s (zones x steps / wall time), the
roofline of the dominant sweep kernel (algorithmic bytes: 8 conserved
variables read and written once per sweep), and the FP64 CPU oracle timed on
a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3          # MI355X vector FP32 with packed FP32 instructions (not generated here)
FP32_UNPACKED_TFLOPS = 78.6       # the same without packed instructions: 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz
# Floating-point operations of one zone-sweep of the method (additions and
# subtractions, multiplications, divisions, square roots), counted by the
# oracle's instrumented build (oracle/flop_count.py: 64 random pencils per
# axis of this workload's start state, FP32 Newton tolerance; the plain
# oracle recomputes the width weights that the kernels share between the 7
# reconstructed variables, so this is above what the kernels execute).
FLOPS_PER_ZONE_SWEEP = 1875.8
FLOPS_SOURCE = "oracle instrumented count (oracle/flop_count.py, 64 pencils per axis of the start state)"
# What the kernels execute: FP32 operations per lane (ADD + MUL + TRANS + 2 FMA)
# of the y sweep from its VALU counters (committed counter summary).
KERNEL_FP32_OPS_PER_LANE = 1119.0
PROFILES = os.path.join(ROOT, "profiles")
# Vector-instruction issue: one wave64 VALU instruction per CU per cycle
# (256 CUs at 2.4 GHz); FP32 transcendentals (rcp, sqrt, rsq) issue at half
# that rate, so each counts twice in the issue-cycle figure.
VALU_ISSUE_PEAK_G = 256 * 2.4


def kernel_source_hash() -> str:
    """Hash of the sweep kernel's HIP sources (the sweep body and the headers
    it includes) with comments and whitespace removed: a comment edit does
    not make the committed counters of the sweep stale, any code edit does.
    The tile shape the counters were taken with is recorded beside them."""
    import re
    h = hashlib.sha256()
    for rel in ("paper_1607_02214_amd/csrc/ppmlr_sweep.hpp", "paper_1607_02214_amd/csrc/ppmlr_mlp.hpp",
                "paper_1607_02214_amd/csrc/ppmlr_char.hpp"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(dtype: str):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, valid only for the kernel source it was taken from."""
    path = os.path.join(PROFILES, f"traffic_sweep_inflow_dipole_{dtype}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None, d.get("source_hash")
    return d, d.get("source_hash")


def shape_record(prof, axis, shape):
    """The record of a committed counter summary taken with the tile shape
    `shape` = (pencils per workgroup, segments, segment order) on `axis`: the
    summary's own shape or one of its alternates; None if none matches (its
    bytes and instruction counts then describe other launches)."""
    if not prof:
        return None
    for rec in [prof] + list(prof.get("alternates", [])):
        if (rec["tiles"][axis], rec["segments"][axis], rec["segment_order"][axis]) == tuple(shape):
            return rec
    return None


def cpu_baseline(setup, dt, seconds_target=15.0, seed=0):
    """FP64 oracle on a bounded sample of pencils of the same state (all three
    sweep directions, equal pencil counts), timed on the host cores."""
    import numpy as np
    from oracle import oracle as O

    prob = O.OracleProblem(setup.faces, bc_lo=setup.bc_lo, bc_hi=setup.bc_hi, dip_moment=setup.moment,
                           dip_dir=setup.direction, inflow=setup.inflow, r_inner=setup.r_inner,
                           inner_rho=setup.inner_rho, inner_p=setup.inner_p, p_floor=setup.p_floor)
    rng = np.random.default_rng(seed)
    n = [len(f) - 1 for f in setup.faces]
    U = setup.U

    def sample(npen):
        zs = 0
        t0 = time.perf_counter()
        for axis in range(3):
            n1, n2 = n[(axis + 1) % 3], n[(axis + 2) % 3]
            j1 = rng.integers(0, n1, npen)
            j2 = rng.integers(0, n2, npen)
            prob.sweep_pencils(U, dt, axis, j1, j2)
            zs += npen * n[axis]
        return zs, time.perf_counter() - t0

    sample(64)                               # warm-up (thread start-up)
    zs = 0
    el = 0.0
    chunks = 0
    while el < seconds_target:
        z, e = sample(2048)
        zs += z
        el += e
        chunks += 1
    threads = O.get_threads()
    # one whole split step of the same state (every pencil of the three
    # sweeps, the oracle's own whole-grid path), when the sampled rate puts
    # it under ~8 s (the whole-grid path ran up to 3x slower than that)
    el_step = None
    if 3.0 * float(np.prod(n)) / (zs / el) < 8.0:
        t0 = time.perf_counter()
        prob.step(U, dt, 0)
        el_step = time.perf_counter() - t0
    # the same sample kind on one core (bounded to ~5 s)
    O.set_threads(1)
    zs1, el1 = 0, 0.0
    while el1 < seconds_target / 3.0:
        z, e = sample(128)
        zs1 += z
        el1 += e
    O.set_threads(threads)
    # the small periodic case in full: 32^3 zones, 20 FP64 steps at CFL 0.4
    from paper_1607_02214_amd import inputs as I
    U1, faces1 = I.c1_state(n=32)
    prob1 = O.OracleProblem(faces1)
    t0 = time.perf_counter()
    for s in range(20):
        U1 = prob1.step(U1, prob1.cfl_dt(U1, 0.4), s)
    el_c1 = time.perf_counter() - t0
    return {
        "value": zs / el / 3.0,
        "unit": "zone-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{chunks} x 2048 random pencils per sweep direction of the 256x192x192 inflow-dipole start "
                  f"state ({zs} zone-sweeps, {el:.1f} s, FP64, OpenMP over pencils); zone-updates = zone-sweeps / 3",
        "whole_step": None if el_step is None else {
            "value": float(np.prod(n)) / el_step, "unit": "zone-updates/s", "cores": threads,
            "sample": f"one whole split step of the {n[0]}x{n[1]}x{n[2]} start state ({el_step:.1f} s)"},
        "single_core": {"value": zs1 / el1 / 3.0, "unit": "zone-updates/s", "cores": 1,
                        "sample": f"128-pencil samples, {zs1} zone-sweeps, {el1:.1f} s"},
        "periodic_32cubed_full": {"value": 32 ** 3 * 20 / el_c1, "unit": "zone-updates/s", "cores": threads,
                                  "sample": f"32^3 periodic box, 20 whole FP64 steps with the CFL 0.4 dt "
                                            f"({el_c1:.2f} s)"},
    }


def series_leg(args, setup, make_ctx, shape_ctx):
    """The FP32 run driven by a seeded synthetic solar-wind time series at
    the inflow face (9 knots over the run's simulated time), with the plain
    run's tile shape; timed like the plain run."""
    import numpy as np
    import torch
    from paper_1607_02214_amd import inputs as I

    ctx = make_ctx()
    for a in range(3):
        ctx.set_tile(a, 1)
        ctx.set_segments(a, shape_ctx.get_segments(a))
        ctx.set_tile(a, shape_ctx.get_tile(a))
        ctx.set_segment_order(a, shape_ctx.get_segment_order(a))
    u = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float32).contiguous()
    t_end = 1.2 * (args.warmup + args.steps) * ctx.cfl_dt(u, args.cfl)
    times, prims = I.solar_wind_series(t_end, n_knots=9, seed=11)
    ctx.set_inflow_series(times, prims)
    ctx.advance(u, args.warmup, args.cfl)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctx.advance(u, args.steps, args.cfl)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    zones = int(np.prod(setup.U.shape[1:]))
    return {"value": zones * args.steps / (ms / 1000.0), "unit": "zone-updates/s", "steps": args.steps,
            "ms_per_step": ms / args.steps, "knots": len(times), "series_span": [0.0, float(t_end)],
            "simulated_time": ctx.time(u), "status": ctx.status_check(),
            "finite": bool(torch.isfinite(u).all().item())}


def ionosphere_leg(args, setup, make_ctx, shape_ctx, u_dev):
    """The ionosphere shell coupling on the headline run's developed flow
    (the plain run's final FP32 state, copied): one coupling timed alone
    (shell current, potential, drift of the reset zones: three kernels and
    a synchronisation), then args.steps steps with a coupling before each,
    the plain run's tile shape."""
    import numpy as np
    import torch
    from paper_1607_02214_amd import ppmlr

    ctx = make_ctx()
    for a in range(3):
        ctx.set_tile(a, 1)
        ctx.set_segments(a, shape_ctx.get_segments(a))
        ctx.set_tile(a, shape_ctx.get_tile(a))
        ctx.set_segment_order(a, shape_ctx.get_segment_order(a))
    u = u_dev.clone()
    prm = ppmlr.iono_default_params()
    shape = (2, prm.n_theta, prm.n_phi)
    jr = torch.zeros(shape, dtype=torch.float64, device="cuda")
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda")
    ctx.ionosphere_couple(u, prm, jr=jr, phi=phi)          # buffers, first use
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.ionosphere_couple(u, prm, jr=jr, phi=phi)
    ms_couple = (time.perf_counter() - t0) * 1000.0 / reps   # host-timed: each call synchronises
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        ctx.ionosphere_couple(u, prm)
        ctx.advance(u, 1, args.cfl)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    zones = int(np.prod(setup.U.shape[1:]))
    # 1 kV in code units: v_0 B_0 R_E = 21.81 km/s * 1 nT * 6371 km
    kv = 21.81e3 * 1e-9 * 6.371e6 / 1e3
    return {"value": zones * args.steps / (ms / 1000.0), "unit": "zone-updates/s", "steps": args.steps,
            "ms_per_step": ms / args.steps, "ms_per_coupling": round(ms_couple, 4),
            "shell_cells": [2, prm.n_theta, prm.n_phi],
            "r_shell": prm.r_shell, "r_fac": prm.r_fac, "sigma_code": prm.sigma,
            "max_abs_jr": float(jr.abs().max().item()),
            "cross_polar_cap_potential_kV": [float((phi[h].max() - phi[h].min()).item()) * kv for h in range(2)],
            "status": ctx.status_check(), "finite": bool(torch.isfinite(u).all().item())}


def characteristic_leg(args, setup, make_ctx, value_plain, fp64=True):
    """The FP32 run in the characteristic mode (the seven waves traced one by
    one and the linearised seven-wave interface problem) from the same start
    state: its own tile search after the warm-up steps (3 repetitions per
    candidate), then args.steps timed steps with per-sweep launch times; and
    its error against the FP64 characteristic run of the same steps."""
    import numpy as np
    import torch
    from paper_1607_02214_amd import ppmlr

    ctx = make_ctx(tracing=ppmlr.TRACE_CHARACTERISTIC)
    u = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float32).contiguous()
    ctx.advance(u, args.warmup, args.cfl)
    torch.cuda.synchronize()
    ctx.autotune(u, reps=3)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctx.advance(u, args.steps, args.cfl)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    kms, kn = ctx.kernel_times()
    zones = int(np.prod(setup.U.shape[1:]))
    value = zones * args.steps / (ms / 1000.0)
    avg = [kms[a] / kn[a] if kn[a] else 0.0 for a in range(3)]
    dom = int(np.argmax(avg))
    out = {"value": value, "unit": "zone-updates/s", "steps": args.steps, "ms_per_step": ms / args.steps,
           "speedup_vs_fp32_plain": value / value_plain,
           "roofline_frac": round(64.0 * zones / (avg[dom] / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
           "dominant_kernel": f"sweep axis {'xyz'[dom]} (f32, characteristic)",
           "tiles": [ctx.get_tile(a) for a in range(3)], "segments": [ctx.get_segments(a) for a in range(3)],
           "segment_order": [ctx.get_segment_order(a) for a in range(3)],
           "avg_launch_ms": [round(a, 4) for a in avg],
           "status": ctx.status_check(), "finite": bool(torch.isfinite(u).all().item()),
           "simulated_time": ctx.time(u)}
    if fp64:
        ctx64 = make_ctx(tracing=ppmlr.TRACE_CHARACTERISTIC)
        u64 = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float64).contiguous()
        ctx64.advance(u64, args.warmup + args.steps, args.cfl)
        torch.cuda.synchronize()
        out["fp32_vs_fp64"] = fp32_vs_fp64(ctx, u, ctx64, u64)
        out["fp32_vs_fp64"]["after_steps"] = args.warmup + args.steps
        del u64
    return out


def learned_leg(args, setup, make_ctx, u_plain, st_plain, value_plain, ref64=None):
    """The learned Riemann guess on the same workload: harvest interface
    records from a plain FP32 run of the start state, train the network on
    them with the GPU kernels, then time the learned-guess run over the same
    warm-up + timed steps as the plain run and compare the final states (with
    the FP32 plain run, and with the FP64 reference run ref64 = (ctx, state)
    of the same step count when given).  Cost breakdown, all three on the
    learned run's tile shapes over the same steps: plain guess; the learned
    mode with a network whose outputs are not finite, so that every selected
    face runs the network and then falls back to the plain guess (the
    network pass at the plain iteration count); the trained network."""
    import numpy as np
    import torch
    from paper_1607_02214_amd import learned, ppmlr

    t0 = time.perf_counter()
    ctx_h = make_ctx()
    u = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float32).contiguous()
    rec, offered = learned.harvest(ctx_h, u, args.harvest_steps, args.cfl, capacity=args.harvest_cap)
    del u
    t_h = time.perf_counter() - t0
    print(f"[bench] learned: {offered} interface records from {args.harvest_steps} steps ({t_h:.1f} s)",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    theta, hist = learned.train(rec, args.train_steps, batch=4096, lr=1e-3, seed=0,
                                log_every=max(1, args.train_steps // 4))
    torch.cuda.synchronize()
    t_t = time.perf_counter() - t0
    print(f"[bench] learned: trained {args.train_steps} Adam steps ({t_t:.1f} s), loss {hist[0][1]:.3e} -> "
          f"{hist[-1][1]:.3e}", file=sys.stderr, flush=True)
    del rec
    ctx = make_ctx()
    ctx.set_guess(ppmlr.GUESS_LEARNED, theta)
    u = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float32).contiguous()
    ctx.advance(u, args.warmup, args.cfl)      # warm-up, then the tile search on that flow
    torch.cuda.synchronize()
    tiles = ctx.autotune(u, reps=5)
    ctx.reset_stats()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctx.advance(u, args.steps, args.cfl)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    st = ctx.stats()
    zones = u[0].numel()
    value = zones * args.steps / (ms / 1000.0)

    def iters(s):
        h = np.array(s["iters_hist"], dtype=np.int64)
        return int((h * np.arange(32)).sum())

    def prim(U):
        U = U.double()
        rho = U[0]
        v2 = (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / (rho * rho)
        b2 = U[4] ** 2 + U[5] ** 2 + U[6] ** 2
        p = (5.0 / 3.0 - 1.0) * (U[7] - 0.5 * rho * v2 - 0.5 * b2)
        return {"rho": rho, "p": p, "|B'|": torch.sqrt(b2)}

    a, b = prim(u), prim(u_plain)
    err = {k: float((a[k] - b[k]).abs().max() / b[k].abs().max()) for k in a}

    def same_tiles(c):
        # segments first: the tile width is checked against the segment length
        for ax in range(3):
            c.set_segments(ax, ctx.get_segments(ax))
            c.set_segment_order(ax, ctx.get_segment_order(ax))
            c.set_tile(ax, ctx.get_tile(ax, ppmlr.F32))

    def timed(c):
        w = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float32).contiguous()
        c.advance(w, args.warmup, args.cfl)
        torch.cuda.synchronize()
        c.reset_stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.advance(w, args.steps, args.cfl)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, iters(c.stats())

    c_plain = make_ctx()
    same_tiles(c_plain)
    ms_plain, it_plain = timed(c_plain)
    th_nan = theta.clone()
    th_nan[-2:] = float("nan")                 # output biases: every network output non-finite
    c_fb = make_ctx()
    c_fb.set_guess(ppmlr.GUESS_LEARNED, th_nan)
    same_tiles(c_fb)
    ms_fb, it_fb = timed(c_fb)
    fb_stats = c_fb.stats()
    c_tr = make_ctx()
    c_tr.set_guess(ppmlr.GUESS_LEARNED, theta)
    same_tiles(c_tr)
    ms_tr, it_tr = timed(c_tr)
    breakdown = {
        "tiles": tiles,
        "ms_per_step": {"plain": round(ms_plain, 4), "network_all_fallback": round(ms_fb, 4),
                        "trained": round(ms_tr, 4)},
        "newton_iterations": {"plain": it_plain, "network_all_fallback": it_fb, "trained": it_tr},
        "network_pass_ms_per_step": round(ms_fb - ms_plain, 4),
        "iterations_saved_ms_per_step": round(ms_fb - ms_tr, 4),
        "all_fallback_faces": {"selected": fb_stats["guess_faces"], "fallbacks": fb_stats["guess_fallbacks"]},
    }
    del c_plain, c_fb, c_tr
    out = {
        "value": value,
        "unit": "zone-updates/s",
        "ms_per_step": ms / args.steps,
        "speedup_vs_fp32_plain": value / value_plain,
        "tiles": tiles,
        "newton_iterations": {"plain": iters(st_plain), "learned": iters(st)},
        "selected_faces": st["guess_faces"],
        "fallbacks": st["guess_fallbacks"],
        "nonconverged": st["nonconverged"],
        "max_rel_error_vs_fp32_plain": err,
        "harvest": {"steps": args.harvest_steps, "records_offered": offered,
                    "records_kept": min(offered, args.harvest_cap), "seconds": round(t_h, 2)},
        "training": {"adam_steps": args.train_steps, "batch": 4096, "lr": 1e-3, "seconds": round(t_t, 2),
                     "loss_first": hist[0][1], "loss_last": hist[-1][1]},
        "cost_breakdown": breakdown,
    }
    if ref64 is not None:
        out["fp32_vs_fp64"] = fp32_vs_fp64(ctx, u, ref64[0], ref64[1])
        out["fp32_vs_fp64"]["after_steps"] = args.warmup + args.steps
    return out


def ensemble_leg(args):
    """The 32-member batched ensemble (uneven cubic grids 96^3..160^3, seeded
    solar-wind inputs), FP32, autotuned workgroup size and segment length, timed over
    args.ensemble_steps steps after 2 warm-up steps."""
    import torch
    from paper_1607_02214_amd import inputs as I
    from paper_1607_02214_amd import ppmlr

    spec = I.ensemble_members(count=32, seed=4)
    setups = []
    for m in spec:
        faces = I.member_faces(m["N"])
        sw = m["sw"]
        setups.append(I.DipoleSetup(faces=faces, U=I.dipole_initial_state(faces, sw), inflow=sw, inner_rho=sw[0],
                                    inner_p=sw[7], p_floor=1e-8 * sw[7]))

    def member_ctx(st):
        c = ppmlr.Context(st.faces, st.bc_lo, st.bc_hi, r_inner=st.r_inner, p_floor=st.p_floor)
        c.set_dipole(st.moment, st.direction)
        c.set_inflow(st.inflow)
        c.set_inner(st.inner_rho, st.inner_p)
        return c

    ctxs = [member_ctx(st) for st in setups]
    us = [torch.from_numpy(st.U).to("cuda", torch.float32).contiguous() for st in setups]
    zones = sum(m["N"] ** 3 for m in spec)
    print(f"[bench] ensemble: {len(spec)} members, {zones} zones", file=sys.stderr, flush=True)
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PER_SWEEP)
    block = ppmlr.ensemble_autotune(ctxs, us, reps=1)
    # the same 10 steps in each launch form, on copies of the states with
    # contexts of their own (the autotuned segments)
    forms = {}
    for name, mode in (("persistent", ppmlr.ENSEMBLE_PERSISTENT), ("per_sweep", ppmlr.ENSEMBLE_PER_SWEEP)):
        ppmlr.set_ensemble_launch(mode)
        cx = [member_ctx(st) for st in setups]
        for c, c0 in zip(cx, ctxs):
            for a in range(3):
                c.set_segments(a, c0.get_segments(a))
        ws = [u.clone() for u in us]
        ppmlr.ensemble_run(cx, ws, 1, args.cfl)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ppmlr.ensemble_run(cx, ws, 10, args.cfl)
        e1.record()
        torch.cuda.synchronize()
        forms[name] = {"ms_per_step": e0.elapsed_time(e1) / 10,
                       "value": zones * 10 / (e0.elapsed_time(e1) / 1000.0)}
        del ws, cx
    # the same members run one after another, each with its own single-run
    # launches (device-resident dt loop, the same segments, the automatic
    # tile): what the batched launches replace
    cx = [member_ctx(st) for st in setups]
    for c, c0 in zip(cx, ctxs):
        for a in range(3):
            c.set_segments(a, c0.get_segments(a))
    ws = [u.clone() for u in us]
    for c, w in zip(cx, ws):
        c.advance(w, 1, args.cfl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for c, w in zip(cx, ws):
        c.advance(w, 10, args.cfl)
    e1.record()
    torch.cuda.synchronize()
    forms["solo_sequential"] = {"ms_per_step": e0.elapsed_time(e1) / 10,
                                "value": zones * 10 / (e0.elapsed_time(e1) / 1000.0)}
    del ws, cx
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PER_SWEEP)
    ppmlr.ensemble_run(ctxs, us, 2, args.cfl)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    status = ppmlr.ensemble_run(ctxs, us, args.ensemble_steps, args.cfl)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    finite = all(bool(torch.isfinite(u).all().item()) for u in us)
    times = [c.time(u) for c, u in zip(ctxs, us)]
    return {
        "value": zones * args.ensemble_steps / (ms / 1000.0),
        "unit": "zone-updates/s",
        "members": len(spec),
        "sizes": [m["N"] for m in spec],
        "zones": zones,
        "steps": args.ensemble_steps,
        "ms_per_step": ms / args.ensemble_steps,
        "launch": "per sweep (one launch per sweep over every member, a dt kernel per step)",
        "block": block,
        "launch_forms_10_steps": forms,
        "segments_of_largest_member": [ctxs[max(range(len(spec)), key=lambda k: spec[k]["N"])].get_segments(a)
                                       for a in range(3)],
        "status": sorted(set(status)),
        "finite": finite,
        "simulated_time_range": [min(times), max(times)],
    }


def fp32_vs_fp64(ctx32, u32, ctx64, u64, gamma=5.0 / 3.0):
    """Error of an FP32 run against the FP64 run of the same workload and
    step count: per field (rho, p, |B'|) the normwise max |f32 - f64| /
    max |f64| and the pointwise max |f32 - f64| / max(|f64|, 1e-6 max |f64|);
    the drift of the FP64 domain totals (rho, |m|, |B'|, E) between the runs,
    |sum32 - sum64| / |sum64|; and the simulated times of both runs."""
    import numpy as np
    import torch

    def prim(U):
        U = U.double()
        rho = U[0]
        v2 = (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / (rho * rho)
        b2 = U[4] ** 2 + U[5] ** 2 + U[6] ** 2
        return {"rho": rho, "p": (gamma - 1.0) * (U[7] - 0.5 * rho * v2 - 0.5 * b2), "|B'|": torch.sqrt(b2)}

    a, b = prim(u32), prim(u64)
    normwise, pointwise = {}, {}
    for k in a:
        d = (a[k] - b[k]).abs()
        scale = b[k].abs().max()
        normwise[k] = float(d.max() / scale)
        pointwise[k] = float((d / torch.clamp(b[k].abs(), min=1e-6 * float(scale))).max())
        del d
    del a, b
    t32 = np.array(ctx32.totals(u32))
    t64 = np.array(ctx64.totals(u64))
    drift = {"rho": abs(t32[0] - t64[0]) / abs(t64[0]),
             "|m|": float(np.linalg.norm(t32[1:4] - t64[1:4]) / np.linalg.norm(t64[1:4])),
             "|B'|": float(np.linalg.norm(t32[4:7] - t64[4:7]) / np.linalg.norm(t64[4:7])),
             "E": abs(t32[7] - t64[7]) / abs(t64[7])}
    return {"normwise": normwise, "pointwise": pointwise, "totals_drift": drift,
            "simulated_time": {"f32": ctx32.time(u32), "f64": ctx64.time(u64)}}


def c3_leg(args, make_ctx_for):
    """The 512 x 384 x 384 form of the workload (every cell of the bench grid
    split in two, 75.5 M zones): the FP32 run (tile search after 2 warm-up
    steps, then args.c3_steps timed steps, FP64 dt and totals) and its error
    against an FP64 run of the same steps from the same start."""
    import numpy as np
    import torch
    from paper_1607_02214_amd import inputs as I

    t0 = time.perf_counter()
    setup = I.c3_setup(dtype=np.float64)
    n = [len(f) - 1 for f in setup.faces]
    zones = int(np.prod(n))
    print(f"[bench] c3: grid {n[0]}x{n[1]}x{n[2]} built in {time.perf_counter() - t0:.0f} s", file=sys.stderr,
          flush=True)
    warm = 2
    ctx = make_ctx_for(setup)
    u = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float32).contiguous()
    ctx.advance(u, warm, args.cfl)
    torch.cuda.synchronize()
    ctx.autotune(u, reps=3)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ctx.advance(u, args.c3_steps, args.cfl)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ctx64 = make_ctx_for(setup)
    u64 = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float64).contiguous()
    del setup
    ctx64.advance(u64, warm + args.c3_steps, args.cfl)
    torch.cuda.synchronize()
    err = fp32_vs_fp64(ctx, u, ctx64, u64)
    out = {"value": zones * args.c3_steps / (ms / 1000.0), "unit": "zone-updates/s", "grid": n,
           "steps": args.c3_steps, "warmup": warm, "ms_per_step": ms / args.c3_steps,
           "tiles": [ctx.get_tile(a) for a in range(3)], "segments": [ctx.get_segments(a) for a in range(3)],
           "status": ctx.status_check(), "finite": bool(torch.isfinite(u).all().item()),
           "fp32_vs_fp64_after_steps": warm + args.c3_steps, "fp32_vs_fp64": err}
    del u, u64
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cfl", type=float, default=0.4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-series", action="store_true")
    ap.add_argument("--no-iono", action="store_true", help="skip the ionosphere coupling leg")
    ap.add_argument("--no-char", action="store_true", help="skip the characteristic-mode leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 512x384x384 leg")
    ap.add_argument("--c3-steps", type=int, default=20)
    ap.add_argument("--harvest-steps", type=int, default=105,
                    help="plain steps whose interfaces are harvested (~96k records per step: 105 give 1e7)")
    ap.add_argument("--harvest-cap", type=int, default=10_000_000)
    ap.add_argument("--train-steps", type=int, default=6000)
    ap.add_argument("--ensemble-steps", type=int, default=50)
    ap.add_argument("--tiles", type=str, default=None,
                    help="pencils per tile x,y,z for the FP32 run (with --segments: no autotuning)")
    ap.add_argument("--segments", type=str, default=None, help="segments per pencil x,y,z for the FP32 run")
    ap.add_argument("--order", type=str, default=None, help="segment tile order x,y,z (1 adjacent, 2 bands) with --tiles")
    ap.add_argument("--tiles64", type=str, default=None, help="pencils per workgroup x,y,z for the FP64 run")
    ap.add_argument("--segments64", type=str, default=None, help="segments per pencil x,y,z for the FP64 run")
    ap.add_argument("--order64", type=str, default=None, help="segment tile order x,y,z for the FP64 run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the sweep path is single-device "
              "(no halo exchange or collectives are built); use --gpus 1", file=sys.stderr)
        sys.exit(3)

    import numpy as np
    import torch

    from paper_1607_02214_amd import inputs as I
    from paper_1607_02214_amd import ppmlr

    setup = I.c2_setup()
    nx, ny, nz = (len(f) - 1 for f in setup.faces)
    zones = nx * ny * nz
    print(f"[bench] grid {nx}x{ny}x{nz} = {zones} zones, building state", file=sys.stderr, flush=True)

    def make_ctx(**over):
        ctx = ppmlr.Context(setup.faces, setup.bc_lo, setup.bc_hi, r_inner=setup.r_inner, p_floor=setup.p_floor,
                            **over)
        ctx.set_dipole(setup.moment, setup.direction)
        ctx.set_inflow(setup.inflow)
        ctx.set_inner(setup.inner_rho, setup.inner_p)
        return ctx

    def refine_yz(ctx, u, dtype, steps=20, rounds=3):
        """Between 4 and 8 pencils per y or z tile the sweep-by-sweep search
        is within its noise; compare those tile sizes (with the search's
        segments and order) on whole steps of a copy of the state, on a
        context of its own, in `rounds` passes over the candidates (each
        candidate's time is its fastest pass), and keep the fastest."""
        pdt = ppmlr.F64 if dtype == torch.float64 else ppmlr.F32
        base = [ctx.get_tile(a, pdt) for a in range(3)]
        segs = [ctx.get_segments(a, pdt) for a in range(3)]
        order = [ctx.get_segment_order(a) for a in range(3)]
        times = {}
        cands = [(py, pz) for py in sorted({base[1], 4, 8}) for pz in sorted({base[2], 4, 8})]
        for _ in range(rounds):
            for py, pz in cands:
                trial = make_ctx()
                try:
                    for a, P in enumerate((base[0], py, pz)):
                        trial.set_tile(a, 1)
                        trial.set_segments(a, segs[a])
                        trial.set_tile(a, P)
                        trial.set_segment_order(a, order[a])
                except ppmlr.PPMLRError:
                    continue                          # does not fit one workgroup
                w = u.clone()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                try:
                    trial.advance(w, 2, args.cfl)
                    e0.record()
                    trial.advance(w, steps, args.cfl)
                    e1.record()
                    torch.cuda.synchronize()
                except ppmlr.PPMLRError:
                    torch.cuda.synchronize()
                    continue                          # does not fit this dtype's workgroup
                ms = e0.elapsed_time(e1)
                times[(py, pz)] = min(ms, times.get((py, pz), float("inf")))
                del w, trial
        best = min(((ms, py, pz) for (py, pz), ms in times.items()), default=None)
        if best is not None:
            for a, P in ((1, best[1]), (2, best[2])):
                ctx.set_tile(a, P)
            print(f"[bench] whole-step check: y/z tiles {best[1]}/{best[2]} ({best[0] / steps:.3f} ms/step; "
                  f"search gave {base[1]}/{base[2]})", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    def run(dtype, steps, warmup, profile=True, shape=None):
        ctx = make_ctx()
        u = torch.from_numpy(setup.U).to(device="cuda", dtype=dtype).contiguous()
        if shape is None:
            # tile search (outside the timed region) on the state after the
            # warm-up steps, which is closer to the timed steps' flow than the
            # start state; it leaves the state untouched
            ctx.advance(u, warmup, args.cfl)
            torch.cuda.synchronize()
            ctx.autotune(u, reps=5)
            refine_yz(ctx, u, dtype)
            warmup = 0
        else:
            for a in range(3):
                ctx.set_tile(a, 1)
                ctx.set_segments(a, shape[1][a])
                ctx.set_tile(a, shape[0][a])
                if shape[2] is not None:
                    ctx.set_segment_order(a, shape[2][a])
        pdt = ppmlr.F64 if dtype == torch.float64 else ppmlr.F32
        print(f"[bench] tiles {[ctx.get_tile(a, pdt) for a in range(3)]} segments {[ctx.get_segments(a, pdt) for a in range(3)]}"
              f" order {[ctx.get_segment_order(a) for a in range(3)]}"
              f"{'' if shape is None else ' (given)'}", file=sys.stderr, flush=True)
        ctx.advance(u, warmup, args.cfl)
        torch.cuda.synchronize()
        ctx.reset_stats()
        ctx.set_profiling(profile)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        ctx.advance(u, steps, args.cfl)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        kms, kn = ctx.kernel_times()
        status = ctx.status_check()
        st = ctx.stats()
        finite = bool(torch.isfinite(u).all().item())
        return ctx, u, ms, wall, kms, kn, status, st, finite

    if args.copy_calibration:
        # plain device-to-device copy of exactly 1 GiB: its FETCH_SIZE and
        # WRITE_SIZE readings give the counter-to-byte scale
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] fp32: warmup {args.warmup}, timed {args.steps} steps", file=sys.stderr, flush=True)
    shape = None
    if args.tiles or args.segments:
        if not (args.tiles and args.segments):
            raise SystemExit("--tiles and --segments go together")
        shape = ([int(x) for x in args.tiles.split(",")], [int(x) for x in args.segments.split(",")],
                 [int(x) for x in args.order.split(",")] if args.order else None)
    ctx, u, ms, wall, kms, kn, status, st, finite = run(torch.float32, args.steps, args.warmup, shape=shape)
    value = zones * args.steps / (ms / 1000.0)
    avg = [kms[a] / kn[a] if kn[a] else 0.0 for a in range(3)]
    dom = int(np.argmax(avg))
    bytes_per_launch = 64.0 * zones            # 8 FP32 variables read + written
    gbs = bytes_per_launch / (avg[dom] / 1000.0) / 1e9
    traffic, _ = load_traffic("f32")
    flops_zone, flops_src = FLOPS_PER_ZONE_SWEEP, FLOPS_SOURCE
    # VALU issue rate of the dominant sweep: its instruction counts per launch
    # from the committed counters (same kernel source and the same tile shape
    # on that axis; the counts do not depend on the box), over the live launch
    # time
    issue = None
    rec = shape_record(traffic, dom, (ctx.get_tile(dom, ppmlr.F32), ctx.get_segments(dom),
                                      ctx.get_segment_order(dom)))
    if rec and "valu_instructions_per_launch" in rec:
        valu = rec["valu_instructions_per_launch"][str(dom)]
        trans = rec["trans_instructions_per_launch"][str(dom)]
        rate = valu / (avg[dom] / 1000.0) / 1e9
        cyc = (valu + trans) / (avg[dom] / 1000.0) / 1e9
        issue = {"achieved": round(rate, 1), "peak": VALU_ISSUE_PEAK_G, "unit": "G wave64 VALU instructions/s",
                 "frac": round(rate / VALU_ISSUE_PEAK_G, 4),
                 "frac_transcendentals_at_half_rate": round(cyc / VALU_ISSUE_PEAK_G, 4),
                 "valu_per_launch": valu, "source": "committed counter summary, live launch time"}
    tflops = flops_zone * zones / (avg[dom] / 1000.0) / 1e12
    roofline = {
        "bound": "hbm",
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4),
        "traffic": rec["bytes_per_launch"][str(dom)] if rec else None,
        "kernel": f"sweep axis {'xyz'[dom]} (f32)",
        "bytes_per_zone_sweep": 64,
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "avg_launch_ms": [round(a, 4) for a in avg],
        "launches": kn,
        "sum_kernel_ms_per_step": round(sum(kms) / args.steps, 4),
        "limiter": "vector-instruction issue (roofline.issue: at the chip issue rate), not HBM",
        "alu": {"achieved": round(tflops, 2), "peak": FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tflops / FP32_UNPACKED_TFLOPS, 4),
                "frac_of_packed_fp32_peak": round(tflops / FP32_PEAK_TFLOPS, 4),
                "flops_per_zone_sweep": flops_zone, "flops_source": flops_src,
                "kernel_fp32_ops_per_lane": KERNEL_FP32_OPS_PER_LANE},
        "issue": issue,
    }
    out = {
        "metric": "zone-updates/s per 3D split step (FP32/learned vs FP64 plain) at stated error; HBM GB/s",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "inflow-dipole stretched grid 256x192x192, FP32 sweeps + FP64 dt, device-resident dt loop",
            "grid": [nx, ny, nz],
            "cfl": args.cfl,
            "tiles": [ctx.get_tile(a, ppmlr.F32) for a in range(3)],
            "segments": [ctx.get_segments(a) for a in range(3)],
            "segment_order": [ctx.get_segment_order(a) for a in range(3)],
            "tile_search": "autotuned (y/z tile sizes checked on whole steps)" if shape is None else "given",
        },
        "roofline": roofline,
        "health": {"status": status, "finite": finite, "floor_hits": st["floor_hits"],
                   "nonconverged": st["nonconverged"], "simulated_time": ctx.time(u)},
    }
    if not args.no_fp64:
        # FP64 run of the same workload and step count (untimed) for the error
        # of the FP32 headline run
        print(f"[bench] fp64 reference run: {args.warmup + args.steps} steps", file=sys.stderr, flush=True)
        ctx_r = make_ctx()
        u_r = torch.from_numpy(setup.U).to(device="cuda", dtype=torch.float64).contiguous()
        ctx_r.advance(u_r, args.warmup + args.steps, args.cfl)
        torch.cuda.synchronize()
        out["fp32_vs_fp64"] = fp32_vs_fp64(ctx, u, ctx_r, u_r)
        out["fp32_vs_fp64"]["after_steps"] = args.warmup + args.steps
    def leg(name, fn, *a, **k):
        # a secondary leg that fails reports its error in its own field and
        # leaves the headline line standing
        print(f"[bench] {name}", file=sys.stderr, flush=True)
        try:
            out[name] = fn(*a, **k)
        except Exception as e:   # noqa: BLE001
            out[name] = {"error": f"{type(e).__name__}: {e}"}
            print(f"[bench] {name} failed: {e}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    if not args.no_series:
        leg("inflow_series", series_leg, args, setup, make_ctx, ctx)
    if not args.no_iono:
        leg("ionosphere", ionosphere_leg, args, setup, make_ctx, ctx, u)
    if not args.no_char:
        leg("characteristic", characteristic_leg, args, setup, make_ctx, value, fp64=not args.no_fp64)
    if not args.no_learned:
        leg("learned", learned_leg, args, setup, make_ctx, u, st, value,
            ref64=None if args.no_fp64 else (ctx_r, u_r))
    if not args.no_fp64:
        del u_r, ctx_r
    del u
    torch.cuda.empty_cache()

    if not args.no_fp64:
        n64 = max(5, min(20, args.steps))
        print(f"[bench] fp64 plain: {n64} steps", file=sys.stderr, flush=True)
        shape64 = None
        if args.tiles64 or args.segments64:
            if not (args.tiles64 and args.segments64):
                raise SystemExit("--tiles64 and --segments64 go together")
            shape64 = ([int(x) for x in args.tiles64.split(",")], [int(x) for x in args.segments64.split(",")],
                       [int(x) for x in args.order64.split(",")] if args.order64 else None)
        ctx64, u64, ms64, _, kms64, kn64, status64, _, fin64 = run(torch.float64, n64, 2, shape=shape64)
        v64 = zones * n64 / (ms64 / 1000.0)
        avg64 = [kms64[a] / kn64[a] if kn64[a] else 0.0 for a in range(3)]
        d64 = int(np.argmax(avg64))
        ach64 = 128.0 * zones / (avg64[d64] / 1000.0) / 1e9
        traffic64, _ = load_traffic("f64")
        sh64 = [(ctx64.get_tile(a, ppmlr.F64), ctx64.get_segments(a, ppmlr.F64), ctx64.get_segment_order(a))
                for a in range(3)]
        rec64 = shape_record(traffic64, d64, sh64[d64])
        out["fp64_plain"] = {"value": v64, "steps": n64, "ms_per_step": ms64 / n64,
                             "roofline_frac": round(ach64 / HBM_PEAK_GBS, 4),
                             "dominant_kernel": f"sweep axis {'xyz'[d64]} (f64)",
                             "avg_launch_ms": [round(a, 4) for a in avg64],
                             "tiles": [x[0] for x in sh64], "segments": [x[1] for x in sh64],
                             "segment_order": [x[2] for x in sh64],
                             "traffic": rec64["bytes_per_launch"][str(d64)] if rec64 else None,
                             "status": status64, "finite": fin64, "fp32_speedup": value / v64}
        del u64
        torch.cuda.empty_cache()

    if not args.no_ensemble:
        leg("ensemble", ensemble_leg, args)

    if not args.no_c3:
        def make_ctx_for(st):
            c = ppmlr.Context(st.faces, st.bc_lo, st.bc_hi, r_inner=st.r_inner, p_floor=st.p_floor)
            c.set_dipole(st.moment, st.direction)
            c.set_inflow(st.inflow)
            c.set_inner(st.inner_rho, st.inner_p)
            return c
        leg("c3_512x384x384", c3_leg, args, make_ctx_for)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        prob = O.OracleProblem(setup.faces, bc_lo=setup.bc_lo, bc_hi=setup.bc_hi, dip_moment=setup.moment,
                               dip_dir=setup.direction, r_inner=setup.r_inner)
        dt = prob.cfl_dt(setup.U, args.cfl)
        leg("cpu_baseline", cpu_baseline, setup, dt, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
