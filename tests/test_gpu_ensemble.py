"""Batched ensemble through the C ABI: one launch per sweep advances members
of different sizes, each with its own solar-wind inflow and its own dt.  Each
member must equal a solo run of the same member with the same tiles, bitwise
(same arithmetic; only the launch differs), including the simulated time and
the counters."""
import numpy as np
import pytest

from paper_1607_02214_amd import inputs as I

import gpu_cases as GC

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_02214_amd import ppmlr
    ppmlr.lib()


def _member(N, sw):
    faces = I.member_faces(N)
    st = I.DipoleSetup(faces=faces, U=I.dipole_initial_state(faces, sw), inflow=sw, inner_rho=sw[0],
                       inner_p=sw[7], p_floor=1e-8 * sw[7])
    return st


def _ctx(st, **over):
    from paper_1607_02214_amd import ppmlr
    c = ppmlr.Context(st.faces, st.bc_lo, st.bc_hi, r_inner=st.r_inner, p_floor=st.p_floor, **over)
    c.set_dipole(st.moment, st.direction)
    c.set_inflow(st.inflow)
    c.set_inner(st.inner_rho, st.inner_p)
    return c


def _members(k=4, seed=4):
    spec = I.ensemble_members(count=k, seed=seed)
    sizes = [24, 32, 40, 28, 36][:k]        # small uneven grids (same generator rule)
    return [_member(N, m["sw"]) for N, m in zip(sizes, spec)]


@pytest.fixture(params=["persistent", "per-sweep"])
def launch(request):
    from paper_1607_02214_amd import ppmlr
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PERSISTENT if request.param == "persistent"
                              else ppmlr.ENSEMBLE_PER_SWEEP)
    yield request.param
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PER_SWEEP)     # the library's default


@pytest.mark.parametrize("dtype,block", [(torch.float32, 256), (torch.float32, 512), (torch.float64, 256)])
def test_ensemble_members_equal_solo_runs_bitwise(dtype, block, launch):
    from paper_1607_02214_amd import ppmlr
    mem = _members()
    GC.log(f"[ensemble] {launch} {len(mem)} members {[len(m.faces[0]) - 1 for m in mem]} {dtype} block {block}")
    ctxs = [_ctx(m) for m in mem]
    us = [torch.from_numpy(m.U).to("cuda", dtype).contiguous() for m in mem]
    steps = 3
    status = ppmlr.ensemble_run(ctxs, us, steps, 0.4, block=block)
    assert status == [0] * len(mem)
    for m, (st, c, u) in enumerate(zip(mem, ctxs, us)):
        solo = _ctx(st)
        for ax in range(3):
            M = len(st.faces[ax]) - 1 + 14
            nq = (len(st.faces[1]) - 1) if ax == 0 else (len(st.faces[0]) - 1)
            solo.set_tile(ax, max(1, min(block // M, nq)))
        w = torch.from_numpy(st.U).to("cuda", dtype).contiguous()
        solo.advance(w, steps, 0.4)
        torch.cuda.synchronize()
        if not torch.equal(u, w):
            d = (u - w).abs().flatten(1).max(dim=1).values.tolist()
            raise AssertionError(f"member {m} differs: max |diff| per variable {d}; "
                                 f"time {c.time(u)!r} vs {solo.time(w)!r}")
        assert c.time(u) == solo.time(w)
        assert c.get_step_index() == steps
        assert c.stats() == solo.stats()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_ensemble_with_segmented_members_equals_solo_runs_bitwise(dtype, launch):
    # members 0 and 2 cut their pencils into segments (on all axes, or on z
    # only), members 1 and 3 keep whole pencils; 3 steps = 9 sweeps, so the
    # alternating members end in their second state and are copied back
    from paper_1607_02214_amd import ppmlr
    mem = _members()
    segs = [(3, 3, 3), (1, 1, 1), (1, 1, 2), (1, 1, 1)]
    block = 256
    ctxs = [_ctx(m) for m in mem]
    for c, sg in zip(ctxs, segs):
        for ax, k in enumerate(sg):
            c.set_segments(ax, k)
    us = [torch.from_numpy(m.U).to("cuda", dtype).contiguous() for m in mem]
    status = ppmlr.ensemble_run(ctxs, us, 3, 0.4, block=block)
    assert status == [0] * len(mem)
    for m, (st, c, u) in enumerate(zip(mem, ctxs, us)):
        solo = _ctx(st)                  # whole pencils, any tile: the same result
        w = torch.from_numpy(st.U).to("cuda", dtype).contiguous()
        solo.advance(w, 3, 0.4)
        torch.cuda.synchronize()
        if not torch.equal(u, w):
            d = (u - w).abs().flatten(1).max(dim=1).values.tolist()
            raise AssertionError(f"member {m} (segments {segs[m]}) differs: max |diff| per variable {d}")
        assert c.time(u) == solo.time(w)
        assert c.stats() == solo.stats()


def test_ensemble_autotune_leaves_states_untouched_and_c4_members_run():
    from paper_1607_02214_amd import ppmlr
    spec = I.ensemble_members(count=32, seed=4)
    # the 32 seeded members of the batched configuration at half linear size
    # (same generator rule), to keep the test short
    mem = [_member(max(32, (m["N"] // 2) // 8 * 8), m["sw"]) for m in spec]
    ctxs = [_ctx(m) for m in mem]
    us = [torch.from_numpy(m.U).to("cuda", torch.float32).contiguous() for m in mem]
    before = [u.clone() for u in us]
    block = ppmlr.ensemble_autotune(ctxs, us, reps=1)
    assert block in (256, 512, 1024)
    GC.log(f"[ensemble] autotuned segments of member 0: {[ctxs[0].get_segments(a) for a in range(3)]}")
    for u, b in zip(us, before):
        assert torch.equal(u, b)
    assert all(c.get_step_index() == 0 for c in ctxs)
    status = ppmlr.ensemble_run(ctxs, us, 4, 0.4)
    GC.log(f"[ensemble] 32 members autotuned block {block}, status {set(status)}")
    assert all(s in (0,) for s in status)
    for u in us:
        assert bool(torch.isfinite(u).all())
    times = [c.time(u) for c, u in zip(ctxs, us)]
    assert len(set(times)) > 1          # every member has its own dt


def test_ensemble_rejects_bad_arguments():
    from paper_1607_02214_amd import ppmlr
    mem = _members(2)
    ctxs = [_ctx(m) for m in mem]
    us = [torch.from_numpy(m.U).to("cuda", torch.float32).contiguous() for m in mem]
    with pytest.raises(ppmlr.PPMLRError):
        ppmlr.ensemble_run(ctxs, us, 1, 0.4, block=128)
    with pytest.raises(ppmlr.PPMLRError):
        ppmlr.ensemble_run(ctxs, [us[0], us[1].double()], 1, 0.4, block=256)


def test_persistent_barrier_gives_up_and_reports():
    # a barrier poll limit of 0 makes every grid-barrier wait of the
    # persistent launch give up at its first poll: the kernel leaves, and the
    # call reports PPMLR_EDEVICE instead of hanging; a later call with the
    # default limit runs normally and equals a solo run
    from paper_1607_02214_amd import ppmlr
    mem = _members(3)
    ctxs = [_ctx(m) for m in mem]
    us = [torch.from_numpy(m.U).to("cuda", torch.float32).contiguous() for m in mem]
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PERSISTENT)
    try:
        ppmlr.set_ensemble_barrier_limit(0)
        try:
            with pytest.raises(ppmlr.PPMLRError) as ei:
                ppmlr.ensemble_run(ctxs, us, 2, 0.4, block=256)
            assert ei.value.status == ppmlr.PPMLR_EDEVICE and "barrier" in str(ei.value)
        finally:
            ppmlr.set_ensemble_barrier_limit(1 << 22)
        ctxs = [_ctx(m) for m in mem]
        us = [torch.from_numpy(m.U).to("cuda", torch.float32).contiguous() for m in mem]
        assert ppmlr.ensemble_run(ctxs, us, 2, 0.4, block=256) == [0, 0, 0]
    finally:
        ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PER_SWEEP)
    solo = _ctx(mem[1])
    for ax in range(3):
        M = len(mem[1].faces[ax]) - 1 + 14
        nq = (len(mem[1].faces[1]) - 1) if ax == 0 else (len(mem[1].faces[0]) - 1)
        solo.set_tile(ax, max(1, min(256 // M, nq)))
    w = torch.from_numpy(mem[1].U).to("cuda", torch.float32).contiguous()
    solo.advance(w, 2, 0.4)
    torch.cuda.synchronize()
    assert torch.equal(us[1], w)


def test_one_failing_member_leaves_the_others_running():
    # member 0 starts with a negative density: its status reports it, and the
    # other members advance exactly as solo runs
    from paper_1607_02214_amd import ppmlr
    mem = _members(3)
    U0 = mem[0].U.copy()
    U0[0, 5, 6, 7] = -1.0
    ctxs = [_ctx(m) for m in mem]
    states = [U0] + [m.U for m in mem[1:]]
    us = [torch.from_numpy(U).to("cuda", torch.float32).contiguous() for U in states]
    status = ppmlr.ensemble_run(ctxs, us, 2, 0.4, block=256)
    assert status[0] == ppmlr.PPMLR_ENONPHYS
    assert status[1:] == [0, 0]
    for m in (1, 2):
        solo = _ctx(mem[m])
        w = torch.from_numpy(mem[m].U).to("cuda", torch.float32).contiguous()
        solo.advance(w, 2, 0.4)
        torch.cuda.synchronize()
        assert torch.equal(us[m], w), m
