"""ppmlr_ensemble_run_noalloc through the C ABI: the ensemble call whose work
tables live in the library's fixed device array instead of being allocated
per call.  Its results must equal ppmlr_ensemble_run's bitwise (same
kernels, same arithmetic), on two calls in a row where the second takes a
smaller ensemble (fewer, smaller members) than the first, so that stale
tables from the first call would show.  Also: more than 64 members and a
segmented member without a second state are refused before any work."""
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
    return I.DipoleSetup(faces=faces, U=I.dipole_initial_state(faces, sw), inflow=sw, inner_rho=sw[0],
                         inner_p=sw[7], p_floor=1e-8 * sw[7])


def _ctx(st, segments):
    from paper_1607_02214_amd import ppmlr
    c = ppmlr.Context(st.faces, st.bc_lo, st.bc_hi, r_inner=st.r_inner, p_floor=st.p_floor)
    c.set_dipole(st.moment, st.direction)
    c.set_inflow(st.inflow)
    c.set_inner(st.inner_rho, st.inner_p)
    for ax in range(3):
        c.set_segments(ax, segments)
    return c


def _prime_second_state(ctx, st, dtype):
    # one segmented sweep of a throw-away copy gives the context its second
    # state; the counters it added are cleared (the simulated time and step
    # index do not move in a lone sweep without an inflow series)
    w = torch.from_numpy(st.U).to("cuda", dtype).contiguous()
    ctx.sweep(w, 1e-6, 0)
    torch.cuda.synchronize()
    ctx.reset_stats()
    del w


def _run_pair(sizes, segs, dtype, steps, seed):
    """The same ensemble through ppmlr_ensemble_run and through
    ppmlr_ensemble_run_noalloc on fresh contexts; every member must agree
    bitwise (state, simulated time, step index, counters)."""
    from paper_1607_02214_amd import ppmlr
    spec = I.ensemble_members(count=len(sizes), seed=seed)
    mem = [_member(N, m["sw"]) for N, m in zip(sizes, spec)]
    GC.log(f"[noalloc] members {sizes} segments {segs} {dtype} steps {steps}")
    ref_ctx = [_ctx(m, s) for m, s in zip(mem, segs)]
    ref_u = [torch.from_numpy(m.U).to("cuda", dtype).contiguous() for m in mem]
    assert ppmlr.ensemble_run(ref_ctx, ref_u, steps, 0.4, block=512) == [0] * len(mem)
    na_ctx = [_ctx(m, s) for m, s in zip(mem, segs)]
    for c, m, s in zip(na_ctx, mem, segs):
        if s > 1:
            _prime_second_state(c, m, dtype)
    na_u = [torch.from_numpy(m.U).to("cuda", dtype).contiguous() for m in mem]
    assert ppmlr.ensemble_run(na_ctx, na_u, steps, 0.4, block=512, noalloc=True) == [0] * len(mem)
    torch.cuda.synchronize()
    for k in range(len(mem)):
        if not torch.equal(ref_u[k], na_u[k]):
            d = (ref_u[k] - na_u[k]).abs().flatten(1).max(dim=1).values.tolist()
            raise AssertionError(f"member {k} (N={sizes[k]}) differs: {d}")
        assert ref_ctx[k].time(ref_u[k]) == na_ctx[k].time(na_u[k])
        assert ref_ctx[k].get_step_index() == na_ctx[k].get_step_index() == steps
        assert ref_ctx[k].stats() == na_ctx[k].stats()
        assert bool(torch.isfinite(na_u[k]).all())


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_equals_ensemble_run_on_two_calls_second_smaller(dtype, persistent):
    # first call: four members, two of them cut into pencil segments; second
    # call (same process, same fixed tables): two smaller members; in both
    # launch forms of the ensemble calls
    from paper_1607_02214_amd import ppmlr
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PERSISTENT if persistent else ppmlr.ENSEMBLE_PER_SWEEP)
    try:
        _run_pair([32, 24, 40, 28], [2, 1, 3, 1], dtype, 3, seed=4)
        _run_pair([20, 16], [1, 2], dtype, 2, seed=9)
    finally:
        ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PER_SWEEP)


def test_noalloc_refuses_too_many_members_and_missing_second_state():
    from paper_1607_02214_amd import ppmlr
    spec = I.ensemble_members(count=1, seed=4)
    st = _member(16, spec[0]["sw"])
    c = _ctx(st, 1)
    u = torch.from_numpy(st.U).to("cuda", torch.float32).contiguous()
    before = u.clone()
    with pytest.raises(ppmlr.PPMLRError) as ei:
        ppmlr.ensemble_run([c] * 65, [u] * 65, 1, 0.4, block=512, noalloc=True)
    assert ei.value.status == ppmlr.PPMLR_EINVAL and "64" in str(ei.value)
    # a segmented member whose context has no second state yet
    cs = _ctx(st, 2)
    with pytest.raises(ppmlr.PPMLRError) as ei:
        ppmlr.ensemble_run([cs], [u], 1, 0.4, block=512, noalloc=True)
    assert ei.value.status == ppmlr.PPMLR_EINVAL and "second state" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
    assert c.get_step_index() == 0 and cs.get_step_index() == 0
