"""Empty and zero-size inputs through the C ABI: zero steps leave every state,
the simulated time and the step index untouched (single run and ensemble,
both launch forms, the allocation-free call); an empty member list and a grid
with an empty axis are refused with EINVAL, before any device work."""
import ctypes as C

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
    yield
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PER_SWEEP)


def _dev(U, dtype):
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype).contiguous()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_zero_steps_leave_state_time_and_step_index(dtype):
    case = GC.smooth_case(shape=(9, 10, 11))
    GC.log(f"[empty] advance 0 steps {dtype}")
    ctx = case.context()
    u = _dev(case.U, dtype)
    before = u.clone()
    t0, k0 = ctx.time(u), ctx.get_step_index()
    ctx.advance(u, 0, 0.4)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
    assert ctx.time(u) == t0 and ctx.get_step_index() == k0


@pytest.mark.parametrize("launch", ["per_sweep", "persistent", "noalloc"])
def test_ensemble_of_zero_steps(launch):
    from paper_1607_02214_amd import ppmlr
    GC.log(f"[empty] ensemble 0 steps {launch}")
    ppmlr.set_ensemble_launch(ppmlr.ENSEMBLE_PERSISTENT if launch == "persistent" else ppmlr.ENSEMBLE_PER_SWEEP)
    cases = [GC.smooth_case(shape=(9, 10, 11), seed=1), GC.smooth_case(shape=(12, 9, 10), seed=2)]
    ctxs = [c.context() for c in cases]
    us = [_dev(c.U, torch.float32) for c in cases]
    before = [u.clone() for u in us]
    status = ppmlr.ensemble_run(ctxs, us, 0, 0.4, noalloc=launch == "noalloc")
    torch.cuda.synchronize()
    assert status == [ppmlr.PPMLR_OK] * 2
    for u, b, c in zip(us, before, ctxs):
        assert torch.equal(u, b)
        assert c.time(u) == 0.0 and c.get_step_index() == 0


def test_empty_member_list_and_empty_axis_are_refused():
    from paper_1607_02214_amd import ppmlr
    GC.log("[empty] refusals")
    lib = ppmlr.lib()
    per = (C.c_int * 1)()
    assert lib.ppmlr_ensemble_run(None, None, 0, 1, 0.4, 0, per) == ppmlr.PPMLR_EINVAL
    assert lib.ppmlr_ensemble_run_noalloc(None, None, 0, 1, 0.4, 0, per) == ppmlr.PPMLR_EINVAL
    blk = C.c_int()
    assert lib.ppmlr_ensemble_autotune(None, None, 0, 1, 0.4, C.byref(blk)) == ppmlr.PPMLR_EINVAL
    with pytest.raises(ValueError):
        ppmlr.ensemble_run([], [], 1, 0.4)
    f = I.uniform_faces(8)
    for empty in (np.array([0.0]), np.array([], dtype=np.float64)):
        with pytest.raises(ppmlr.PPMLRError) as e:
            ppmlr.Context([f, empty, f])
        assert e.value.status == ppmlr.PPMLR_EINVAL
