"""Pencil segments: a sweep whose tiles hold pencil segments (interior zones
plus the 7 ghost zones on either side that the sweep's stencils reach) gives
the whole-pencil result bit for bit, with the same counters, on every axis,
in FP32 and FP64, for segment counts that leave a short last segment, with
periodic, outflow and inflow boundaries, with the fused signal-speed
maximum, and in the learned and harvest initial-guess modes."""
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


def _segments_for(n):
    """Segment counts for a pencil of n zones: even and ragged splits, down to
    segments of about 7 zones."""
    out = []
    for k in (2, 3, 4, 5):
        L = -(-n // k)
        if L >= 7 and (k - 1) * L < n:
            out.append(k)
    return out


def _sweep(case, dtype, axis, segments, dt, order=0):
    ctx = case.context()
    ctx.set_segments(axis, segments)
    ctx.set_segment_order(axis, order)
    u = torch.from_numpy(case.U).to("cuda", dtype).contiguous()
    ctx.reset_stats()
    ctx.sweep(u, dt, axis)
    torch.cuda.synchronize()
    return u, ctx.stats()


@pytest.mark.parametrize("maker", [GC.blast_case, GC.dipole_case, GC.c1_case])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_segmented_sweep_is_bitwise_whole_pencil(maker, dtype):
    case = maker()
    n = [len(f) - 1 for f in case.faces]
    ctx = case.context()
    u0 = torch.from_numpy(case.U).to("cuda", dtype).contiguous()
    dt = ctx.cfl_dt(u0, 0.4)
    for axis in range(3):
        ref, st_ref = _sweep(case, dtype, axis, 1, dt)
        for k in _segments_for(n[axis]):
            for order in (1, 2):             # segments adjacent / segment bands
                GC.log(f"[segments] {case.name} {dtype} axis {axis} N={n[axis]} segments {k} order {order}")
                got, st = _sweep(case, dtype, axis, k, dt, order)
                assert torch.equal(got, ref), (axis, k, order)
                assert st == st_ref, (axis, k, order)


def test_segmented_advance_matches_whole_pencils():
    # fused signal-speed maximum (next dt) and Strang ordering over steps
    case = GC.dipole_case()
    res = []
    for segs in ((1, 1, 1), (3, 2, 2)):
        ctx = case.context()
        for axis, k in enumerate(segs):
            ctx.set_segments(axis, k)
        u = torch.from_numpy(case.U).to("cuda", torch.float32).contiguous()
        ctx.advance(u, 4, 0.4)
        torch.cuda.synchronize()
        res.append((u, ctx.time(u), ctx.stats()))
    assert torch.equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]
    assert res[0][2] == res[1][2]


def test_segmented_learned_and_harvest_modes():
    from paper_1607_02214_amd import ppmlr
    case = GC.blast_case()
    thd = torch.from_numpy(I.mlp_init(2, scale=0.5)).cuda()
    u0 = torch.from_numpy(case.U).to("cuda", torch.float32).contiguous()
    outs = []
    for k in (1, 3):
        ctx = case.context()
        for axis in range(3):
            ctx.set_segments(axis, k)
        ctx.set_guess(ppmlr.GUESS_LEARNED, thd)
        u = u0.clone()
        ctx.advance(u, 2, 0.4)
        torch.cuda.synchronize()
        outs.append((u, ctx.stats()))
    assert torch.equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    assert outs[0][1]["guess_faces"] > 0
    # harvest: every owned face once, so the same record set
    from paper_1607_02214_amd import learned
    recs = []
    for k in (1, 3):
        ctx = case.context()
        for axis in range(3):
            ctx.set_segments(axis, k)
        rec, offered = learned.harvest(ctx, u0.clone(), 2, 0.4, capacity=400000)
        R = rec.cpu().numpy()
        recs.append((offered, R[np.lexsort(R.T[::-1])]))
    assert recs[0][0] == recs[1][0] > 500
    assert np.array_equal(recs[0][1], recs[1][1])


def test_segment_arguments():
    from paper_1607_02214_amd import ppmlr
    case = GC.blast_case()                 # n = 40, 33, 30
    ctx = case.context()
    assert ctx.get_segments(0) == 1
    assert [ctx.get_segment_order(a) for a in range(3)] == [1, 2, 2]
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_segment_order(0, 3)
    ctx.set_segments(0, 5)                 # segments of 8
    assert ctx.get_segments(0) == 5
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_segments(0, 7)             # segments of 6 < 7 ghost zones
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_segments(2, 100)           # empty segments
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_segments(1, -1)
    ctx.set_segments(0, 4)                 # 10 + 14 zones per segment
    ctx.set_tile(0, 40)                    # 960 lanes
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_segments(0, 1)             # 40 whole pencils exceed a workgroup
    with pytest.raises(ppmlr.PPMLRError):
        ctx.set_segments(0, 0)             # automatic = one segment: same
    ctx.set_tile(0, 0)
    ctx.set_segments(0, 0)
    assert ctx.get_segments(0) == 1


def test_full_size_z_sweep_segments_bitwise():
    # the 256 x 192 x 192 inflow-dipole workload, FP32: z sweeps with the
    # segment counts the autotuner searches give the whole-pencil result
    from paper_1607_02214_amd import ppmlr
    setup = I.c2_setup(dtype=np.float32)
    ctx = ppmlr.Context(setup.faces, setup.bc_lo, setup.bc_hi, r_inner=setup.r_inner, p_floor=setup.p_floor)
    ctx.set_dipole(setup.moment, setup.direction)
    ctx.set_inflow(setup.inflow)
    ctx.set_inner(setup.inner_rho, setup.inner_p)
    u0 = torch.from_numpy(setup.U).to("cuda", torch.float32).contiguous()
    dt = ctx.cfl_dt(u0, 0.4)
    ref = None
    for k, P in ((1, 4), (2, 8), (4, 16), (8, 16)):
        ctx.set_tile(2, 1)
        ctx.set_segments(2, k)
        ctx.set_tile(2, P)
        GC.log(f"[segments] full-size z sweep, {k} segments, {P} pencils per tile")
        u = u0.clone()
        ctx.sweep(u, dt, 2)
        torch.cuda.synchronize()
        if ref is None:
            ref = u
        else:
            assert torch.equal(u, ref), k


@pytest.mark.parametrize("shape,axis", [((1100, 8, 7), 0), ((7, 8, 900), 2)])
def test_long_pencils_use_segments_and_match_oracle(shape, axis):
    # pencils longer than one workgroup holds (1010 zones FP32, 818 FP64)
    # are swept in segments automatically; one FP64 step against the oracle
    from oracle import oracle as O
    from paper_1607_02214_amd import ppmlr
    case = GC.blast_case(n=shape, seed=7)
    ctx = case.context()
    n = shape[axis]
    assert ctx.get_segments(axis, ppmlr.F64) == 2
    assert ctx.get_segments(axis, ppmlr.F32) == (2 if n > 1010 else 1)
    ora = case.oracle()
    dt = ora.cfl_dt(case.U, 0.4)
    st = O.Stats()
    ref = ora.step(case.U, dt, 0, st)
    GC.log(f"[segments] long pencils {shape} axis {axis}: FP64 step vs oracle")
    u = torch.from_numpy(case.U).cuda().contiguous()
    ctx.step(u, dt)
    torch.cuda.synchronize()
    err = GC.normwise_errors(u.cpu().numpy(), ref)
    assert np.all(err <= 1e-11), err
    assert ctx.stats()["nonconverged"] == st.nonconverged == 0
    # FP32: automatic segments equal three explicit segments bitwise
    res = []
    for k in (0, 3):
        c = case.context()
        c.set_segments(axis, k)
        w = torch.from_numpy(case.U).to("cuda", torch.float32).contiguous()
        c.step(w, dt)
        torch.cuda.synchronize()
        res.append(w)
    assert torch.equal(res[0], res[1])


def test_autotune_leaves_state_untouched_and_tuned_shape_is_bitwise_default():
    # the tile search (pencils, segments, order) times sweeps on its own copy;
    # whatever shape it picks, the run equals the default shape bitwise
    case = GC.dipole_case()
    ctx = case.context()
    u = torch.from_numpy(case.U).to("cuda", torch.float32).contiguous()
    before = u.clone()
    tiles = ctx.autotune(u, reps=1)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
    shape = [(ctx.get_tile(a), ctx.get_segments(a), ctx.get_segment_order(a)) for a in range(3)]
    GC.log(f"[segments] autotuned (pencils, segments, order) per axis: {shape}")
    assert [s[0] for s in shape] == list(tiles)
    assert all(o in (1, 2) for _, _, o in shape)
    ctx.reset_stats()
    ctx.advance(u, 3, 0.4)
    ref = case.context()
    w = before.clone()
    ref.advance(w, 3, 0.4)
    torch.cuda.synchronize()
    assert torch.equal(u, w)
    assert ctx.time(u) == ref.time(w)
    assert ctx.stats() == ref.stats()
