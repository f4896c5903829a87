"""BF16 matrix-core MLP kernels (learned Riemann guess) against the FP64 MLP
oracle, through the C ABI.

Both sides get the same parameters and inputs, rounded to BF16 where the GPU
rounds them (weights and inputs); biases stay FP32 on both sides.  The GPU
also rounds the hidden activations and the backpropagated errors to BF16
(FP32 accumulation), so the comparison is normwise with a tolerance of 1e-2
(BF16 has an 8-bit significand: 2^-9 relative rounding per operand, a few
roundings along each path)."""
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


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _params(seed, scale=1.0):
    """Parameters whose weights are BF16 values (biases FP32, non-zero)."""
    from oracle import oracle as O
    th = I.mlp_init(seed, scale=scale).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = O.mlp_unpack(th)
    rng = np.random.default_rng(seed + 100)
    for W in (W1, W2, W3):
        W[...] = bf16_round(W)
    for b in (b1, b2, b3):
        b[...] = rng.normal(0.0, 0.1, b.shape).astype(np.float32)
    return th


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _blocks(g):
    from oracle import oracle as O
    return O.mlp_unpack(np.asarray(g, dtype=np.float64))


@pytest.mark.parametrize("n", [1, 64, 200])
def test_forward_matches_oracle(n):
    from oracle import oracle as O
    from paper_1607_02214_amd import ppmlr
    th = _params(1)
    X = bf16_round(I.mlp_samples(n, seed=2)).astype(np.float64)
    ref = O.mlp_forward(th, X)
    mlp = ppmlr.MLP(256)
    got = mlp.forward(_dev(th), _dev(X)).cpu().numpy().astype(np.float64)
    err = np.max(np.abs(got - ref), axis=0) / np.max(np.abs(ref), axis=0)
    GC.log(f"[mlp] forward n={n} normwise error per output {err}")
    assert np.all(err <= 1e-2), err


def test_forward_strided_rows_and_empty():
    # rows with a leading dimension (a harvest record buffer), and n = 0
    from oracle import oracle as O
    from paper_1607_02214_amd import ppmlr
    th = _params(3)
    X = bf16_round(I.mlp_samples(130, seed=4)).astype(np.float64)
    R = np.zeros((130, 28), dtype=np.float32)
    R[:, :14] = X
    mlp = ppmlr.MLP(64)
    Rd = _dev(R)
    got = mlp.forward(_dev(th), Rd[:, :14]).cpu().numpy()
    ref = O.mlp_forward(th, X)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= 1e-2
    empty = mlp.forward(_dev(th), Rd[:0, :14])
    assert empty.shape == (0, 2)


@pytest.mark.parametrize("n", [64, 300])
def test_gradient_matches_oracle(n):
    from oracle import oracle as O
    from paper_1607_02214_amd import ppmlr
    th = _params(5)
    X = bf16_round(I.mlp_samples(n, seed=6)).astype(np.float64)
    Y = np.random.default_rng(7).normal(0.0, 0.3, (n, 2))
    loss_ref, g_ref = O.mlp_loss_grad(th, X, Y)
    mlp = ppmlr.MLP(512)
    g, loss = mlp.grad(_dev(th), _dev(X), _dev(Y))
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.item())
    GC.log(f"[mlp] grad n={n} loss gpu {loss:.6e} oracle {loss_ref:.6e}")
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    for name, a, b in zip(names, _blocks(g), _blocks(g_ref)):
        e = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)
        GC.log(f"[mlp]   d{name}: normwise error {e:.3e}")
        assert e <= 2e-2, (name, e)


def test_gradient_is_deterministic():
    from paper_1607_02214_amd import ppmlr
    th = _dev(_params(8))
    X = _dev(I.mlp_samples(1000, seed=9))
    Y = _dev(np.random.default_rng(10).normal(0.0, 0.3, (1000, 2)))
    mlp = ppmlr.MLP(1024)
    g1, l1 = mlp.grad(th, X, Y)
    g2, l2 = mlp.grad(th, X, Y)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_adam_step_matches_oracle():
    # the GPU step = the GPU gradient + the Adam update; the update is checked
    # against the oracle's Adam applied to that same gradient
    from oracle import oracle as O
    from paper_1607_02214_amd import ppmlr
    th = _params(11)
    X = _dev(I.mlp_samples(256, seed=12))
    Y = _dev(np.random.default_rng(13).normal(0.0, 0.3, (256, 2)))
    rng = np.random.default_rng(14)
    m = rng.normal(0.0, 1e-3, th.size)
    v = rng.uniform(0.0, 1e-5, th.size)
    mlp = ppmlr.MLP(256)
    thd, md, vd = _dev(th), _dev(m), _dev(v)
    g, _ = mlp.grad(thd, X, Y)
    t = 7
    mlp.train_step(thd, md, vd, X, Y, t, lr=1e-3)
    th_ref = th.astype(np.float32).astype(np.float64).copy()
    m_ref = m.astype(np.float32).astype(np.float64).copy()
    v_ref = v.astype(np.float32).astype(np.float64).copy()
    O.mlp_adam(th_ref, m_ref, v_ref, g.cpu().numpy().astype(np.float64), t, lr=1e-3)
    for got, ref, name in ((thd, th_ref, "theta"), (md, m_ref, "m"), (vd, v_ref, "v")):
        d = np.max(np.abs(got.cpu().numpy() - ref)) / np.max(np.abs(ref))
        assert d <= 1e-5, (name, d)


def test_training_fits_a_teacher_network():
    # a student trained with the GPU Adam steps on samples labelled by a
    # random teacher network (the oracle's forward pass) reduces its loss
    from oracle import oracle as O
    from paper_1607_02214_amd import ppmlr
    teacher = _params(20, scale=0.7)
    X = I.mlp_samples(8192, seed=21, spread=0.7)
    Y = O.mlp_forward(teacher, X.astype(np.float64))
    Xd, Yd = _dev(X), _dev(Y)
    th = _dev(I.mlp_init(22))
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    mlp = ppmlr.MLP(1024)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    _, l0 = mlp.grad(th, Xd[:1024], Yd[:1024])
    l0 = float(l0.item())
    for t in range(1, 601):
        b = (t - 1) % 8
        mlp.train_step(th, m, v, Xd[b * 1024:(b + 1) * 1024], Yd[b * 1024:(b + 1) * 1024], t, lr=3e-3, loss=loss)
    _, l1 = mlp.grad(th, Xd[:1024], Yd[:1024])
    l1 = float(l1.item())
    GC.log(f"[mlp] teacher fit: loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.2 * l0


def test_rejects_bad_batches():
    from paper_1607_02214_amd import ppmlr
    mlp = ppmlr.MLP(64)
    th = _dev(I.mlp_init(0))
    X = _dev(I.mlp_samples(65))
    Y = _dev(np.zeros((65, 2)))
    with pytest.raises(ppmlr.PPMLRError):
        mlp.grad(th, X, Y)           # more samples than the workspace holds
    with pytest.raises(ValueError):
        mlp.forward(th, X[:, :10])   # too few input columns
