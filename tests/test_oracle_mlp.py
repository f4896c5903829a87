"""Pins of the oracle of the learned Riemann initial guess (14 -> 64 -> 64 -> 2
network, tanh-form GELU, MSE loss, Adam), against independent references:
the exact GELU x Phi(x), central finite differences, torch CPU autograd and
torch's Adam in float64."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def test_gelu_tanh_form_is_close_to_exact_gelu():
    from scipy.special import ndtr
    xs = np.linspace(-6, 6, 241)
    approx = np.array([O.mlp_gelu(x) for x in xs])
    exact = xs * ndtr(xs)
    assert np.max(np.abs(approx - exact)) < 1e-3       # published accuracy of the tanh form
    assert O.mlp_gelu(0.0) == 0.0
    assert abs(O.mlp_gelu(20.0) - 20.0) < 1e-12 and abs(O.mlp_gelu(-20.0)) < 1e-12


def test_gelu_derivative_matches_central_differences():
    for x in np.linspace(-5, 5, 41):
        h = 1e-6
        fd = (O.mlp_gelu(x + h) - O.mlp_gelu(x - h)) / (2 * h)
        assert abs(O.mlp_gelu_grad(x) - fd) < 1e-8


def _problem(seed=0, n=16):
    rng = np.random.default_rng(seed)
    theta = rng.normal(size=O.mlp_num_params()) * 0.2
    X = rng.normal(size=(n, O.MLP_IN))
    Y = rng.normal(size=(n, O.MLP_OUT))
    return theta, X, Y


def test_backward_matches_central_differences():
    theta, X, Y = _problem()
    loss, g = O.mlp_loss_grad(theta, X, Y)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(theta), 300, replace=False)
    for i in idx:
        h = 1e-5
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (O.mlp_loss_grad(tp, X, Y)[0] - O.mlp_loss_grad(tm, X, Y)[0]) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


def test_forward_and_backward_match_torch_autograd():
    torch = pytest.importorskip("torch")
    theta, X, Y = _problem(seed=3, n=32)
    W1, b1, W2, b2, W3, b3 = O.mlp_unpack(theta)
    T = lambda a: torch.tensor(np.array(a), dtype=torch.float64, requires_grad=True)
    tW1, tb1, tW2, tb2, tW3, tb3 = map(T, (W1, b1, W2, b2, W3, b3))
    x = torch.tensor(X)
    gelu = lambda z: torch.nn.functional.gelu(z, approximate="tanh")
    out = gelu(gelu(x @ tW1 + tb1) @ tW2 + tb2) @ tW3 + tb3
    loss = 0.5 * ((out - torch.tensor(Y)) ** 2).sum() / X.shape[0]
    loss.backward()
    assert np.allclose(O.mlp_forward(theta, X), out.detach().numpy(), rtol=1e-12, atol=1e-12)
    l_o, g_o = O.mlp_loss_grad(theta, X, Y)
    assert abs(l_o - loss.item()) < 1e-12
    g_t = np.concatenate([t.grad.numpy().ravel() for t in (tW1, tb1, tW2, tb2, tW3, tb3)])
    assert np.allclose(g_o, g_t, rtol=1e-10, atol=1e-13)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    theta, X, Y = _problem(seed=5)
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th = theta.copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, 6):
        _, g = O.mlp_loss_grad(th, X, Y)
        O.mlp_adam(th, m, v, g, t)
        opt.zero_grad()
        p.grad = torch.tensor(O.mlp_loss_grad(p.detach().numpy(), X, Y)[1])
        opt.step()
    assert np.allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_training_reduces_the_loss():
    theta, X, Y = _problem(seed=9, n=64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = O.mlp_loss_grad(theta, X, Y)[0]
    for t in range(1, 201):
        _, g = O.mlp_loss_grad(theta, X, Y)
        O.mlp_adam(theta, m, v, g, t, lr=3e-3)
    assert O.mlp_loss_grad(theta, X, Y)[0] < 0.5 * l0
