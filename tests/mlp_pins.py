"""Pins of the surrogate-network oracle (oracle/mlp.py) to facts outside it.

Each pin takes the oracle module as an argument so that the mutation test can
run the same pins against deliberately broken copies of it.
"""
import math

import numpy as np
from scipy.stats import norm

import synth


def _net(M, n_in, hidden, seed):
    g = np.random.default_rng(seed)
    P = g.normal(0.0, 0.7, M.param_count(n_in, hidden))
    return P


def pin_gelu_closed_forms(M):
    """GELU(x) = x Phi(x): GELU(0) = 0, GELU(x) - GELU(-x) = x, values against the
    normal CDF of scipy, derivative against central differences of scipy's form."""
    x = np.linspace(-6, 6, 97)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(M.gelu(x) - M.gelu(-x), x, rtol=0, atol=1e-14)
    assert np.allclose(M.gelu(x), x * norm.cdf(x), rtol=1e-13, atol=1e-15)
    h = 1e-5
    fd = ((x + h) * norm.cdf(x + h) - (x - h) * norm.cdf(x - h)) / (2 * h)
    assert np.allclose(M.gelu_d(x), fd, rtol=0, atol=1e-9)
    assert abs(M.gelu_d(np.array([0.0]))[0] - 0.5) < 1e-15


def pin_gradient_finite_differences(M):
    """Exact (unrounded) network: every parameter's gradient against central
    differences of the mean squared error."""
    n_in, hidden, B = 5, 4, 7
    P = _net(M, n_in, hidden, 1)
    g = np.random.default_rng(2)
    X = g.normal(size=(B, n_in))
    t = g.normal(size=B)
    loss, G = M.loss_grad(P, X, t, n_in, hidden, rounding=False)
    y = M.forward(P, X, n_in, hidden, rounding=False)["y"]
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-14 * max(1.0, loss)
    h = 1e-6
    for i in range(P.size):
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        lp = np.mean((M.forward(Pp, X, n_in, hidden, rounding=False)["y"] - t) ** 2)
        lm = np.mean((M.forward(Pm, X, n_in, hidden, rounding=False)["y"] - t) ** 2)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - G[i]) <= 1e-7 * (1.0 + abs(fd)), (i, fd, G[i])


def pin_against_torch_autograd(M):
    """Exact network: output and gradient against PyTorch float64 autograd
    (linear layers, exact GELU, mean squared error)."""
    import torch
    n_in, hidden, B = 32, 48, 50
    P = _net(M, n_in, hidden, 3) * 0.3
    g = np.random.default_rng(4)
    X = g.normal(size=(B, n_in))
    t = g.normal(size=B)
    loss, G = M.loss_grad(P, X, t, n_in, hidden, rounding=False)
    parts = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in M.unpack(P, n_in, hidden)]
    W1, b1, W2, b2, w3, b3 = parts
    Xt = torch.tensor(X)
    h1 = torch.nn.functional.gelu(Xt @ W1.T + b1, approximate="none")
    h2 = torch.nn.functional.gelu(h1 @ W2.T + b2, approximate="none")
    y = h2 @ w3 + b3
    lt = torch.mean((y - torch.tensor(t)) ** 2)
    lt.backward()
    Gt = np.concatenate([p.grad.numpy().ravel() for p in parts])
    assert abs(loss - lt.item()) <= 1e-13 * lt.item()
    assert np.max(np.abs(G - Gt)) <= 1e-12 * np.max(np.abs(Gt))


def pin_adam_against_torch(M):
    """Three Adam steps against torch.optim.Adam in float64 (same gradients)."""
    import torch
    g = np.random.default_rng(5)
    P = g.normal(size=40)
    p = torch.tensor(P.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    for step in range(3):
        Gs = g.normal(size=P.size) * 10.0 ** g.uniform(-3, 1, P.size)
        p.grad = torch.tensor(Gs)
        opt.step()
        P, m, v = M.adam(P, Gs, m, v, step, 1e-2)
        assert np.max(np.abs(P - p.detach().numpy())) < 1e-14, step
    # first step from zero moments moves every parameter by lr * g / (|g| + eps)
    P1, _, _ = M.adam(np.zeros(3), np.array([2.0, -3e-4, 0.0]), np.zeros(3), np.zeros(3), 0, 0.1)
    assert np.allclose(P1, [-0.1 * 2 / (2 + 1e-8), 0.1 * 3e-4 / (3e-4 + 1e-8), 0.0], rtol=1e-14, atol=0)


def pin_features(M):
    """Canonical features: unit norm, V_0 real and non-negative, invariant under
    a global complex factor; a single wave maps to (1, 0); order of waves kept."""
    g = np.random.default_rng(6)
    V = synth.draw_v(g, 20, 7)
    X = M.features(V)
    C = X[:, 0::2] + 1j * X[:, 1::2]
    assert np.allclose(np.linalg.norm(C, axis=1), 1.0, atol=1e-15)
    assert np.all(np.abs(C[:, 0].imag) < 1e-15) and np.all(C[:, 0].real > 0)
    c = 3.7 * np.exp(1.1j)
    assert np.allclose(M.features(V * c), X, atol=1e-14)
    # |C_a| is |V_a| / |V| wave by wave
    assert np.allclose(np.abs(C), np.abs(V) / np.linalg.norm(V, axis=1, keepdims=True), atol=1e-15)
    # relative phases are kept: arg(C_a / C_0) = arg(V_a / V_0)
    assert np.allclose(np.exp(1j * np.angle(C[:, 1:] / C[:, :1])), np.exp(1j * np.angle(V[:, 1:] / V[:, :1])),
                       atol=1e-12)
    assert np.allclose(M.features(np.array([[-2.0 + 2.0j]])), [[1.0, 0.0]], atol=1e-15)


def pin_targets(M):
    nll = np.array([5.0, 3.0, np.inf, 3.0 + math.e - 1.0, np.nan])
    t = M.targets(nll)
    assert t[1] == 0.0 and t[0] == math.log(3.0) and abs(t[3] - 1.0) < 1e-15
    cap = math.log(3.0) + 1.0
    assert t[2] == cap and t[4] == cap


def pin_topk(M):
    """Smallest keys by brute force; ties by index; NaN last."""
    keys = np.array([3.0, 1.0, np.nan, 1.0, -2.0, 7.0, 1.0])
    assert list(M.topk(keys, 5)) == [4, 1, 3, 6, 0]
    assert list(M.topk(keys, 7)) == [4, 1, 3, 6, 0, 5, 2]
    g = np.random.default_rng(7)
    k2 = g.integers(0, 50, 1000).astype(float)
    brute = sorted(range(1000), key=lambda i: (k2[i], i))[:100]
    assert list(M.topk(k2, 100)) == brute


def pin_fp16_rounding(M):
    """Round-to-nearest-even at FP16 precision (11-bit significand), overflow to
    infinity above 65504 + half an ulp, subnormals down to 2^-24."""
    vals = np.array([1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 65504.0, 65520.0, 2.0 ** -24, 2.0 ** -25,
                     3 * 2.0 ** -25, -(1 + 2.0 ** -10)])
    want = np.array([1.0, 1 + 2.0 ** -9, 65504.0, np.inf, 2.0 ** -24, 0.0, 2 * 2.0 ** -24, -(1 + 2.0 ** -10)])
    assert np.array_equal(M.f16(vals), want)


def pin_rounding_points(M):
    """With FP16-exact inputs and weights the rounded network equals the exact one
    in its first layer (rounding acts on operands, not on results), and differs
    from it afterwards by no more than the FP16 operand error allows."""
    n_in, hidden, B = 8, 16, 9
    g = np.random.default_rng(8)
    P = np.round(g.normal(size=M.param_count(n_in, hidden)) * 64) / 256      # multiples of 2^-8, |.| < 2
    X = np.round(g.normal(size=(B, n_in)) * 64) / 256
    a = M.forward(P, X, n_in, hidden, rounding=True)
    b = M.forward(P, X, n_in, hidden, rounding=False)
    assert np.array_equal(a["Z1"], b["Z1"])
    W1, b1, W2, b2, w3, b3 = M.unpack(P, n_in, hidden)
    bound = 2.0 ** -10 * (np.abs(b["H1"]) @ np.abs(W2).T)            # one relative ulp on the H1 operand
    assert np.all(np.abs(a["Z2"] - b["Z2"]) <= bound * 1.01 + 1e-15)
    assert not np.array_equal(a["Z2"], b["Z2"])


PINS = [pin_gelu_closed_forms, pin_gradient_finite_differences, pin_against_torch_autograd, pin_adam_against_torch,
        pin_features, pin_targets, pin_topk, pin_fp16_rounding, pin_rounding_points]
