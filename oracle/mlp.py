"""FP64 CPU oracle of the NLL surrogate network (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the library never does.

Fits are repeated from many starting points to find the global minimum
(Berger, Section 2, and Section 4 on fits with many parameters).  A small
network ranks candidate starting vectors by a learned estimate of their NLL:

  features   V^ = V e^{-i arg V_0} / |V|, as (Re, Im) pairs: the Eq. 2 NLL does
             not change under a global phase or a global scale of V, so these
             are the coordinates it depends on;
  target     t = ln(1 + NLL - min NLL) over the training set;
  network    in -> H -> H -> 1, y = w3 . GELU(W2 GELU(W1 x + b1) + b2) + b3,
             GELU(x) = x Phi(x) with the exact normal CDF (erf form);
  loss       mean over the batch of (y - t)^2;
  optimiser  Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.

Parameters are one flat FP32 array [W1 (H x in) | b1 | W2 (H x H) | b2 | w3 | b3],
W stored row-major as (output, input).

With ``rounding=True`` the oracle rounds to FP16 at the points where the
matrix-core kernels do (every operand of a matrix product, and the head's
activations and weights) and keeps everything else in FP64, so that the
remaining difference from the kernels is FP32 accumulation and FP32 GELU
only.  With ``rounding=False`` it is the plain FP64 network, which the tests
pin to finite differences and to an independent autograd implementation.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

_SQRT1_2 = 0.70710678118654752440
_INV_SQRT_2PI = 0.39894228040143267794


def param_count(n_in: int, hidden: int) -> int:
    return hidden * n_in + hidden + hidden * hidden + hidden + hidden + 1


def unpack(P, n_in: int, hidden: int):
    P = np.asarray(P, dtype=np.float64)
    assert P.shape == (param_count(n_in, hidden),)
    o = 0
    W1 = P[o:o + hidden * n_in].reshape(hidden, n_in); o += hidden * n_in
    b1 = P[o:o + hidden]; o += hidden
    W2 = P[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b2 = P[o:o + hidden]; o += hidden
    w3 = P[o:o + hidden]; o += hidden
    b3 = P[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, np.ravel(b3)])


def f16(x):
    """Round to FP16 through FP32 (the kernels convert FP32 values)."""
    with np.errstate(over="ignore"):
        return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x * _SQRT1_2))


def gelu_d(x):
    """d GELU / dx = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x * _SQRT1_2)) + x * _INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(P, X, n_in: int, hidden: int, rounding: bool = True) -> dict:
    """Activations of every layer for the rows of X [B, n_in]."""
    r = f16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(P, n_in, hidden)
    X = np.asarray(X, dtype=np.float64)
    Z1 = r(X) @ r(W1).T + b1
    H1 = gelu(Z1)
    Z2 = r(H1) @ r(W2).T + b2
    H2 = gelu(Z2)
    y = r(H2) @ r(w3) + b3[0]
    return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, y=y)


def loss_grad(P, X, t, n_in: int, hidden: int, rounding: bool = True):
    """Mean squared error over the rows and its gradient with respect to P.

    Backward pass by the chain rule, layer by layer:
      dy = 2 (y - t) / B
      dw3 = H2^T dy, db3 = sum dy
      dZ2 = (dy w3^T) * GELU'(Z2); dW2 = dZ2^T H1, db2 = column sums of dZ2
      dZ1 = (dZ2 W2) * GELU'(Z1);  dW1 = dZ1^T X,  db1 = column sums of dZ1
    With rounding, every matrix-product operand is rounded as in the forward.
    The kernels carry dy without the 1/B (keeping the FP16 operands of the
    weight-gradient products away from the subnormal range) and scale the
    gradient by 1/B at the end; that is the same value up to rounding.
    """
    r = f16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, w3, b3 = unpack(P, n_in, hidden)
    a = forward(P, X, n_in, hidden, rounding)
    t = np.asarray(t, dtype=np.float64)
    B = t.shape[0]
    res = a["y"] - t
    loss = float(np.mean(res * res))
    dy_sum = 2.0 * res                      # gradient of the sum of squares
    dw3 = r(a["H2"]).T @ dy_sum
    db3 = np.array([dy_sum.sum()])
    dZ2 = np.outer(dy_sum, r(w3)) * gelu_d(a["Z2"])
    dW2 = r(dZ2).T @ r(a["H1"])
    db2 = dZ2.sum(0)
    dZ1 = (r(dZ2) @ r(W2)) * gelu_d(a["Z1"])
    dW1 = r(dZ1).T @ r(a["X"])
    db1 = dZ1.sum(0)
    G = pack(dW1, db1, dW2, db2, dw3, db3) / B
    return loss, G


def adam(P, G, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); step is the count before it."""
    t = step + 1
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * G
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * G * G
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return np.asarray(P, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def features(V) -> np.ndarray:
    """Canonical coordinates (Re, Im interleaved) of complex vectors V [n, k]."""
    V = np.asarray(V, dtype=np.complex128)
    nrm = np.linalg.norm(V, axis=1, keepdims=True)
    ph = np.exp(-1j * np.angle(V[:, :1]))
    C = V * ph / np.where(nrm > 0, nrm, 1.0)
    C[:, 0] = np.abs(V[:, 0]) / np.where(nrm[:, 0] > 0, nrm[:, 0], 1.0)     # real by construction
    X = np.empty((V.shape[0], 2 * V.shape[1]), dtype=np.float64)
    X[:, 0::2] = C.real
    X[:, 1::2] = C.imag
    return X


def targets(nll) -> np.ndarray:
    """t = ln(1 + NLL - min NLL) over finite values; a non-finite NLL gets the
    largest finite target plus one."""
    nll = np.asarray(nll, dtype=np.float64)
    fin = np.isfinite(nll)
    lo, hi = nll[fin].min(), nll[fin].max()
    t = np.full(nll.shape, np.log1p(hi - lo) + 1.0)
    t[fin] = np.log1p(nll[fin] - lo)
    return t


def topk(keys, k: int) -> np.ndarray:
    """Indices of the k smallest keys, ascending, ties by index, NaN counted as +inf."""
    keys = np.asarray(keys, dtype=np.float64)
    keys = np.where(np.isnan(keys), np.inf, keys)
    order = np.lexsort((np.arange(keys.shape[0]), keys))
    return order[:k]
