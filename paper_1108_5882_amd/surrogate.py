"""Surrogate-screened multi-start: the network picks the starts, the exact likelihood
judges and refines them.

Fits are repeated from many starting points because a minimiser can stop in a
local minimum (Berger, Section 2); with many parameters, repeating fits from
random starting values becomes very expensive (Section 4).  The pipeline:

  1. pairs    NLL of training vectors (matrix-core batched pass, split 3);
  2. train    the network on (canonical features, ln(1 + NLL - min NLL));
  3. screen   predict every candidate start and keep the `top` best;
  4. refine   batched L-BFGS from the kept starts (pwa_batch_fit);
  5. judge    exact NLL of the refined points (one streaming pass each).

The plain method runs steps 4-5 from random starts.  Every step is a call of
the library; this module moves arrays between them and times them.
"""
from __future__ import annotations

import time

import numpy as np


def _now(torch):
    torch.cuda.synchronize()
    return time.perf_counter()


def _interleave(V: np.ndarray) -> np.ndarray:
    out = np.empty((V.shape[0], 2 * V.shape[1]))
    out[:, 0::2], out[:, 1::2] = V.real, V.imag
    return out


def exact_pairs(ctx, V: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """NLL of every row of V [n, k] by the matrix-core pass with small coherent sums
    recomputed exactly (split 3), `chunk` vectors per call (a domain failure gives
    +inf for that vector only)."""
    from ._lib import DomainError
    out = np.empty(V.shape[0])
    for c in range(0, V.shape[0], chunk):
        part = V[c:c + chunk]
        try:
            out[c:c + part.shape[0]] = ctx.nll_batch(part, grad=False, split=3)
        except DomainError:
            out[c:c + part.shape[0]] = [_one(ctx, v) for v in part]
    return out


def _one(ctx, v):
    from ._lib import DomainError
    try:
        return ctx.nll_batch(v[None], grad=False, split=3)[0]
    except DomainError:
        return np.inf


def train(mlp, V: np.ndarray, nll: np.ndarray, perm: np.ndarray, batch: int, lr: float = 1e-3):
    """Fit the network to (features(V), ln(1 + NLL - min NLL)); perm gives the
    mini-batch order (int32, a multiple of batch long).  Returns per-step losses
    and ms per step."""
    import torch
    dev = mlp.device
    Vd = torch.from_numpy(_interleave(V)).to(dev)
    X = mlp.features(Vd)
    t = mlp.targets(torch.from_numpy(np.ascontiguousarray(nll, dtype=np.float64)).to(dev))
    losses, ms = mlp.train(X, t, torch.from_numpy(np.ascontiguousarray(perm, dtype=np.int32)).to(dev), batch, lr)
    return losses.cpu().numpy(), ms


def screen(mlp, V: np.ndarray, top: int):
    """Indices of the `top` candidates with the lowest predicted NLL, and all predictions."""
    import torch
    Vd = torch.from_numpy(_interleave(V)).to(mlp.device)
    y = mlp.predict(mlp.features(Vd))
    idx = mlp.select(y, top)
    return idx.cpu().numpy().astype(np.int64), y.cpu().numpy()


def refine_and_judge(ctx, V0: np.ndarray, iters: int):
    """Batched L-BFGS from V0, then the exact NLL (streaming pass) of each result."""
    V, nll_fit, status, ms = ctx.batch_fit(V0, iters)
    judged = ctx.nll_batch(V, grad=False, split=0)
    return dict(V=V, nll=judged, nll_fit=nll_fit, status=status, ms_per_iter=ms)


def multistart(ctx, mlp, V_train, V_screen, V_plain, perm, batch: int, iters: int, top: int = 256,
               lr: float = 1e-3, init=None):
    """Both arms on one likelihood context: the surrogate-screened starts and
    len(V_plain) random starts, refined for the same number of iterations.

    Returns a dict with each arm's judged NLLs, the wall time of every stage
    (seconds, device synchronised) and the training losses.
    """
    import torch
    if init is not None:
        mlp.set_params(init)
    t0 = _now(torch)
    nll_train = exact_pairs(ctx, V_train)
    t1 = _now(torch)
    losses, ms_step = train(mlp, V_train, nll_train, perm, batch, lr)
    t2 = _now(torch)
    idx, pred = screen(mlp, V_screen, top)
    t3 = _now(torch)
    sel = refine_and_judge(ctx, V_screen[idx], iters)
    t4 = _now(torch)
    plain = refine_and_judge(ctx, V_plain, iters)
    t5 = _now(torch)
    return dict(
        surrogate=dict(sel=idx, pred=pred, **sel),
        plain=plain,
        train_nll=nll_train,
        losses=losses,
        ms_per_train_step=ms_step,
        seconds=dict(pairs=t1 - t0, train=t2 - t1, screen=t3 - t2, refine_selected=t4 - t3,
                     refine_plain=t5 - t4),
    )
