"""Relative error measures for comparing GPU results with the FP64 oracle.

The NLL has an arbitrary additive offset and the gradient vanishes at the
minimum, so errors are scaled by the size of the terms that make them up:
  e_nll  = |dNLL| / (sum_i |ln I_i| + N_D |ln S|)      (Eq. 2 form; + S for Eq. 3)
  e_grad = max|dgrad| / (max|grad_data| + max|grad_MC|)
with grad_data = -2 sum conj(A) z/I and grad_MC = 2 c sum w conj(A) z taken
separately (c = N_D / sum w I, or 1/N_gen for the Eq. 3 form).
"""
import numpy as np

import oracle

TOL = {"f32": 1e-6, "f64": 1e-12}


def reference(Ad, Am, V, w=None, n_gen=None, extended=False):
    nll, grad, parts = oracle.nll_grad(Ad, Am, V, w=w, n_gen=n_gen, extended=extended, parts=True)
    nd = Ad.shape[0]
    ng = float(n_gen) if n_gen else float(Am.shape[0])
    S = parts["s_raw"] / ng
    I = oracle.intensity(Ad, V) if nd else np.ones(0)
    if extended:
        s_nll = float(np.sum(np.abs(np.log(I)))) + abs(S)
        c = 1.0 / ng
    else:
        s_nll = float(np.sum(np.abs(np.log(I)))) + nd * abs(np.log(S)) if nd else 1.0
        c = nd / parts["s_raw"] if nd else 0.0
    gd = np.max(np.abs(2 * parts["GD"])) if nd else 0.0
    gm = np.max(np.abs(2 * c * parts["HM"]))
    return dict(nll=nll, grad=grad, s_nll=max(s_nll, 1e-300), s_grad=max(gd + gm, 1e-300))


def errors(ref, nll, grad):
    e_n = abs(nll - ref["nll"]) / ref["s_nll"]
    e_g = float(np.max(np.abs(np.asarray(grad) - ref["grad"]))) / ref["s_grad"]
    return e_n, e_g


def reference_fast(Ad, Am, V, w=None, n_gen=None, extended=False, threads=0):
    """reference() for large samples: the oracle's chunked sums on `threads`
    host threads (0: all), whose values agree with the single-pass oracle
    within 1e-14 of the term scale (pinned on the CPU), and the NLL scale's
    sum |ln I| from a numpy pass.  Pass complex128 arrays to avoid a copy per
    call."""
    nll, grad, parts = oracle.nll_grad_chunked(Ad, Am, V, w=w, n_gen=n_gen, extended=extended, threads=threads,
                                               parts=True)
    nd = Ad.shape[0]
    ng = float(n_gen) if n_gen else float(Am.shape[0])
    S = parts["s_raw"] / ng
    Vc = np.asarray(V, dtype=np.complex128)
    abs_log = 0.0
    for r0 in range(0, nd, 1 << 18):
        z = Ad[r0:r0 + (1 << 18)] @ Vc
        abs_log += float(np.sum(np.abs(np.log(z.real * z.real + z.imag * z.imag))))
    if extended:
        s_nll = abs_log + abs(S)
        c = 1.0 / ng
    else:
        s_nll = abs_log + nd * abs(np.log(S)) if nd else 1.0
        c = nd / parts["s_raw"] if nd else 0.0
    gd = np.max(np.abs(2 * parts["GD"])) if nd else 0.0
    gm = np.max(np.abs(2 * c * parts["HM"]))
    return dict(nll=nll, grad=grad, s_nll=max(s_nll, 1e-300), s_grad=max(gd + gm, 1e-300))
