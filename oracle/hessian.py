"""FP64 CPU oracle for the Hessian of the negative log-likelihood (error matrix).

TEST INFRASTRUCTURE ONLY: the test suite is the only code allowed to import
this module; the GPU library shares no code with it.

The fit's error matrix is the inverse of the NLL's second-derivative matrix
(Berger, Section 4: error calculations take much of a fit's computing time).
Written from the definitions in the real parameters x (x_{2a} = Re V_a,
x_{2a+1} = Im V_a), with no simplification:

  z_i = sum_a V_a A_ia = b_i . x,   b_{i,2a} = A_ia,  b_{i,2a+1} = i A_ia
  I_i = |z_i|^2
  dI_i/dx_m        = 2 Re(conj(z_i) b_im)
  d2I_i/dx_m dx_n  = 2 Re(conj(b_im) b_in)
  d2 ln I_i        = d2I_i / I_i - dI_i dI_i^T / I_i^2
  S                = (1/N_gen) sum_j w_j I_j          (MC rows, Eq. 2 and 3)
  Eq. 2 form:  H = -sum_i d2 ln I_i + N_D (d2S / S - dS dS^T / S^2)
  Eq. 3 form:  H = -sum_i d2 ln I_i + d2S

Every input is converted to complex128 / float64 first (exact for FP32 data).
"""
from __future__ import annotations

import numpy as np


def _b(A: np.ndarray) -> np.ndarray:
    """dz/dx per row: [n, 2K] complex."""
    A = np.asarray(A, dtype=np.complex128)
    b = np.empty((A.shape[0], 2 * A.shape[1]), dtype=np.complex128)
    b[:, 0::2] = A
    b[:, 1::2] = 1j * A
    return b


def _x(V: np.ndarray) -> np.ndarray:
    V = np.asarray(V, dtype=np.complex128).ravel()
    x = np.empty(2 * V.shape[0])
    x[0::2], x[1::2] = V.real, V.imag
    return x


def _intensity_derivs(A, x):
    """I, dI [n, 2K] and the pieces of d2I for each row."""
    b = _b(A)
    z = b @ x
    I = (z.real ** 2 + z.imag ** 2)
    dI = 2.0 * (np.conj(z)[:, None] * b).real
    return b, z, I, dI


def hessian_parts(A_data, A_mc, V, w=None, n_gen=None):
    """Raw sums: (sum_i d2 ln I_i, S, dS, d2S, N_D) in the real parameters."""
    x = _x(V)
    bd, _, Id, dId = _intensity_derivs(A_data, x)
    nd = bd.shape[0]
    # sum_i d2I_i / I_i, term by term
    d2 = 2.0 * np.einsum("im,in,i->mn", np.conj(bd), bd, 1.0 / Id).real if nd else np.zeros((x.size, x.size))
    outer = np.einsum("im,in,i->mn", dId, dId, 1.0 / Id ** 2) if nd else np.zeros((x.size, x.size))
    h_log = d2 - outer
    bm, _, Im, dIm = _intensity_derivs(A_mc, x)
    wm = np.ones(bm.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    ng = float(n_gen) if n_gen else float(bm.shape[0])
    S = float(np.sum(wm * Im)) / ng
    dS = (wm[:, None] * dIm).sum(axis=0) / ng
    d2S = 2.0 * np.einsum("jm,jn,j->mn", np.conj(bm), bm, wm).real / ng
    return h_log, S, dS, d2S, nd


def hessian(A_data, A_mc, V, w=None, n_gen=None, extended=False, parts=False):
    """2K x 2K Hessian of the NLL at V (Eq. 2 form, or Eq. 3 if extended).

    With parts=True also returns the data term (-sum d2 ln I) and the
    normalisation term separately (their scales set the comparison tolerance).
    """
    h_log, S, dS, d2S, nd = hessian_parts(A_data, A_mc, V, w=w, n_gen=n_gen)
    h_data = -h_log
    if extended:
        h_mc = d2S
    else:
        h_mc = nd * (d2S / S - np.outer(dS, dS) / S ** 2) if nd else np.zeros_like(d2S)
    H = h_data + h_mc
    return (H, h_data, h_mc) if parts else H
