"""FP64 CPU oracle for the unbinned partial-wave likelihood and its gradient.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  The GPU
library never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain double loops with Neumaier sums,
written from Eq. 1-3 of Berger, "Partial Wave Analysis using Graphics Cards",
Section 2); this module only marshals numpy arrays to it.  Every input is
converted to complex128/float64 first, which is exact for FP32 inputs.

Conventions (same as the C file):
  NLL      = -sum_i ln I_i + N_D ln S          (Eq. 2 form, default)
  NLL_ext  = -sum_i ln I_i + S                 (Eq. 3 form, extended=True)
  S        = (1/N_gen) sum_j w_j I_j
  gradient = real 2K vector (dNLL/dRe V_a, dNLL/dIm V_a) interleaved.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
KIN_SRC = os.path.join(_HERE, "kin.c")
LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off", "-fopenmp"]


def build(force: bool = True, src: str = SRC, out: str = LIB, kin_src: str = KIN_SRC) -> str:
    """Compile the oracle (oracle.c and kin.c) with gcc (no fast-math: the
    compensated sums need IEEE order)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["gcc", *CFLAGS, src, kin_src, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def _c128(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Bindings to one build of oracle.c (the default build, or a test's variant)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.orc_intensity.argtypes = [I64, I32, P, I64, P, P]
        lib.orc_nll_grad.argtypes = [I64, P, I64, I64, P, I64, P, D, I32, P, ctypes.c_int, P, P, P]
        lib.orc_gram.argtypes = [I64, P, I64, P, D, I32, P]
        lib.orc_nll_grad_gram.argtypes = [I64, P, I64, I32, P, P, ctypes.c_int, P, P]
        fns = [lib.orc_intensity, lib.orc_nll_grad, lib.orc_gram, lib.orc_nll_grad_gram]
        self.has_chunked = hasattr(lib, "orc_nll_grad_chunked")
        if self.has_chunked:
            lib.orc_nll_grad_chunked.argtypes = [I64, P, I64, I64, P, I64, P, D, I32, P, ctypes.c_int,
                                                 ctypes.c_int, P, P, P]
            fns.append(lib.orc_nll_grad_chunked)
        self.has_kin = hasattr(lib, "orc_kin_nll_grad")
        if self.has_kin:
            lib.orc_kin_amplitudes.argtypes = [I64, P, I32, P, P, P]
            lib.orc_kin_nll_grad.argtypes = [I64, P, I64, P, P, D, I32, P, P, P, ctypes.c_int, P, P, P, P]
            fns += [lib.orc_kin_amplitudes, lib.orc_kin_nll_grad]
        for f in fns:
            f.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def intensity(self, A, V) -> np.ndarray:
        """Eq. 1 per event: I_i = |sum_a V_a A_ia|^2."""
        A = _c128(A)
        V = _c128(V).ravel()
        n, k = A.shape
        out = np.empty(n)
        if self.lib.orc_intensity(n, k, _ptr(A), k, _ptr(V), _ptr(out)):
            raise ValueError("oracle: invalid arguments")
        return out

    def nll_grad(self, A_data, A_mc, V, w=None, n_gen=None, extended=False, parts=False):
        """NLL and real gradient by streaming both samples (Eq. 2, or Eq. 3 if extended).

        Returns (nll, grad[2K]) or, with parts=True, (nll, grad, raw sums).
        """
        V = _c128(V).ravel()
        k = V.shape[0]
        Ad = _c128(A_data).reshape(-1, k)
        Am = _c128(A_mc).reshape(-1, k)
        wm = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        ng = float(n_gen) if n_gen is not None else 0.0
        nll = np.zeros(1)
        grad = np.zeros(2 * k)
        pr = np.zeros(2 + 4 * k)
        if self.lib.orc_nll_grad(Ad.shape[0], _ptr(Ad), k, Am.shape[0], _ptr(Am), k, _ptr(wm), ng,
                                 k, _ptr(V), int(bool(extended)), _ptr(nll), _ptr(grad), _ptr(pr)):
            raise ValueError("oracle: invalid arguments")
        if parts:
            d = dict(sum_log=pr[0], s_raw=pr[1], GD=pr[2:2 + 2 * k].copy(), HM=pr[2 + 2 * k:].copy())
            return float(nll[0]), grad, d
        return float(nll[0]), grad

    def nll_grad_chunked(self, A_data, A_mc, V, w=None, n_gen=None, extended=False, threads=0, parts=False):
        """nll_grad with the events cut into fixed chunks summed on `threads` threads
        (0: all); the result does not depend on the thread count."""
        V = _c128(V).ravel()
        k = V.shape[0]
        Ad = _c128(A_data).reshape(-1, k)
        Am = _c128(A_mc).reshape(-1, k)
        wm = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        ng = float(n_gen) if n_gen is not None else 0.0
        nll = np.zeros(1)
        grad = np.zeros(2 * k)
        pr = np.zeros(2 + 4 * k)
        if self.lib.orc_nll_grad_chunked(Ad.shape[0], _ptr(Ad), k, Am.shape[0], _ptr(Am), k, _ptr(wm), ng, k,
                                         _ptr(V), int(bool(extended)), int(threads), _ptr(nll), _ptr(grad),
                                         _ptr(pr)):
            raise ValueError("oracle: invalid arguments")
        if parts:
            d = dict(sum_log=pr[0], s_raw=pr[1], GD=pr[2:2 + 2 * k].copy(), HM=pr[2 + 2 * k:].copy())
            return float(nll[0]), grad, d
        return float(nll[0]), grad

    def kin_amplitudes(self, mx, spins, res) -> np.ndarray:
        """A [n, k] complex: BW_a(m) Y_{J_a}^0(x) from the kinematics mx [n, 2] = (m, cos theta),
        res = (m_a, Gamma_a) interleaved and the spins J_a."""
        mx = np.ascontiguousarray(mx, dtype=np.float64).reshape(-1, 2)
        sp = np.ascontiguousarray(spins, dtype=np.int32)
        r = np.ascontiguousarray(res, dtype=np.float64).ravel()
        A = np.empty((mx.shape[0], sp.size), dtype=np.complex128)
        if self.lib.orc_kin_amplitudes(mx.shape[0], _ptr(mx), sp.size, _ptr(sp), _ptr(r), _ptr(A)):
            raise ValueError("oracle: invalid arguments")
        return A

    def kin_nll_grad(self, mx_data, mx_mc, V, res, spins, w=None, n_gen=None, extended=False, parts=False):
        """NLL, V gradient [2k] and resonance gradient [2k] = (dNLL/dm_a, dNLL/dGamma_a)
        with amplitudes from the kinematics (Eq. 2, or Eq. 3 if extended); with
        parts=True also the raw sums (sum_log, s_raw, GD, HM, RD, RM)."""
        V = _c128(V).ravel()
        k = V.size
        sp = np.ascontiguousarray(spins, dtype=np.int32)
        r = np.ascontiguousarray(res, dtype=np.float64).ravel()
        md = np.ascontiguousarray(mx_data, dtype=np.float64).reshape(-1, 2)
        mm = np.ascontiguousarray(mx_mc, dtype=np.float64).reshape(-1, 2)
        wm = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        nll = np.zeros(1)
        gv = np.zeros(2 * k)
        gr = np.zeros(2 * k)
        pr = np.zeros(2 + 8 * k)
        if sp.size != k or r.size != 2 * k or self.lib.orc_kin_nll_grad(
                md.shape[0], _ptr(md), mm.shape[0], _ptr(mm), _ptr(wm), float(n_gen or 0.0), k, _ptr(sp),
                _ptr(r), _ptr(V), int(bool(extended)), _ptr(nll), _ptr(gv), _ptr(gr), _ptr(pr)):
            raise ValueError("oracle: invalid arguments")
        if parts:
            d = dict(sum_log=pr[0], s_raw=pr[1], GD=pr[2:2 + 2 * k].copy(), HM=pr[2 + 2 * k:2 + 4 * k].copy(),
                     RD=pr[2 + 4 * k:2 + 6 * k].copy(), RM=pr[2 + 6 * k:].copy())
            return float(nll[0]), gv, gr, d
        return float(nll[0]), gv, gr

    def gram(self, A_mc, w=None, n_gen=None) -> np.ndarray:
        """MC integral matrix M_ab = (1/N_gen) sum_j w_j conj(A_ja) A_jb (bracket of Eq. 3)."""
        Am = _c128(A_mc)
        n, k = Am.shape
        wm = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        M = np.zeros((k, k), dtype=np.complex128)
        if self.lib.orc_gram(n, _ptr(Am), k, _ptr(wm), float(n_gen) if n_gen else 0.0, k, _ptr(M)):
            raise ValueError("oracle: invalid arguments")
        return M

    def nll_grad_gram(self, A_data, M, V, extended=False):
        """NLL and gradient with the precomputed MC matrix: S = V^H M V."""
        V = _c128(V).ravel()
        k = V.shape[0]
        Ad = _c128(A_data).reshape(-1, k)
        M = _c128(M).reshape(k, k)
        nll = np.zeros(1)
        grad = np.zeros(2 * k)
        if self.lib.orc_nll_grad_gram(Ad.shape[0], _ptr(Ad), k, k, _ptr(M), _ptr(V),
                                      int(bool(extended)), _ptr(nll), _ptr(grad)):
            raise ValueError("oracle: invalid arguments")
        return float(nll[0]), grad

    def nll_grad_batch(self, A_data, A_mc, Vs, w=None, n_gen=None, extended=False):
        """nll_grad for each row of Vs [nv, K]: (nll[nv], grad[nv, 2K])."""
        Vs = _c128(Vs)
        Ad = _c128(A_data)
        Am = _c128(A_mc)
        out_n = np.empty(Vs.shape[0])
        out_g = np.empty((Vs.shape[0], 2 * Vs.shape[1]))
        for b in range(Vs.shape[0]):
            out_n[b], out_g[b] = self.nll_grad(Ad, Am, Vs[b], w=w, n_gen=n_gen, extended=extended)
        return out_n, out_g


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build()
        _default = Oracle(LIB)
    return _default


def intensity(A, V):
    return default().intensity(A, V)


def nll_grad(A_data, A_mc, V, w=None, n_gen=None, extended=False, parts=False):
    return default().nll_grad(A_data, A_mc, V, w=w, n_gen=n_gen, extended=extended, parts=parts)


def nll_grad_chunked(A_data, A_mc, V, w=None, n_gen=None, extended=False, threads=0, parts=False):
    return default().nll_grad_chunked(A_data, A_mc, V, w=w, n_gen=n_gen, extended=extended, threads=threads,
                                      parts=parts)


def kin_amplitudes(mx, spins, res):
    return default().kin_amplitudes(mx, spins, res)


def kin_nll_grad(mx_data, mx_mc, V, res, spins, w=None, n_gen=None, extended=False, parts=False):
    return default().kin_nll_grad(mx_data, mx_mc, V, res, spins, w=w, n_gen=n_gen, extended=extended, parts=parts)


def gram(A_mc, w=None, n_gen=None):
    return default().gram(A_mc, w=w, n_gen=n_gen)


def nll_grad_gram(A_data, M, V, extended=False):
    return default().nll_grad_gram(A_data, M, V, extended=extended)


def nll_grad_batch(A_data, A_mc, Vs, w=None, n_gen=None, extended=False):
    return default().nll_grad_batch(A_data, A_mc, Vs, w=w, n_gen=n_gen, extended=extended)


def complex_grad(grad) -> np.ndarray:
    """Real interleaved gradient -> complex dNLL/dRe V + i dNLL/dIm V."""
    g = np.asarray(grad)
    return g[..., 0::2] + 1j * g[..., 1::2]
