"""ctypes binding of libpwa.so (include/pwa.h): argument marshalling only.

Every computation runs in the library's HIP kernels.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpwa.so")

# status codes (pwa_status)
OK, E_INVAL, E_NOMEM, E_HIP, E_DOMAIN, E_STATE, E_UNSUPPORTED = range(7)
F32, F64 = 0, 1
DATA, MC = 0, 1
MC_STREAM, MC_GRAM = 0, 1
HOST, DEVICE, BORROW = 0, 1, 2
MAX_K = 64

# every entry point declared in include/pwa.h
EXPORTS = [
    "pwa_create", "pwa_destroy", "pwa_set_amplitudes", "pwa_set_mc_mode", "pwa_nll",
    "pwa_nll_grad", "pwa_nll_grad_async", "pwa_nll_batch", "pwa_nll_batch_async", "pwa_hessian", "pwa_last_flags",
    "pwa_last_error",
    "pwa_layout_ld", "pwa_set_timing", "pwa_kernel_time", "pwa_get_stream_cfg",
    "pwa_set_stream_cfg", "pwa_autotune", "pwa_batch_kernel_time", "pwa_hessian_kernel_time",
    "pwa_multi_create", "pwa_multi_destroy", "pwa_multi_eval", "pwa_multi_reset", "pwa_multi_step",
    "pwa_multi_get", "pwa_multi_autotune", "pwa_multi_last_error", "pwa_batch_fit",
    "pwa_mlp_param_count", "pwa_mlp_create", "pwa_mlp_destroy", "pwa_mlp_set_params", "pwa_mlp_get_params",
    "pwa_mlp_features", "pwa_mlp_targets", "pwa_mlp_predict", "pwa_mlp_loss_grad", "pwa_mlp_train",
    "pwa_mlp_select", "pwa_mlp_last_error", "pwa_nll_grad_noalloc",
    "pwa_kin_create", "pwa_kin_destroy", "pwa_kin_set_events", "pwa_kin_set_mode", "pwa_kin_nll_grad",
    "pwa_kin_nll_grad_async", "pwa_kin_last_error",
]


class FitDesc(ctypes.Structure):
    """pwa_fit_desc: one fit of a multi-fit set (host arrays)."""
    _fields_ = [("A_data", ctypes.c_void_p), ("n_data", ctypes.c_int64), ("A_mc", ctypes.c_void_p),
                ("n_mc", ctypes.c_int64), ("w_mc", ctypes.c_void_p), ("n_gen", ctypes.c_double),
                ("k", ctypes.c_int32), ("ld", ctypes.c_int64), ("V0", ctypes.c_void_p)]


class StreamCfg(ctypes.Structure):
    """pwa_stream_cfg: launch configuration of the single-V streaming kernel."""
    _fields_ = [("lanes_per_row", ctypes.c_int32), ("complex_per_lane", ctypes.c_int32),
                ("rows_per_stage", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PwaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"pwa status {status}: {message}")
        self.status = status
        self.message = message


class DomainError(PwaError):
    """NLL = +inf: a data intensity or the normalisation is not positive."""


_lib = None


def _hip_runtime_of_torch() -> Optional[str]:
    """Path of the HIP runtime bundled with PyTorch, if PyTorch is installed."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return None
    p = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    return p if os.path.exists(p) else None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built).

    A process must hold one HIP runtime so that streams and device pointers
    can pass between PyTorch and this library.  PyTorch ships its own
    libamdhip64 (same soname as the system one, different file), so that file
    is loaded first when PyTorch is installed; the library's dependency on
    the soname then resolves to it, whichever of the two is imported first.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_1108_5882_amd.build.build()")
    rt = _hip_runtime_of_torch()
    if rt is not None:
        ctypes.CDLL(rt, mode=ctypes.RTLD_GLOBAL)
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    sig = {
        "pwa_create": [ctypes.POINTER(P), ctypes.c_int, ctypes.c_int, P],
        "pwa_destroy": [P],
        "pwa_set_amplitudes": [P, ctypes.c_int, P, I64, I32, I64, ctypes.c_int, P, D],
        "pwa_set_mc_mode": [P, ctypes.c_int, ctypes.c_int],
        "pwa_nll": [P, P, P],
        "pwa_nll_grad": [P, P, P, P],
        "pwa_nll_grad_async": [P, P, P],
        "pwa_nll_batch": [P, I32, P, P, P, I32],
        "pwa_nll_batch_async": [P, I32, P, P, I32],
        "pwa_hessian": [P, P, P],
        "pwa_last_flags": [P, ctypes.POINTER(ctypes.c_uint32)],
        "pwa_layout_ld": [P, I32, ctypes.POINTER(I64)],
        "pwa_set_timing": [P, ctypes.c_int],
        "pwa_kernel_time": [P, ctypes.POINTER(D), ctypes.POINTER(I64)],
        "pwa_batch_kernel_time": [P, ctypes.POINTER(D), ctypes.POINTER(I64)],
        "pwa_hessian_kernel_time": [P, ctypes.POINTER(D), ctypes.POINTER(I64)],
        "pwa_get_stream_cfg": [P, ctypes.POINTER(StreamCfg)],
        "pwa_set_stream_cfg": [P, ctypes.POINTER(StreamCfg)],
        "pwa_autotune": [P, I32, ctypes.POINTER(StreamCfg), ctypes.POINTER(D)],
        "pwa_batch_fit": [P, I32, P, I32, ctypes.c_int, D, P, P, P, ctypes.POINTER(D)],
        "pwa_multi_create": [ctypes.POINTER(P), ctypes.c_int, I32, ctypes.POINTER(FitDesc), P],
        "pwa_multi_destroy": [P],
        "pwa_multi_eval": [P, P, P, P],
        "pwa_multi_reset": [P, P],
        "pwa_multi_step": [P, I32, ctypes.POINTER(D)],
        "pwa_multi_get": [P, P, P, P, P],
        "pwa_multi_autotune": [P, I32, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(D)],
        "pwa_mlp_create": [ctypes.POINTER(P), ctypes.c_int, I32, I32, I32, P],
        "pwa_mlp_destroy": [P],
        "pwa_mlp_set_params": [P, P, ctypes.c_int],
        "pwa_mlp_get_params": [P, P, ctypes.c_int],
        "pwa_mlp_features": [P, P, I64, I32, P],
        "pwa_mlp_targets": [P, P, I64, P],
        "pwa_mlp_predict": [P, P, I64, P],
        "pwa_mlp_loss_grad": [P, P, P, I32, ctypes.POINTER(ctypes.c_float), P],
        "pwa_mlp_train": [P, P, P, I64, P, I32, I32, ctypes.c_float, P, ctypes.POINTER(D)],
        "pwa_mlp_select": [P, P, I64, I32, P],
        "pwa_nll_grad_noalloc": [ctypes.c_int, P, I64, P, I64, P, D, I32, I64, ctypes.c_int, P, P, P],
        "pwa_kin_create": [ctypes.POINTER(P), ctypes.c_int, I32, P, P],
        "pwa_kin_destroy": [P],
        "pwa_kin_set_events": [P, ctypes.c_int, P, I64, ctypes.c_int, P, D],
        "pwa_kin_set_mode": [P, ctypes.c_int],
        "pwa_kin_nll_grad": [P, P, P, P, P, P],
        "pwa_kin_nll_grad_async": [P, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = st
    lib.pwa_last_error.argtypes = [P]
    lib.pwa_last_error.restype = ctypes.c_char_p
    lib.pwa_multi_last_error.argtypes = [P]
    lib.pwa_multi_last_error.restype = ctypes.c_char_p
    lib.pwa_kin_last_error.argtypes = [P]
    lib.pwa_kin_last_error.restype = ctypes.c_char_p
    lib.pwa_mlp_last_error.argtypes = [P]
    lib.pwa_mlp_last_error.restype = ctypes.c_char_p
    lib.pwa_mlp_param_count.argtypes = [I32, I32]
    lib.pwa_mlp_param_count.restype = I64
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)    # torch.cuda.Stream


def nll_grad_noalloc(A_data, A_mc, V_dev, out_dev, w_mc=None, n_gen: Optional[float] = None,
                     extended: bool = False, stream=None, k: Optional[int] = None):
    """NLL and gradient over caller-owned GPU samples with no context and no
    allocation (pwa_nll_grad_noalloc): A_data [n_d, ld], A_mc [n_m, ld] complex64
    or complex128 GPU tensors in the library's layout (ld = layout width of k,
    zero padding columns; k defaults to ld), w_mc matching real weights or None,
    V_dev float64 [2k], out_dev float64 [2k + 2] (nll, grad[2k], flags).  The
    kernel is enqueued on `stream` (torch.cuda.Stream, raw handle or None) of the
    tensors' device; nothing waits."""
    import torch
    lib = load()
    if A_data.dtype not in (torch.complex64, torch.complex128) or A_mc.dtype != A_data.dtype:
        raise TypeError("A_data and A_mc must both be complex64 or both complex128")
    prec = F32 if A_data.dtype == torch.complex64 else F64
    dev = A_data.device
    real = torch.float32 if prec == F32 else torch.float64
    for t, name, dt in ((A_mc, "A_mc", A_data.dtype), (V_dev, "V_dev", torch.float64),
                        (out_dev, "out_dev", torch.float64)) + (((w_mc, "w_mc", real),) if w_mc is not None else ()):
        if not _is_torch(t) or not t.is_cuda or t.device != dev or t.dtype != dt:
            raise TypeError(f"{name} must be a {dt} tensor on {dev}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if not A_data.is_cuda or not A_data.is_contiguous() or A_data.dim() != 2 or A_mc.dim() != 2:
        raise ValueError("A_data and A_mc must be contiguous 2-d GPU tensors")
    ld = A_data.shape[1]
    if A_mc.shape[1] != ld:
        raise ValueError("A_data and A_mc must have the same row width")
    k = ld if k is None else int(k)
    if V_dev.numel() != 2 * k or out_dev.numel() != 2 * k + 2:
        raise ValueError("V_dev must hold 2k and out_dev 2k + 2 doubles")
    if w_mc is not None and w_mc.numel() != A_mc.shape[0]:
        raise ValueError("w_mc must hold one weight per MC row")
    s = _stream_handle(stream)
    with torch.cuda.device(dev):
        st = lib.pwa_nll_grad_noalloc(prec, ctypes.c_void_p(A_data.data_ptr()), A_data.shape[0],
                                      ctypes.c_void_p(A_mc.data_ptr()), A_mc.shape[0],
                                      None if w_mc is None else ctypes.c_void_p(w_mc.data_ptr()),
                                      float(n_gen or 0.0), k, ld, int(bool(extended)),
                                      ctypes.c_void_p(V_dev.data_ptr()), ctypes.c_void_p(out_dev.data_ptr()),
                                      None if s is None else ctypes.c_void_p(s))
    if st != OK:
        msg = lib.pwa_last_error(None)
        raise PwaError(st, msg.decode() if msg else "")


class Context:
    """One likelihood context on one GPU (pwa_ctx).

    precision: "f32" (FP32 amplitudes, FP64 sums) or "f64".
    stream: torch.cuda.Stream, raw hipStream_t int, or None for a private stream.
    """

    def __init__(self, device: int = 0, precision: str = "f32", stream=None):
        self.lib = load()
        self.device = int(device)
        self.prec = {"f32": F32, "f64": F64}[precision]
        self.real = np.float32 if self.prec == F32 else np.float64
        self.cplx = np.complex64 if self.prec == F32 else np.complex128
        self._stream_obj = stream          # keep a torch stream alive
        self._borrowed = {}                # sample -> tensors the library reads in place
        self._vbuf = self._obuf = None     # host V and result buffers of the synchronous calls
        h = ctypes.c_void_p()
        s = _stream_handle(stream)
        self._check(self.lib.pwa_create(ctypes.byref(h), device, self.prec,
                                        None if s is None else ctypes.c_void_p(s)), None)
        self.h = h
        self.k = None

    # ------------------------------------------------------------ helpers
    def _check(self, status: int, h=-1):
        if status == OK:
            return
        msg = self.lib.pwa_last_error(self.h if h == -1 else h)
        msg = msg.decode() if msg else ""
        cls = DomainError if status == E_DOMAIN else PwaError
        raise cls(status, msg)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.pwa_destroy(self.h)
            self.h = ctypes.c_void_p()
        self._borrowed = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ samples
    def _check_device_tensor(self, t, name: str, dtype):
        """t must be a tensor on this context's GPU with the given torch dtype."""
        if not _is_torch(t) or not t.is_cuda:
            raise TypeError(f"{name} must be a torch tensor on a GPU")
        if t.device.index != self.device:
            raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")

    def set_amplitudes(self, which: str, A, w=None, n_gen: Optional[float] = None, borrow: bool = False,
                       k: Optional[int] = None):
        """which: "data" or "mc".  A: numpy [n, k] complex (host) or a torch
        tensor [n, k] complex (a CPU tensor is read as host memory, a GPU tensor
        must be on the context's device); w: matching weights or None.

        borrow=True: A (a GPU tensor [n, layout_ld(k)] with zero padding
        columns; k defaults to its width) and w are used in place with no
        copy; the context keeps references to them until the sample is
        replaced or the context closed."""
        wh = {"data": DATA, "mc": MC}[which]
        if _is_torch(A) and not A.is_cuda:
            if borrow:
                raise TypeError("only a GPU tensor can be borrowed")
            A = A.numpy()
            w = None if w is None else (w.numpy() if _is_torch(w) else w)
        if _is_torch(A):
            import torch
            self._check_device_tensor(A, "A", {F32: torch.complex64, F64: torch.complex128}[self.prec])
            if A.dim() != 2:
                raise ValueError("A must be [n, k]")
            n = A.shape[0]
            k = A.shape[1] if k is None else int(k)
            if not 1 <= k <= A.shape[1]:
                raise ValueError("k must be between 1 and the width of A")
            ld = A.stride(0)
            if A.stride(1) != 1:
                raise ValueError("A must have unit stride along k")
            if borrow:
                ld_dev = self.layout_ld(k)
                if n > 1 and ld != ld_dev:
                    raise ValueError(f"a borrowed A needs row stride {ld_dev} for k = {k}, got {ld}")
                ld = ld_dev
            wp = None
            if w is not None:
                self._check_device_tensor(w, "w", {F32: torch.float32, F64: torch.float64}[self.prec])
                if not w.is_contiguous() or w.numel() != n:
                    raise ValueError("w must be contiguous [n]")
                wp = ctypes.c_void_p(w.data_ptr())
            self._check(self.lib.pwa_set_amplitudes(self.h, wh, ctypes.c_void_p(A.data_ptr()), n, k, ld,
                                                    BORROW if borrow else DEVICE, wp, float(n_gen or 0.0)))
            if borrow:
                self._borrowed[which] = (A, w)
            else:
                self._borrowed.pop(which, None)
        else:
            if borrow:
                raise TypeError("only a GPU tensor can be borrowed")
            A = np.ascontiguousarray(A, dtype=self.cplx)
            if A.ndim != 2:
                raise ValueError("A must be [n, k]")
            n, k = A.shape
            wa = None if w is None else np.ascontiguousarray(w, dtype=self.real)
            if wa is not None and wa.shape != (n,):
                raise ValueError("w must be [n]")
            self._check(self.lib.pwa_set_amplitudes(self.h, wh, _ptr(A), n, k, k, HOST, _ptr(wa),
                                                    float(n_gen or 0.0)))
            self._borrowed.pop(which, None)
        if self.k != k:
            self._borrowed = {which: self._borrowed[which]} if which in self._borrowed else {}
        self.k = k

    def set_mc_mode(self, mode: str = "stream", extended: bool = False):
        self._check(self.lib.pwa_set_mc_mode(self.h, {"stream": MC_STREAM, "gram": MC_GRAM}[mode],
                                             int(bool(extended))))

    # --------------------------------------------------------- evaluation
    def _v(self, V) -> np.ndarray:
        V = np.asarray(V)
        if np.iscomplexobj(V):
            out = np.empty(2 * V.size)
            out[0::2], out[1::2] = V.real, V.imag
            return out
        return np.ascontiguousarray(V, dtype=np.float64)

    def _stage_v(self, V):
        """Copies V ([k] complex or [2k] real) into the context's host buffer;
        returns (address of V, address of the result buffer [nll, grad[2k]])."""
        if self.k is None:
            raise PwaError(E_STATE, "no sample set")
        n = 2 * self.k
        if self._vbuf is None or self._vbuf.size != n:
            self._vbuf = np.zeros(n)
            self._obuf = np.zeros(n + 1)
            self._vptr = self._vbuf.ctypes.data
            self._optr = self._obuf.ctypes.data
        if isinstance(V, np.ndarray) and V.dtype == np.complex128 and V.ndim == 1 and V.flags.c_contiguous:
            v = V.view(np.float64)
        else:
            v = self._v(V).ravel()
        if v.size != n:
            raise ValueError(f"V must hold {self.k} complex (or {n} real) values, got {v.size} reals")
        self._vbuf[:] = v
        return self._vptr, self._optr

    def nll(self, V) -> float:
        vp, op = self._stage_v(V)
        self._check(self.lib.pwa_nll(self.h, vp, op))
        return float(self._obuf[0])

    def nll_grad(self, V):
        """(NLL, gradient[2k]) with gradient = (dNLL/dRe V_a, dNLL/dIm V_a) interleaved."""
        vp, op = self._stage_v(V)
        self._check(self.lib.pwa_nll_grad(self.h, vp, op, op + 8))
        return float(self._obuf[0]), self._obuf[1:].copy()

    def nll_grad_async(self, V_dev, out_dev):
        """V_dev: torch float64 [2k] on the context's GPU; out_dev: the same, [2k+2]."""
        import torch
        self._check_device_tensor(V_dev, "V_dev", torch.float64)
        self._check_device_tensor(out_dev, "out_dev", torch.float64)
        if self.k is None or V_dev.numel() != 2 * self.k or out_dev.numel() != 2 * self.k + 2:
            raise ValueError("V_dev must hold 2k and out_dev 2k + 2 doubles")
        if not (V_dev.is_contiguous() and out_dev.is_contiguous()):
            raise ValueError("V_dev and out_dev must be contiguous")
        self._check(self.lib.pwa_nll_grad_async(self.h, ctypes.c_void_p(V_dev.data_ptr()),
                                                ctypes.c_void_p(out_dev.data_ptr())))

    def nll_batch(self, Vs, grad: bool = True, split: int = 2):
        """NLL (and gradients) for the rows of Vs [nv, k] complex (or [nv, 2k] real).
        split 2: matrix-core pass for all vectors; split 3: the same with small
        coherent sums recomputed exactly; split 0: one streaming pass each."""
        Vs = np.asarray(Vs)
        if np.iscomplexobj(Vs):
            v = np.empty((Vs.shape[0], 2 * Vs.shape[1]))
            v[:, 0::2], v[:, 1::2] = Vs.real, Vs.imag
        else:
            v = np.ascontiguousarray(Vs, dtype=np.float64).reshape(Vs.shape[0], -1)
        nv = v.shape[0]
        nll = np.zeros(nv)
        g = np.zeros_like(v) if grad else None
        self._check(self.lib.pwa_nll_batch(self.h, nv, _ptr(v), _ptr(nll), _ptr(g), int(split)))
        return (nll, g) if grad else nll

    def hessian(self, V):
        """2k x 2k Hessian of the NLL at V ([k] complex or [2k] real) in the real
        parameters (Re V_a, Im V_a interleaved)."""
        V = np.asarray(V)
        if np.iscomplexobj(V):
            v = np.empty(2 * V.shape[0])
            v[0::2], v[1::2] = V.real, V.imag
        else:
            v = np.ascontiguousarray(V, dtype=np.float64).ravel()
        H = np.zeros((v.shape[0], v.shape[0]))
        self._check(self.lib.pwa_hessian(self.h, _ptr(v), _ptr(H)))
        return H

    def nll_batch_async(self, V_dev, out_dev, split: int = 2):
        """V_dev: torch cuda float64 [nv, 2k] contiguous; out_dev: torch cuda float64
        [nv, 2k + 2] contiguous (per vector: nll, grad[2k], flags).  Enqueued on
        the context's stream; a synchronous nll_batch with at least nv vectors and
        the same split must have prepared the workspace."""
        import torch
        self._check_device_tensor(V_dev, "V_dev", torch.float64)
        self._check_device_tensor(out_dev, "out_dev", torch.float64)
        if V_dev.dim() != 2 or out_dev.dim() != 2:
            raise ValueError("V_dev must be [nv, 2k] and out_dev [nv, 2k + 2]")
        nv = V_dev.shape[0]
        if not (V_dev.is_contiguous() and out_dev.is_contiguous()):
            raise ValueError("V_dev and out_dev must be contiguous")
        if V_dev.shape[1] != 2 * self.k or tuple(out_dev.shape) != (nv, 2 * self.k + 2):
            raise ValueError("V_dev must be [nv, 2k] and out_dev [nv, 2k + 2]")
        self._check(self.lib.pwa_nll_batch_async(self.h, nv, ctypes.c_void_p(V_dev.data_ptr()),
                                                 ctypes.c_void_p(out_dev.data_ptr()), int(split)))

    def batch_fit(self, V0, iters: int, polar: bool = False, rmin: float = 0.0):
        """L-BFGS from every row of V0 [nv, k] (complex) at once, each iteration one
        split-3 matrix-core evaluation of all trial points; in (Re, Im) or, with
        polar, in (|V|, arg V) with |V| >= rmin and arg V_0 = 0.  Returns
        (V [nv, k] complex, nll [nv], status [nv], ms per iteration)."""
        V0 = np.asarray(V0)
        v = np.empty((V0.shape[0], 2 * V0.shape[1]))
        v[:, 0::2], v[:, 1::2] = V0.real, V0.imag
        out = np.zeros_like(v)
        nll = np.zeros(V0.shape[0])
        st = np.zeros(V0.shape[0], dtype=np.int32)
        ms = ctypes.c_double()
        self._check(self.lib.pwa_batch_fit(self.h, V0.shape[0], _ptr(v), int(iters), int(bool(polar)), float(rmin),
                                           _ptr(out), _ptr(nll), _ptr(st), ctypes.byref(ms)))
        return out[:, 0::2] + 1j * out[:, 1::2], nll, st, ms.value

    def last_flags(self) -> int:
        f = ctypes.c_uint32()
        self._check(self.lib.pwa_last_flags(self.h, ctypes.byref(f)))
        return int(f.value)

    def layout_ld(self, k: int) -> int:
        ld = ctypes.c_int64()
        self._check(self.lib.pwa_layout_ld(self.h, k, ctypes.byref(ld)))
        return int(ld.value)

    def set_timing(self, enable: bool):
        self._check(self.lib.pwa_set_timing(self.h, int(bool(enable))))

    def stream_cfg(self) -> dict:
        c = StreamCfg()
        self._check(self.lib.pwa_get_stream_cfg(self.h, ctypes.byref(c)))
        return c.as_dict()

    def set_stream_cfg(self, lanes_per_row, complex_per_lane, rows_per_stage, blocks_per_cu):
        c = StreamCfg(lanes_per_row, complex_per_lane, rows_per_stage, blocks_per_cu)
        self._check(self.lib.pwa_set_stream_cfg(self.h, ctypes.byref(c)))

    def autotune(self, reps: int = 5):
        """Times every compiled configuration on the current samples; keeps the fastest.
        Returns (configuration dict, average kernel ms)."""
        c = StreamCfg()
        ms = ctypes.c_double()
        self._check(self.lib.pwa_autotune(self.h, int(reps), ctypes.byref(c), ctypes.byref(ms)))
        return c.as_dict(), ms.value

    def kernel_time(self):
        """(average ms, count) of the single-V streaming kernels since the last query."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.pwa_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def batch_kernel_time(self):
        """(average ms, count) of the matrix-core batched kernels since the last query."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.pwa_batch_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def hessian_kernel_time(self):
        """(average ms, count) of the Hessian's kernels (per call) since the last query."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.pwa_hessian_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class KinContext:
    """Likelihood with amplitudes formed on the GPU from each event's kinematics
    (pwa_kin): resonance masses and widths are parameters next to V.

    spins: the J of each wave (0..4).  Events: (m, cos theta) pairs [n, 2].
    """

    def __init__(self, spins, device: int = 0, stream=None):
        self.lib = load()
        self.device = int(device)
        sp = np.ascontiguousarray(spins, dtype=np.int32)
        self.k = int(sp.size)
        self._stream_obj = stream
        self._borrowed = {}
        h = ctypes.c_void_p()
        s = _stream_handle(stream)
        self._check(self.lib.pwa_kin_create(ctypes.byref(h), device, self.k, _ptr(sp),
                                            None if s is None else ctypes.c_void_p(s)), None)
        self.h = h
        self._buf = np.zeros(4 * self.k + 1)
        self._in = np.zeros(4 * self.k)

    def _check(self, status: int, h=-1):
        if status == OK:
            return
        msg = self.lib.pwa_kin_last_error(self.h if h == -1 else h)
        msg = msg.decode() if msg else ""
        raise (DomainError if status == E_DOMAIN else PwaError)(status, msg)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.pwa_kin_destroy(self.h)
            self.h = ctypes.c_void_p()
        self._borrowed = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_events(self, which: str, mx, w=None, n_gen: Optional[float] = None, borrow: bool = False):
        """mx: [n, 2] float32 (m, cos theta) as numpy (host) or a GPU tensor (copied, or
        used in place with borrow=True); w: matching float32 weights or None."""
        wh = {"data": DATA, "mc": MC}[which]
        if _is_torch(mx) and mx.is_cuda:
            import torch
            for t, name in ((mx, "mx"),) + (((w, "w"),) if w is not None else ()):
                if not _is_torch(t) or t.device.index != self.device or t.dtype != torch.float32 \
                        or not t.is_contiguous():
                    raise TypeError(f"{name} must be a contiguous float32 tensor on cuda:{self.device}")
            if mx.dim() != 2 or mx.shape[1] != 2 or (w is not None and w.numel() != mx.shape[0]):
                raise ValueError("mx must be [n, 2] and w [n]")
            self._check(self.lib.pwa_kin_set_events(self.h, wh, ctypes.c_void_p(mx.data_ptr()), mx.shape[0],
                                                    BORROW if borrow else DEVICE,
                                                    None if w is None else ctypes.c_void_p(w.data_ptr()),
                                                    float(n_gen or 0.0)))
            if borrow:
                self._borrowed[which] = (mx, w)
            else:
                self._borrowed.pop(which, None)
            return
        if borrow:
            raise TypeError("only a GPU tensor can be borrowed")
        mx = np.ascontiguousarray(mx.cpu().numpy() if _is_torch(mx) else mx, dtype=np.float32)
        if mx.ndim != 2 or mx.shape[1] != 2:
            raise ValueError("mx must be [n, 2]")
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        if wa is not None and wa.shape != (mx.shape[0],):
            raise ValueError("w must be [n]")
        self._check(self.lib.pwa_kin_set_events(self.h, wh, _ptr(mx), mx.shape[0], HOST, _ptr(wa),
                                                float(n_gen or 0.0)))
        self._borrowed.pop(which, None)

    def set_mode(self, extended: bool = False):
        self._check(self.lib.pwa_kin_set_mode(self.h, int(bool(extended))))

    def nll_grad(self, V, res):
        """(NLL, gradient in V [2k] (Re, Im interleaved), gradient in res [2k]
        (d/dm_a, d/dGamma_a interleaved)) at V ([k] complex or [2k] real) and
        res = (m_a, Gamma_a) interleaved [2k]."""
        V = np.asarray(V)
        k = self.k
        if np.iscomplexobj(V):
            self._in[0:2 * k:2], self._in[1:2 * k:2] = V.real, V.imag
        else:
            self._in[:2 * k] = np.asarray(V, dtype=np.float64).ravel()
        self._in[2 * k:] = np.asarray(res, dtype=np.float64).ravel()
        b = self._buf.ctypes.data
        self._check(self.lib.pwa_kin_nll_grad(self.h, self._in.ctypes.data, self._in.ctypes.data + 16 * k, b,
                                              b + 8, b + 8 + 16 * k))
        return float(self._buf[0]), self._buf[1:1 + 2 * k].copy(), self._buf[1 + 2 * k:].copy()

    def nll_grad_async(self, V_dev, res_dev, out_dev):
        """V_dev, res_dev: float64 GPU tensors [2k]; out_dev float64 [4k + 2]
        (nll, grad_v[2k], grad_res[2k], flags); enqueued on the context's stream."""
        import torch
        for t, name, nv in ((V_dev, "V_dev", 2 * self.k), (res_dev, "res_dev", 2 * self.k),
                            (out_dev, "out_dev", 4 * self.k + 2)):
            if not _is_torch(t) or not t.is_cuda or t.device.index != self.device or t.dtype != torch.float64:
                raise TypeError(f"{name} must be a float64 tensor on cuda:{self.device}")
            if t.numel() != nv or not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous with {nv} elements")
        self._check(self.lib.pwa_kin_nll_grad_async(self.h, ctypes.c_void_p(V_dev.data_ptr()),
                                                    ctypes.c_void_p(res_dev.data_ptr()),
                                                    ctypes.c_void_p(out_dev.data_ptr())))


class MultiFit:
    """Many independent fits minimised together on one GPU (pwa_multi).

    samples: list of (A_data [n_d, k] complex64, A_mc [n_m, k] complex64, w_mc or None,
    n_gen or None); V0: list of complex [k] start vectors.
    """

    def __init__(self, samples, V0, device: int = 0, stream=None):
        self.lib = load()
        self.ks = []
        self._keep = []
        descs = (FitDesc * len(samples))()
        for f, ((Ad, Am, w, ng), v0) in enumerate(zip(samples, V0)):
            Ad = np.ascontiguousarray(Ad, dtype=np.complex64)
            Am = np.ascontiguousarray(Am, dtype=np.complex64)
            k = Ad.shape[1]
            wa = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
            v = np.empty(2 * k)
            v0 = np.asarray(v0)
            v[0::2], v[1::2] = v0.real, v0.imag
            self._keep += [Ad, Am, wa, v]
            self.ks.append(k)
            descs[f] = FitDesc(Ad.ctypes.data, Ad.shape[0], Am.ctypes.data, Am.shape[0],
                               None if wa is None else wa.ctypes.data, float(ng or 0.0), k, k,
                               v.ctypes.data)
        h = ctypes.c_void_p()
        s = _stream_handle(stream)
        st = self.lib.pwa_multi_create(ctypes.byref(h), device, len(samples), descs,
                                       None if s is None else ctypes.c_void_p(s))
        self._keep = []
        self.h = h
        self._check(st, None)
        self.n = 2 * sum(self.ks)

    def _check(self, status: int, h=-1):
        if status == OK:
            return
        msg = self.lib.pwa_multi_last_error(self.h if h == -1 else h)
        msg = msg.decode() if msg else ""
        raise (DomainError if status == E_DOMAIN else PwaError)(status, msg)

    def _concat(self, Vs):
        out = np.empty(self.n)
        off = 0
        for k, v in zip(self.ks, Vs):
            v = np.asarray(v)
            out[off:off + 2 * k:2], out[off + 1:off + 2 * k:2] = v.real, v.imag
            off += 2 * k
        return out

    def _split(self, flat):
        res, off = [], 0
        for k in self.ks:
            res.append(flat[off:off + 2 * k:2] + 1j * flat[off + 1:off + 2 * k:2])
            off += 2 * k
        return res

    def eval(self, Vs):
        """(nll[nfits], list of real gradients) at the complex vectors Vs."""
        v = self._concat(Vs)
        nll = np.zeros(len(self.ks))
        g = np.zeros(self.n)
        self._check(self.lib.pwa_multi_eval(self.h, _ptr(v), _ptr(nll), _ptr(g)))
        grads, off = [], 0
        for k in self.ks:
            grads.append(g[off:off + 2 * k].copy())
            off += 2 * k
        return nll, grads

    def reset(self, Vs):
        v = self._concat(Vs)
        self._check(self.lib.pwa_multi_reset(self.h, _ptr(v)))

    def step(self, steps: int = 1) -> float:
        """Replay `steps` minimiser iterations; returns the average ms per iteration."""
        ms = ctypes.c_double()
        self._check(self.lib.pwa_multi_step(self.h, int(steps), ctypes.byref(ms)))
        return ms.value

    def get(self):
        """(list of complex V, nll[nfits], status[nfits], iters[nfits])."""
        v = np.zeros(self.n)
        nll = np.zeros(len(self.ks))
        st = np.zeros(len(self.ks), dtype=np.int32)
        it = np.zeros(len(self.ks), dtype=np.int32)
        self._check(self.lib.pwa_multi_get(self.h, _ptr(v), _ptr(nll), _ptr(st), _ptr(it)))
        return self._split(v), nll, st, it

    def autotune(self, reps: int = 3):
        b = ctypes.c_int64()
        c = ctypes.c_int32()
        ms = ctypes.c_double()
        self._check(self.lib.pwa_multi_autotune(self.h, int(reps), ctypes.byref(b), ctypes.byref(c),
                                                ctypes.byref(ms)))
        return {"item_bytes": b.value, "blocks_per_cu": c.value}, ms.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.pwa_multi_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """Surrogate network in -> hidden -> hidden -> 1 on one GPU (pwa_mlp).

    Array arguments are torch CUDA tensors (the library reads and writes them in
    place); work is ordered after the caller's current PyTorch stream and the
    calls return when it has finished.
    """

    def __init__(self, n_in: int, hidden: int = 256, max_batch: int = 8192, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        self.n_in, self.hidden, self.max_batch = int(n_in), int(hidden), int(max_batch)
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        self.h = None
        self._check(self.lib.pwa_mlp_create(ctypes.byref(h), device, self.n_in, self.hidden, self.max_batch,
                                            ctypes.c_void_p(int(self.stream.cuda_stream))), None)
        self.h = h
        self.nparams = int(self.lib.pwa_mlp_param_count(self.n_in, self.hidden))

    def _check(self, status: int, h=-1):
        if status == OK:
            return
        msg = self.lib.pwa_mlp_last_error(self.h if h == -1 else h)
        msg = msg.decode() if msg else ""
        raise PwaError(status, msg)

    def _dev(self, t, dtype, shape=None, name="array"):
        torch = self.torch
        if not (torch.is_tensor(t) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous CUDA tensor of {dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def _sync_in(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def set_params(self, P):
        """P: host numpy float32 [nparams] or a CUDA float32 tensor; resets Adam."""
        if self.torch.is_tensor(P):
            self._sync_in()
            self._check(self.lib.pwa_mlp_set_params(self.h, self._dev(P, self.torch.float32, (self.nparams,)),
                                                    DEVICE))
        else:
            p = np.ascontiguousarray(P, dtype=np.float32)
            if p.shape != (self.nparams,):
                raise ValueError(f"P must have shape ({self.nparams},)")
            self._check(self.lib.pwa_mlp_set_params(self.h, _ptr(p), HOST))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.pwa_mlp_get_params(self.h, _ptr(p), HOST))
        return p

    def features(self, V):
        """V: CUDA float64 [n, 2k] (interleaved complex) -> CUDA float32 [n, 2k]."""
        torch = self.torch
        n, kk = V.shape
        X = torch.empty((n, kk), dtype=torch.float32, device=self.device)
        self._sync_in()
        self._check(self.lib.pwa_mlp_features(self.h, self._dev(V, torch.float64, name="V"), n, kk // 2,
                                              ctypes.c_void_p(X.data_ptr())))
        return X

    def targets(self, nll):
        torch = self.torch
        t = torch.empty(nll.shape[0], dtype=torch.float32, device=self.device)
        self._sync_in()
        self._check(self.lib.pwa_mlp_targets(self.h, self._dev(nll, torch.float64, name="nll"), nll.shape[0],
                                             ctypes.c_void_p(t.data_ptr())))
        return t

    def predict(self, X):
        torch = self.torch
        n = X.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        self._sync_in()
        self._check(self.lib.pwa_mlp_predict(self.h, self._dev(X, torch.float32, (n, self.n_in), "X"), n,
                                             ctypes.c_void_p(y.data_ptr())))
        return y

    def loss_grad(self, X, t):
        torch = self.torch
        B = X.shape[0]
        G = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        loss = ctypes.c_float()
        self._sync_in()
        self._check(self.lib.pwa_mlp_loss_grad(self.h, self._dev(X, torch.float32, (B, self.n_in), "X"),
                                               self._dev(t, torch.float32, (B,), "t"), B, ctypes.byref(loss),
                                               ctypes.c_void_p(G.data_ptr())))
        return float(loss.value), G

    def train(self, X, t, perm, batch: int, lr: float = 1e-3):
        """Adam steps over the rows perm[s * batch: (s + 1) * batch] for every s;
        perm: CUDA int32 tensor.  Returns (per-step losses, ms per step)."""
        torch = self.torch
        n = X.shape[0]
        nsteps = perm.numel() // batch
        hist = torch.empty(max(nsteps, 1), dtype=torch.float32, device=self.device)
        ms = ctypes.c_double()
        self._sync_in()
        self._check(self.lib.pwa_mlp_train(self.h, self._dev(X, torch.float32, (n, self.n_in), "X"),
                                           self._dev(t, torch.float32, (n,), "t"),
                                           n, self._dev(perm, torch.int32, name="perm"), int(batch), int(nsteps),
                                           float(lr), ctypes.c_void_p(hist.data_ptr()), ctypes.byref(ms)))
        return hist[:nsteps], ms.value

    def select(self, keys, k: int):
        """Indices (CUDA int32 [k]) of the k smallest keys, ascending."""
        torch = self.torch
        idx = torch.empty(k, dtype=torch.int32, device=self.device)
        self._sync_in()
        self._check(self.lib.pwa_mlp_select(self.h, self._dev(keys, torch.float32, name="keys"), keys.shape[0],
                                            int(k), ctypes.c_void_p(idx.data_ptr())))
        return idx

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.pwa_mlp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
