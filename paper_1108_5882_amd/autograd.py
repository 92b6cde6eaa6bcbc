"""PyTorch autograd for the likelihood: dNLL/dV through torch.autograd.Function.

The forward pass is the library's fused NLL + gradient evaluation (one pass
over the amplitude rows, Eq. 2 or Eq. 3 of Berger, Section 2); it saves the
gradient, and the backward pass only scales it by the incoming gradient, so a
backward costs no extra pass over the rows.

Gradient convention: for the real NLL of complex V, PyTorch's gradient is
dNLL/dRe V + i dNLL/dIm V (twice the conjugate Wirtinger derivative), which is
the library's real gradient (dNLL/dRe V_a, dNLL/dIm V_a) read as complex
numbers.  Minimisers that work on real parameters (Section 4, "Fits with
complex parameters") can use V.grad directly.

V on a GPU: the evaluation is enqueued with the device-side entry point on
the context's stream, ordered after the current PyTorch stream and before
later work on it (no host synchronisation).  V on the CPU: the synchronous
entry point.  NLL is +inf where the likelihood is not defined (a data
intensity or the normalisation is not positive).
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import Context


class _NLLFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, V: torch.Tensor, lik: "Likelihood"):
        if not V.is_complex():
            raise TypeError("V must be a complex tensor")
        k = V.shape[-1]
        if V.dim() != 1 or k != lik.k:
            raise ValueError(f"V must have shape [{lik.k}]")
        if V.is_cuda:
            v = torch.view_as_real(V.detach().to(torch.complex128).contiguous()).reshape(-1).contiguous()
            out = torch.empty(2 * k + 2, dtype=torch.float64, device=V.device)
            cur = torch.cuda.current_stream(V.device)
            lik.stream.wait_stream(cur)
            lik.ctx.nll_grad_async(v, out)
            cur.wait_stream(lik.stream)
            v.record_stream(lik.stream)
            out.record_stream(lik.stream)
            nll = out[0]
            g = out[1:1 + 2 * k]
        else:
            nll_f, g_np = lik.ctx.nll_grad(V.detach().to(torch.complex128).numpy())
            nll = torch.tensor(nll_f, dtype=torch.float64)
            g = torch.from_numpy(g_np)
        grad_c = torch.complex(g[0::2], g[1::2]).to(V.dtype)
        fctx.save_for_backward(grad_c)
        return nll.to(V.real.dtype)

    @staticmethod
    def backward(fctx, grad_out):
        (grad_c,) = fctx.saved_tensors
        return grad_out.to(grad_c.real.dtype) * grad_c, None


class Likelihood:
    """Differentiable unbinned NLL over samples held by one library context.

    Build with the amplitude samples, then call ``lik(V)`` on a complex tensor
    V [k]; ``nll.backward()`` fills ``V.grad``.  ``precision`` "f32" or "f64";
    ``mode`` "stream" or "gram"; ``extended`` selects the Eq. 3 form.
    """

    def __init__(self, A_data, A_mc, w=None, n_gen=None, precision="f32", device=0,
                 mode="stream", extended=False):
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.ctx = Context(device, precision, stream=self.stream)
        self.ctx.set_amplitudes("data", A_data)
        self.ctx.set_amplitudes("mc", A_mc, w=w, n_gen=n_gen)
        self.ctx.set_mc_mode(mode, extended)
        self.k = int(np.shape(A_data)[1]) if not torch.is_tensor(A_data) else int(A_data.shape[1])
        if mode == "gram":
            # build the MC matrix now: the device-side entry point never allocates or waits
            try:
                self.ctx.nll(np.ones(self.k, dtype=np.complex128))
            except Exception:
                pass

    def __call__(self, V: torch.Tensor) -> torch.Tensor:
        return _NLLFunction.apply(V, self)

    def close(self):
        self.ctx.close()
