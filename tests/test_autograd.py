"""dNLL/dV through torch.autograd.Function: PyTorch's complex-gradient convention,
central finite differences (h = 1e-4, FP64), gradcheck, and the oracle gradient."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1108_5882_amd.autograd import _NLLFunction


class _OracleBacked:
    """Stand-in for a library context on the CPU: only for testing the autograd glue."""

    def __init__(self, Ad, Am):
        self.Ad, self.Am, self.k = Ad, Am, Ad.shape[1]
        self.ctx = self

    def nll_grad(self, V):
        return oracle.nll_grad(self.Ad, self.Am, V)


def test_glue_gradcheck_cpu():
    """The Function's backward follows PyTorch's convention (checked with the oracle on CPU)."""
    g = np.random.default_rng(3)
    lik = _OracleBacked(synth.random_amplitudes(g, 40, 3, np.complex128),
                        synth.random_amplitudes(g, 120, 3, np.complex128))
    V = torch.tensor(synth.draw_v(g, 1, 3)[0], dtype=torch.complex128, requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: _NLLFunction.apply(v, lik), (V,), eps=1e-6, atol=1e-5)
    nll = _NLLFunction.apply(V, lik)
    nll.backward()
    _, ref = oracle.nll_grad(lik.Ad, lik.Am, V.detach().numpy())
    assert np.allclose(V.grad.numpy(), ref[0::2] + 1j * ref[1::2], rtol=1e-12, atol=0)


@pytest.mark.gpu
@pytest.mark.parametrize("device", ["cuda", "cpu"])
def test_autograd_gpu_gradcheck_and_fd(device):
    from paper_1108_5882_amd.autograd import Likelihood
    g = np.random.default_rng(5)
    Ad = synth.random_amplitudes(g, 60, 3, np.complex128)
    Am = synth.random_amplitudes(g, 200, 3, np.complex128)
    lik = Likelihood(Ad, Am, precision="f64")
    V = torch.tensor(synth.draw_v(g, 1, 3)[0], dtype=torch.complex128, device=device, requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: lik(v), (V,), eps=1e-6, atol=1e-6)
    nll = lik(V)
    nll.backward()
    grad = V.grad.detach().cpu().numpy()
    # central differences, h = 1e-4, one Richardson step, in (Re V, Im V)
    v0 = V.detach().cpu().numpy()
    f = lambda v: oracle.nll_grad(Ad, Am, v)[0]
    fd = np.empty(3, complex)
    for a in range(3):
        parts = []
        for e in (1.0, 1j):
            def d(h):
                dv = np.zeros(3, complex)
                dv[a] = e * h
                return (f(v0 + dv) - f(v0 - dv)) / (2 * h)
            parts.append((4 * d(5e-5) - d(1e-4)) / 3)
        fd[a] = parts[0] + 1j * parts[1]
    assert np.max(np.abs(grad - fd)) < 1e-7 * np.max(np.abs(fd))
    _, ref = oracle.nll_grad(Ad, Am, v0)
    assert np.max(np.abs(grad - (ref[0::2] + 1j * ref[1::2]))) < 1e-12 * np.max(np.abs(ref))
    lik.close()


@pytest.mark.gpu
def test_autograd_fp32_config_and_optimiser():
    """K = 4 stand-in (FP32 context): torch L-BFGS through the Function lowers the NLL
    and the gradient at the end matches the oracle at 1e-6."""
    from paper_1108_5882_amd.autograd import Likelihood
    from tests.tolerance import errors, reference
    s = synth.make_sample(0)
    Ad, Am = s.A_data.astype(np.complex64), s.A_mc.astype(np.complex64)
    lik = Likelihood(Ad, Am, precision="f32")
    V = torch.tensor(synth.eval_vectors(0, 1, 4)[0], dtype=torch.complex128, device="cuda",
                     requires_grad=True)
    opt = torch.optim.LBFGS([V], max_iter=60, line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        nll = lik(V)
        nll.backward()
        return nll

    start = float(lik(V.detach()))
    opt.step(closure)
    end = float(lik(V.detach()))
    assert end < start
    v = V.detach().cpu().numpy()
    vv = V.detach().clone().requires_grad_()
    out = lik(vv)
    out.backward()
    g = vv.grad.cpu().numpy()
    e_n, e_g = errors(reference(Ad, Am, v), float(out), np.stack([g.real, g.imag], 1).ravel())
    assert e_n < 1e-6 and e_g < 1e-6
    lik.close()
