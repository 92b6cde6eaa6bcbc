"""The entry point that allocates nothing (pwa_nll_grad_noalloc) against the
context's device-side evaluation (pwa_nll_grad_async) on the same samples, two
calls in a row, the second on smaller samples, and against the FP64 oracle."""
import sys

import numpy as np
import pytest

import synth
from tests.tolerance import TOL, errors, reference

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _layout(torch, A, ld):
    n, k = A.shape
    t = torch.zeros((n, ld), dtype=torch.complex64 if A.dtype == np.complex64 else torch.complex128,
                    device="cuda:0")
    t[:, :k] = torch.from_numpy(A).cuda()
    return t


@pytest.mark.parametrize("prec,k", [("f32", 16), ("f32", 10), ("f64", 5)])
def test_noalloc_matches_async(prec, k):
    import torch

    import paper_1108_5882_amd as pwa
    g = np.random.default_rng(900 + k)
    dt = np.complex64 if prec == "f32" else np.complex128
    rdt = np.float32 if prec == "f32" else np.float64
    sizes = [(200003, 600011), (3001, 9007)]           # the second call is smaller
    for call, (nd, nm) in enumerate(sizes):
        _say(f"case noalloc prec={prec} k={k} call={call} nd={nd} nm={nm}")
        Ad = synth.random_amplitudes(g, nd, k, dt)
        Am = synth.random_amplitudes(g, nm, k, dt)
        w = g.uniform(0.5, 2.0, nm).astype(rdt)
        V = synth.draw_v(g, 1, k)[0]
        v = np.empty(2 * k)
        v[0::2], v[1::2] = V.real, V.imag
        Vd = torch.from_numpy(v).cuda()
        for extended in (False, True):
            with pwa.Context(0, prec) as c:
                ld = c.layout_ld(k)
                td, tm = _layout(torch, Ad, ld), _layout(torch, Am, ld)
                tw = torch.from_numpy(w).cuda()
                c.set_amplitudes("data", td, borrow=True, k=k)
                c.set_amplitudes("mc", tm, w=tw, n_gen=nm + 11, borrow=True, k=k)
                c.set_mc_mode("stream", extended)
                out_a = torch.full((2 * k + 2,), -7.0, dtype=torch.float64, device="cuda:0")
                c.nll_grad_async(Vd, out_a)
                torch.cuda.synchronize()
            out_n = torch.full((2 * k + 2,), -7.0, dtype=torch.float64, device="cuda:0")
            stream = torch.cuda.current_stream()
            pwa.nll_grad_noalloc(td, tm, Vd, out_n, w_mc=tw, n_gen=nm + 11, extended=extended, stream=stream, k=k)
            torch.cuda.synchronize()
            a, n = out_a.cpu().numpy(), out_n.cpu().numpy()
            ref = reference(Ad, Am, V, w=w, n_gen=nm + 11, extended=extended)
            e_n, e_g = errors(ref, n[0], n[1:1 + 2 * k])
            _say(f"  extended={extended} nll={n[0]:.12g} async={a[0]:.12g} e_nll={e_n:.2e} e_grad={e_g:.2e}")
            assert n[-1] == 0.0
            assert e_n < TOL[prec] and e_g < TOL[prec]
            ea, eg = errors(ref, a[0], a[1:1 + 2 * k])
            # same kernel, same grid and the same fixed summation order as the context's call
            assert np.array_equal(a, n), (a - n)


def test_noalloc_rejects_bad_arguments():
    import torch

    import paper_1108_5882_amd as pwa
    from paper_1108_5882_amd import _lib
    k = 10
    A = torch.zeros((64, 12), dtype=torch.complex64, device="cuda:0")
    Vd = torch.zeros(2 * k, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(2 * k + 2, dtype=torch.float64, device="cuda:0")
    lib = _lib.load()
    # row stride other than the layout width of k
    st = lib.pwa_nll_grad_noalloc(_lib.F32, A.data_ptr(), 64, A.data_ptr(), 64, None, 0.0, k, 11, 0,
                                  Vd.data_ptr(), out.data_ptr(), None)
    assert st == _lib.E_INVAL and b"layout" in lib.pwa_last_error(None)
    # k beyond the largest supported
    st = lib.pwa_nll_grad_noalloc(_lib.F32, A.data_ptr(), 64, A.data_ptr(), 64, None, 0.0, 65, 64, 0,
                                  Vd.data_ptr(), out.data_ptr(), None)
    assert st == _lib.E_UNSUPPORTED
    # data without MC rows
    st = lib.pwa_nll_grad_noalloc(_lib.F32, A.data_ptr(), 64, A.data_ptr(), 0, None, 0.0, k, 12, 0,
                                  Vd.data_ptr(), out.data_ptr(), None)
    assert st == _lib.E_INVAL
    # misaligned base
    flat = torch.zeros(64 * 12 + 1, dtype=torch.complex64, device="cuda:0")
    st = lib.pwa_nll_grad_noalloc(_lib.F32, flat[1:].data_ptr(), 64, A.data_ptr(), 64, None, 0.0, k, 12, 0,
                                  Vd.data_ptr(), out.data_ptr(), None)
    assert st == _lib.E_INVAL
    # no data rows (Eq. 2 form): NLL 0, gradient 0
    out.fill_(5.0)
    pwa.nll_grad_noalloc(A[:0], A, Vd, out, k=k)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 0.0)
