"""Samples the library reads in place (PWA_BORROW), device-pointer checks, and
non-finite amplitudes.

A borrowed sample must give bitwise the results of the same sample copied into
the library's layout (same kernels, same launch configuration), must not cost
sample memory, and must be refused when it does not have the device layout.
Non-finite amplitudes give PWA_E_DOMAIN and NLL = +inf, and the context stays
usable.
"""
import ctypes
import sys

import numpy as np
import pytest

import synth
from tests.tolerance import TOL, errors, reference

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pwa():
    import paper_1108_5882_amd as p
    return p


def _padded(torch, A, ld):
    """A [n, k] complex numpy -> GPU tensor [n, ld] with zero columns k..ld-1."""
    n, k = A.shape
    t = torch.zeros((n, ld), dtype=torch.complex64 if A.dtype == np.complex64 else torch.complex128,
                    device="cuda:0")
    t[:, :k] = torch.from_numpy(A).cuda()
    return t


@pytest.mark.parametrize("prec,k", [("f32", 16), ("f32", 10), ("f64", 7), ("f32", 32)])
def test_borrow_matches_copy_bitwise(pwa, prec, k):
    import torch
    _say(f"case borrow prec={prec} k={k}")
    g = np.random.default_rng(500 + k)
    dt = np.complex64 if prec == "f32" else np.complex128
    nd, nm = 20011, 70001
    Ad = synth.random_amplitudes(g, nd, k, dt)
    Am = synth.random_amplitudes(g, nm, k, dt)
    w = g.uniform(0.5, 2.0, nm).astype(np.float32 if prec == "f32" else np.float64)
    V = synth.draw_v(g, 1, k)[0]
    Vs = synth.draw_v(g, 8, k)
    with pwa.Context(0, prec) as c1, pwa.Context(0, prec) as c2:
        ld = c1.layout_ld(k)
        c1.set_amplitudes("data", Ad)
        c1.set_amplitudes("mc", Am, w=w, n_gen=nm + 3)
        td, tm = _padded(torch, Ad, ld), _padded(torch, Am, ld)
        tw = torch.from_numpy(w).cuda()
        c2.set_amplitudes("data", td, borrow=True, k=k)
        c2.set_amplitudes("mc", tm, w=tw, n_gen=nm + 3, borrow=True, k=k)
        c2.set_stream_cfg(**c1.stream_cfg())
        for mode in ("stream", "gram"):
            for ext in (False, True):
                c1.set_mc_mode(mode, ext)
                c2.set_mc_mode(mode, ext)
                r1, r2 = c1.nll_grad(V), c2.nll_grad(V)
                _say(f"  mode={mode} extended={ext} nll={r1[0]:.12g}")
                assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1])
        c1.set_mc_mode("stream")
        c2.set_mc_mode("stream")
        ref = reference(Ad, Am, V, w=w, n_gen=nm + 3)
        e_n, e_g = errors(ref, *c2.nll_grad(V))
        _say(f"  borrowed vs oracle e_nll={e_n:.2e} e_grad={e_g:.2e}")
        assert e_n < TOL[prec] and e_g < TOL[prec]
        if prec == "f32":
            for split in (2, 3):
                b1, b2 = c1.nll_batch(Vs, split=split), c2.nll_batch(Vs, split=split)
                assert np.array_equal(b1[0], b2[0]) and np.array_equal(b1[1], b2[1])
        # the library keeps the borrowed tensors alive and reads them in place
        assert c2._borrowed["data"][0] is td and c2._borrowed["mc"][1] is tw
        torch.cuda.synchronize()


def test_borrow_allocates_no_sample_memory(pwa):
    import torch
    k, nd, nm = 16, 1 << 20, 1 << 22          # 128 MB + 512 MB of FP32 rows
    _say(f"case borrow memory k={k} nd={nd} nm={nm}")
    td = torch.randn((nd, k), dtype=torch.complex64, device="cuda:0")
    tm = torch.randn((nm, k), dtype=torch.complex64, device="cuda:0")
    torch.cuda.synchronize()
    sample_bytes = (nd + nm) * k * 8
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", td[:8].cpu().numpy())   # fix k, allocate the context's own buffers
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        c.set_amplitudes("data", td, borrow=True)
        c.set_amplitudes("mc", tm, borrow=True)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        _say(f"  borrow: free memory change {free0 - free1} bytes (sample {sample_bytes})")
        assert free0 - free1 < sample_bytes // 64
        nll_b, g_b = c.nll_grad(np.ones(k, dtype=np.complex128))
        c.set_amplitudes("data", td)
        c.set_amplitudes("mc", tm)
        torch.cuda.synchronize()
        free2 = torch.cuda.mem_get_info()[0]
        _say(f"  copy: free memory change {free0 - free2} bytes")
        assert free0 - free2 >= 0.99 * sample_bytes
        nll_c, g_c = c.nll_grad(np.ones(k, dtype=np.complex128))
        assert nll_b == nll_c and np.array_equal(g_b, g_c)


def test_borrow_rejects_bad_layouts(pwa):
    import torch
    from paper_1108_5882_amd import _lib
    _say("case borrow rejections")
    g = np.random.default_rng(3)
    k, n = 10, 4096
    A = synth.random_amplitudes(g, n, k)
    with pwa.Context(0, "f32") as c:
        ld = c.layout_ld(k)
        assert ld == 12
        good = _padded(torch, A, ld)
        lib, h = c.lib, c.h
        # row stride other than the device layout
        st = lib.pwa_set_amplitudes(h, _lib.DATA, ctypes.c_void_p(good.data_ptr()), n, k, 11, _lib.BORROW, None, 0.0)
        assert st == _lib.E_INVAL
        # base not 16-byte aligned (one complex in)
        flat = torch.zeros(n * ld + 1, dtype=torch.complex64, device="cuda:0")
        st = lib.pwa_set_amplitudes(h, _lib.DATA, ctypes.c_void_p(flat[1:].data_ptr()), n, k, ld, _lib.BORROW,
                                    None, 0.0)
        assert st == _lib.E_INVAL
        # nonzero padding in one row
        bad = good.clone()
        bad[n - 1, k + 1] = 1e-30
        with pytest.raises(_lib.PwaError) as ei:
            c.set_amplitudes("data", bad, borrow=True, k=k)
        assert ei.value.status == _lib.E_INVAL and "zeros" in ei.value.message
        # host memory passed as device memory (copy and borrow)
        Ah = np.zeros((n, ld), dtype=np.complex64)
        for where in (_lib.DEVICE, _lib.BORROW):
            st = lib.pwa_set_amplitudes(h, _lib.DATA, ctypes.c_void_p(Ah.ctypes.data), n, k, ld, where, None, 0.0)
            assert st == _lib.E_INVAL
        # the context still works after the refusals
        c.set_amplitudes("data", good, borrow=True, k=k)
        c.set_amplitudes("mc", _padded(torch, synth.random_amplitudes(g, 3 * n, k), ld), borrow=True, k=k)
        V = synth.draw_v(g, 1, k)[0]
        nll, grad = c.nll_grad(V)
        ref = reference(A, c._borrowed["mc"][0][:, :k].cpu().numpy(), V)
        e_n, e_g = errors(ref, nll, grad)
        assert e_n < TOL["f32"] and e_g < TOL["f32"]
        # async entry points refuse host pointers
        vh = np.zeros(2 * k)
        oh = np.zeros(2 * k + 2)
        assert lib.pwa_nll_grad_async(h, ctypes.c_void_p(vh.ctypes.data), ctypes.c_void_p(oh.ctypes.data)) \
            == _lib.E_INVAL


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("where,value", [("data", np.nan), ("data", np.inf), ("mc", np.nan), ("mc", -np.inf)])
def test_non_finite_amplitudes(pwa, prec, where, value):
    _say(f"case non-finite prec={prec} sample={where} value={value}")
    g = np.random.default_rng(11)
    dt = np.complex64 if prec == "f32" else np.complex128
    k, nd, nm = 12, 5001, 15001
    Ad = synth.random_amplitudes(g, nd, k, dt)
    Am = synth.random_amplitudes(g, nm, k, dt)
    V = synth.draw_v(g, 1, k)[0]
    bad = (Ad if where == "data" else Am).copy()
    bad[bad.shape[0] // 2, 3] = complex(value, 0.0)
    with pwa.Context(0, prec) as c:
        c.set_amplitudes("data", bad if where == "data" else Ad)
        c.set_amplitudes("mc", bad if where == "mc" else Am)
        for mode in ("stream", "gram"):
            c.set_mc_mode(mode)
            with pytest.raises(pwa.DomainError):
                c.nll_grad(V)
            assert c.last_flags() != 0
        # the NLL the failed call wrote is +inf
        from paper_1108_5882_amd import _lib
        v = np.empty(2 * k)
        v[0::2], v[1::2] = V.real, V.imag
        out = np.zeros(1)
        assert c.lib.pwa_nll(c.h, v.ctypes.data, out.ctypes.data) == _lib.E_DOMAIN
        assert out[0] == np.inf
        # replacing the bad sample restores normal evaluations
        c.set_mc_mode("stream")
        c.set_amplitudes(where, Ad if where == "data" else Am)
        nll, grad = c.nll_grad(V)
        e_n, e_g = errors(reference(Ad, Am, V), nll, grad)
        assert e_n < TOL[prec] and e_g < TOL[prec]
