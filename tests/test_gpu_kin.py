"""GPU parity of the kinematic path (amplitudes formed on the device from (m,
cos theta), floating masses and widths) against the FP64 kinematic oracle.

The kernel's arithmetic after the FP32 kinematics is FP64, so the bar here is
1e-10 of the term scale (tighter than the 1e-6 of FP32 contexts): the NLL
scale is sum |ln I| + N_D |ln S|, the V-gradient scale max|2 G| + max|2 c H|,
the resonance-gradient scale max|R_data| + max|c R_MC| (data and MC terms
taken separately, as in tests/tolerance.py).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pwa():
    import paper_1108_5882_amd as p
    return p


def _errors(s_or_mx, mx_mc, V, res, spins, w, n_gen, extended, got):
    nll, gv, gr, P = oracle.kin_nll_grad(s_or_mx, mx_mc, V, res, spins, w=w, n_gen=n_gen, extended=extended,
                                         parts=True)
    nd = s_or_mx.shape[0]
    ng = float(n_gen) if n_gen else float(mx_mc.shape[0])
    S = P["s_raw"] / ng
    if nd:
        A = oracle.kin_amplitudes(s_or_mx, spins, res)
        I = np.abs(A @ np.asarray(V, dtype=complex)) ** 2
        s_nll = float(np.sum(np.abs(np.log(I)))) + (abs(S) if extended else nd * abs(np.log(S)))
    else:
        s_nll = abs(S) if extended else 1.0
    c = 1.0 / ng if extended else (nd / P["s_raw"] if nd else 0.0)
    s_gv = np.max(np.abs(2 * P["GD"])) + np.max(np.abs(2 * c * P["HM"]))
    s_gr = np.max(np.abs(P["RD"])) + np.max(np.abs(c * P["RM"]))
    gn, ggv, ggr = got
    return (abs(gn - nll) / max(s_nll, 1e-300), np.max(np.abs(ggv - gv)) / max(s_gv, 1e-300),
            np.max(np.abs(ggr - gr)) / max(s_gr, 1e-300))


def _random_case(seed, k, nd, nm, weighted):
    g = np.random.default_rng(seed)
    mx_d = np.stack([g.uniform(0.99, 3.0, nd), g.uniform(-1, 1, nd)], 1).astype(np.float32)
    mx_m = np.stack([g.uniform(0.99, 3.0, nm), g.uniform(-1, 1, nm)], 1).astype(np.float32)
    w = g.uniform(0.3, 2.0, nm).astype(np.float32) if weighted else None
    spins = g.integers(0, 5, k).astype(np.int32)
    res = np.empty(2 * k)
    res[0::2] = g.uniform(1.2, 2.8, k)
    res[1::2] = g.uniform(0.03, 0.3, k)
    V = synth.draw_v(g, 1, k)[0]
    return mx_d, mx_m, w, spins, res, V


@pytest.mark.parametrize("k,nd,nm", [(1, 1001, 3001), (3, 777, 2049), (4, 4096, 8192), (5, 3001, 7003),
                                     (8, 2048, 5000), (16, 10007, 30011), (17, 999, 4001), (33, 1500, 4500),
                                     (64, 701, 2101)])
def test_random_shapes(pwa, k, nd, nm):
    weighted = k % 2 == 1
    _say(f"case kin random k={k} nd={nd} nm={nm} weighted={weighted}")
    mx_d, mx_m, w, spins, res, V = _random_case(300 + k, k, nd, nm, weighted)
    with pwa.KinContext(spins) as c:
        c.set_events("data", mx_d)
        c.set_events("mc", mx_m, w=w, n_gen=nm + 13)
        for ext in (False, True):
            c.set_mode(ext)
            got = c.nll_grad(V, res)
            e = _errors(mx_d, mx_m, V, res, spins, w, nm + 13, ext, got)
            _say(f"  extended={ext} e_nll={e[0]:.2e} e_grad_v={e[1]:.2e} e_grad_res={e[2]:.2e}")
            assert max(e) < TOL
            again = c.nll_grad(V, res)
            assert again[0] == got[0] and np.array_equal(again[1], got[1]) and np.array_equal(again[2], got[2])


def test_workload_k16_full_size(pwa):
    """The single-V workload's kinematics (K = 16, 1e6 data + 5e6 MC events), at
    the generating resonance parameters and at shifted ones."""
    s = synth.make_kin_sample(1)
    V = synth.eval_vectors(1, 1, s.k)[0]
    _say(f"case kin full size: {s.mx_data.shape[0]} data + {s.mx_mc.shape[0]} MC events, K={s.k}")
    shifted = s.res * (1.0 + 0.02 * np.sin(np.arange(2 * s.k)))
    with pwa.KinContext(s.waves.J) as c:
        c.set_events("data", s.mx_data)
        c.set_events("mc", s.mx_mc)
        for res in (s.res, shifted):
            got = c.nll_grad(V, res)
            e = _errors(s.mx_data, s.mx_mc, V, res, s.waves.J, None, None, False, got)
            _say(f"  e_nll={e[0]:.2e} e_grad_v={e[1]:.2e} e_grad_res={e[2]:.2e}")
            assert max(e) < TOL


def test_matches_precomputed_amplitude_path(pwa):
    """With masses and widths fixed, the kinematic path and the precomputed-amplitude
    path (FP64 context fed with the oracle's amplitude rows) give the same NLL and V
    gradient."""
    s = synth.make_kin_sample(1, scale=0.01, weighted=True)
    V = synth.eval_vectors(1, 1, s.k, stream=2)[0]
    Ad = oracle.kin_amplitudes(s.mx_data, s.waves.J, s.res)
    Am = oracle.kin_amplitudes(s.mx_mc, s.waves.J, s.res)
    _say("case kin vs precomputed")
    with pwa.KinContext(s.waves.J) as kc, pwa.Context(0, "f64") as c:
        kc.set_events("data", s.mx_data)
        kc.set_events("mc", s.mx_mc, w=s.w_mc)
        c.set_amplitudes("data", Ad)
        c.set_amplitudes("mc", Am, w=s.w_mc.astype(np.float64))
        n1, g1, _ = kc.nll_grad(V, s.res)
        n2, g2 = c.nll_grad(V)
    assert abs(n1 - n2) < 1e-11 * abs(n2)
    assert np.max(np.abs(g1 - g2)) < 1e-10 * np.max(np.abs(g2))


def test_async_borrow_and_edge_cases(pwa):
    import torch
    mx_d, mx_m, w, spins, res, V = _random_case(7, 12, 5000, 15000, True)
    v = np.empty(24)
    v[0::2], v[1::2] = V.real, V.imag
    with pwa.KinContext(spins) as c:
        td = torch.from_numpy(mx_d).cuda()
        tm = torch.from_numpy(mx_m).cuda()
        tw = torch.from_numpy(w).cuda()
        c.set_events("data", td, borrow=True)
        c.set_events("mc", tm, w=tw, borrow=True)
        ref = c.nll_grad(V, res)
        out = torch.zeros(4 * 12 + 2, dtype=torch.float64, device="cuda:0")
        c.nll_grad_async(torch.from_numpy(v).cuda(), torch.from_numpy(res).cuda(), out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert o[0] == ref[0] and np.array_equal(o[1:25], ref[1]) and np.array_equal(o[25:49], ref[2]) and o[49] == 0
        # copied events give the same bits as borrowed ones
        c.set_events("data", mx_d)
        c.set_events("mc", mx_m, w=w)
        cp = c.nll_grad(V, res)
        assert cp[0] == ref[0] and np.array_equal(cp[1], ref[1]) and np.array_equal(cp[2], ref[2])
        # a non-positive width is refused on the host; a zero vector is a domain failure
        bad = res.copy()
        bad[3] = 0.0
        with pytest.raises(pwa.PwaError):
            c.nll_grad(V, bad)
        with pytest.raises(pwa.DomainError):
            c.nll_grad(np.zeros(12, dtype=complex), res)
        # no data events: NLL 0 and zero gradients (Eq. 2 form)
        c.set_events("data", mx_d[:0])
        n0, gv0, gr0 = c.nll_grad(V, res)
        assert n0 == 0.0 and not gv0.any() and not gr0.any()
        # the context recovers
        c.set_events("data", mx_d)
        again = c.nll_grad(V, res)
        assert again[0] == ref[0]
