"""GPU parity of the NLL Hessian (pwa_hessian) against the FP64 oracle.

Error measure, like the gradient's: max |dH| over the scale of the terms,
  scale = 2 max_ac sum_i |A_ia A_ic| / I_i  (the data sum before cancellation)
        + max |H_MC|                         (the normalisation term),
with 1e-6 for FP32 contexts and 1e-12 for FP64 contexts.  The GPU output is
also checked against the exact identity H x = -g of the Eq. 2 form (g from
the library's own gradient)."""
import sys

import numpy as np
import pytest

import oracle.hessian as OH
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _scale(Ad, V, h_mc):
    Ad = Ad.astype(np.complex128)
    I = np.abs(Ad @ V.astype(np.complex128)) ** 2
    absA = np.abs(Ad)
    s_data = 2 * np.max(np.einsum("ia,ic,i->ac", absA, absA, 1.0 / I)) if Ad.shape[0] else 0.0
    return s_data + np.max(np.abs(h_mc))


CASES = [(16, 5003, 20011, "f32"), (4, 3000, 9000, "f32"), (33, 2049, 6007, "f32"), (1, 1000, 3000, "f32"),
         (48, 1500, 4000, "f32"), (64, 1201, 3000, "f32"), (16, 3001, 9007, "f64"), (5, 2000, 6000, "f64"),
         (64, 800, 2000, "f64"), (16, 200003, 30011, "f32"), (48, 60001, 20011, "f32"), (56, 1001, 3001, "f32"),
         (9, 2003, 5003, "f32")]


@pytest.mark.parametrize("k,nd,nm,prec", CASES)
def test_hessian_matches_oracle(k, nd, nm, prec):
    import paper_1108_5882_amd as pwa
    s = synth.make_sample(2, n_data=nd, n_mc=nm, k=k, seed=k + 40)
    Vs = synth.eval_vectors(2, 3, k, seed=k + 40)
    w = np.linspace(0.25, 1.75, nm)
    tol = 1e-6 if prec == "f32" else 1e-12
    Ad = s.A_data if prec == "f32" else s.A_data.astype(np.complex128)
    Am = s.A_mc if prec == "f32" else s.A_mc.astype(np.complex128)
    with pwa.Context(0, prec) as c:
        c.set_amplitudes("data", Ad)
        c.set_amplitudes("mc", Am, w=w.astype(np.float32 if prec == "f32" else np.float64), n_gen=1.5 * nm)
        wq = w.astype(np.float32).astype(np.float64) if prec == "f32" else w
        for extended in (False, True):
            c.set_mc_mode("stream", extended)
            for b in range(Vs.shape[0]):
                H = c.hessian(Vs[b])
                ref, _, h_mc = OH.hessian(Ad, Am, Vs[b], w=wq, n_gen=1.5 * nm, extended=extended, parts=True)
                e = np.max(np.abs(H - ref)) / _scale(Ad, Vs[b], h_mc)
                _say(f"  k={k} {prec} ext={extended} V{b}: e_H {e:.2e}")
                assert e < tol, (k, prec, extended, b, e)
                assert np.array_equal(H, H.T) or np.max(np.abs(H - H.T)) <= tol * np.max(np.abs(H))


def test_hessian_identities_and_edges():
    import paper_1108_5882_amd as pwa
    k = 16
    s = synth.make_sample(1, n_data=20000, n_mc=60000, k=k, seed=5)
    V = synth.eval_vectors(1, 1, k, seed=5)[0]
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        H = c.hessian(V)
        _, g = c.nll_grad(V)
        x = np.empty(2 * k)
        x[0::2], x[1::2] = V.real, V.imag
        r = np.max(np.abs(H @ x + g)) / (np.max(np.abs(H)) * np.max(np.abs(x)))
        _say(f"  H x + g: {r:.2e}")
        assert r < 1e-6
        # the Gram mode gives the same matrix (the normalisation term always comes from M)
        c.set_mc_mode("gram", False)
        assert np.array_equal(c.hessian(V), H)
        c.set_mc_mode("stream", False)
        # V = 0: every coherent sum vanishes
        with pytest.raises(pwa.DomainError):
            c.hessian(np.zeros(k, dtype=np.complex64))
        # no data events, Eq. 2 form: H = 0
        c.set_amplitudes("data", s.A_data[:0])
        assert np.all(c.hessian(V) == 0)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_hessian_nonfinite_rows(bad):
    """A non-finite amplitude in one data row gives PWA_E_DOMAIN wherever the row
    falls (first and last rows, rows that a neighbouring block's last step reads
    past its range), and the context then gives the unchanged result on clean
    rows.  1e5 rows spread over more blocks than one step's 64 rows each."""
    import paper_1108_5882_amd as pwa
    k, nd = 16, 100000
    s = synth.make_sample(1, n_data=nd, n_mc=30000, k=k, seed=8)
    V = synth.eval_vectors(1, 1, k, seed=8)[0]
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        H0 = c.hessian(V)
        for row in (0, 97, 98, 100, 50001, nd - 1):
            _say(f"  non-finite ({bad}) in data row {row}")
            A = s.A_data.copy()
            A[row, 3] = complex(bad, 0.0)
            c.set_amplitudes("data", A)
            with pytest.raises(pwa.DomainError):
                c.hessian(V)
        c.set_amplitudes("data", s.A_data)
        assert np.array_equal(c.hessian(V), H0)
