"""GPU parity of the batched (many-V) matrix-core path against the FP64 oracle.

Split 2: FP16 two-term forward, BF16 two-term adjoint on v_mfma_f32_16x16x32,
FP32 accumulation.  Its error is stated, not bounded by 1e-6 for every vector:
the coherent sum z carries an absolute error of about 2^-21 sum_a |V_a A_a|
(22-bit operands, FP32 accumulation), so an event whose |z| is far below that
sum has a large relative error in z/I, and when such an event dominates a
small sample's gradient the gradient error grows.  Stated bound (the shapes
below, small samples of 10^3-10^4 data events): NLL below 2e-7 for every
vector; gradient median below 1e-6, 95th percentile below 1e-4, maximum below
1e-3.  At the batched workload's full size (2e6 data events) the sampled
vectors meet 1e-6.

Split 3 is split 2 plus an exact treatment of those events: a data event
whose coherent sum is small against the bound |z| <= |V| |A_i| (|z| < c |V|
|A_i|, c^2 = min(1/64, sqrt(K)/N_D)) is left out of the matrix-core sums, flagged,
and recomputed in FP64 by a second kernel; it meets 1e-6 for every vector.  Split 0 (one exact streaming
pass per vector) meets 1e-6 everywhere and is tested here too.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.tolerance import errors, reference, reference_fast

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pwa():
    import paper_1108_5882_amd as p
    return p


STATED = dict(nll_max=2e-7, grad_median=1e-6, grad_p95=1e-4, grad_max=1e-3)


def _check_stated(Ad, Am, Vs, nll, grad, w=None, n_gen=None, extended=False, label=""):
    """Split 2 against its stated error distribution."""
    en, eg = [], []
    for b in range(Vs.shape[0]):
        e_n, e_g = errors(reference(Ad, Am, Vs[b], w=w, n_gen=n_gen, extended=extended), nll[b], grad[b])
        en.append(e_n)
        eg.append(e_g)
    en, eg = np.array(en), np.array(eg)
    _say(f"  {label} e_nll max {en.max():.2e}; e_grad median {np.median(eg):.2e} "
         f"p95 {np.percentile(eg, 95):.2e} max {eg.max():.2e} (>1e-6: {int((eg >= 1e-6).sum())}/{len(eg)})")
    assert en.max() < STATED["nll_max"], label
    assert np.median(eg) < STATED["grad_median"], label
    assert np.percentile(eg, 95) < STATED["grad_p95"], label
    assert eg.max() < STATED["grad_max"], label


def _check(Ad, Am, Vs, nll, grad, w=None, n_gen=None, extended=False, tol=1e-6, label=""):
    en, eg = [], []
    for b in range(Vs.shape[0]):
        ref = reference(Ad, Am, Vs[b], w=w, n_gen=n_gen, extended=extended)
        e_n, e_g = errors(ref, nll[b], grad[b])
        en.append(e_n)
        eg.append(e_g)
    en, eg = np.array(en), np.array(eg)
    _say(f"  {label} e_nll max {en.max():.2e} median {np.median(en):.2e}; e_grad max {eg.max():.2e} "
         f"median {np.median(eg):.2e}; over tol {int((en >= tol).sum())}/{int((eg >= tol).sum())}"
         f" of {len(en)} worst V {int(eg.argmax())}")
    assert en.max() < tol and eg.max() < tol, label


CONFIG_LIKE = [(16, 40, 5003, 20011), (32, 33, 4097, 9001), (4, 7, 3000, 9000), (5, 17, 2000, 8000),
               (48, 20, 3001, 6007), (64, 9, 2500, 5000), (1, 3, 1000, 3000), (33, 65, 4096, 8192)]


@pytest.mark.parametrize("k,nv,nd,nm", CONFIG_LIKE)
def test_batch_config_like(pwa, k, nv, nd, nm):
    """Breit-Wigner x Y_J^0 amplitudes (data drawn from the model), V from the V law.
    Split 2 against its stated error; split 3 (flagged small coherent sums recomputed
    exactly) at 1e-6 for every vector."""
    _say(f"case batch k={k} nv={nv} nd={nd} nm={nm}")
    s = synth.make_sample(2, n_data=nd, n_mc=nm, k=k, seed=k)
    Vs = synth.eval_vectors(2, nv, k, seed=k)
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        for extended in (False, True):
            c.set_mc_mode("stream", extended)
            nll, grad = c.nll_batch(Vs, split=2)
            _check_stated(s.A_data, s.A_mc, Vs, nll, grad, extended=extended, label=f"extended={extended}")
            nll3, grad3 = c.nll_batch(Vs, split=3)
            _check(s.A_data, s.A_mc, Vs, nll3, grad3, extended=extended, label=f"split 3 extended={extended}")


def test_batch_weighted_gram_and_vs_single(pwa):
    s = synth.make_sample(2, n_data=20000, n_mc=60000, k=32, weighted=True, accept_fraction=0.8)
    Vs = synth.eval_vectors(2, 64, 32, stream=3)
    _say("case batch weighted/gram")
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc, w=s.w_mc, n_gen=s.n_gen)
        nll, grad = c.nll_batch(Vs, split=2)
        _check_stated(s.A_data, s.A_mc, Vs, nll, grad, w=s.w_mc, n_gen=s.n_gen, label="weighted stream")
        n0, g0 = c.nll_batch(Vs[:4], split=0)
        _check(s.A_data, s.A_mc, Vs[:4], n0, g0, w=s.w_mc, n_gen=s.n_gen, label="split 0")
        c.set_mc_mode("gram")
        nll, grad = c.nll_batch(Vs, split=2)
        _check_stated(s.A_data, s.A_mc, Vs, nll, grad, w=s.w_mc, n_gen=s.n_gen, label="weighted gram")
        nll3, grad3 = c.nll_batch(Vs, split=3)
        nll3b, grad3b = c.nll_batch(Vs, split=3)
        assert np.array_equal(nll3, nll3b) and np.array_equal(grad3, grad3b)      # deterministic
        _check(s.A_data, s.A_mc, Vs, nll3, grad3, w=s.w_mc, n_gen=s.n_gen, label="split 3 weighted gram")


def test_batch_256_vectors_reduced(pwa):
    """K = 32, 256 vectors (all checked), 2% of the batched workload's rows."""
    s = synth.make_sample(2, scale=0.02)
    Vs = synth.eval_vectors(2, 256, s.k)
    _say("case batch 256 V reduced")
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        nll, grad = c.nll_batch(Vs, split=2)
        nll2, grad2 = c.nll_batch(Vs, split=2)
    assert np.array_equal(nll, nll2) and np.array_equal(grad, grad2)      # deterministic
    _check_stated(s.A_data, s.A_mc, Vs, nll, grad, label="256 V")


@pytest.mark.timeout(900)
def test_batch_full_size_every_vector(pwa):
    """K = 32, 2e6 data + 1e7 MC, 256 vectors in one call, in the launch
    configuration the bench times.  Split 3: every vector against the FP64
    oracle at 1e-6 (the long FP32 accumulations of the full-size blocks
    included); split 2: three vectors against its stated bound."""
    import time
    s = synth.make_sample(2)
    Vs = synth.eval_vectors(2, 256, s.k)
    _say("case batch full size, every vector")
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        nll3, grad3 = c.nll_batch(Vs, split=3)
        nll2, grad2 = c.nll_batch(Vs[:3], split=2)
    Ad = s.A_data.astype(np.complex128)
    Am = s.A_mc.astype(np.complex128)
    del s
    t0 = time.perf_counter()
    en, eg = np.zeros(256), np.zeros(256)
    for b in range(256):
        en[b], eg[b] = errors(reference_fast(Ad, Am, Vs[b]), nll3[b], grad3[b])
        if b % 32 == 31:
            _say(f"  oracle checked {b + 1}/256 vectors ({time.perf_counter() - t0:.0f} s)")
    _say(f"  split 3, 256 vectors: e_nll worst {en.max():.2e} p99 {np.percentile(en, 99):.2e}; "
         f"e_grad worst {eg.max():.2e} p99 {np.percentile(eg, 99):.2e}")
    assert en.max() < 1e-6 and eg.max() < 1e-6
    for b in range(3):
        e_n, e_g = errors(reference_fast(Ad, Am, Vs[b]), nll2[b], grad2[b])
        _say(f"  split 2 V{b}: e_nll={e_n:.2e} e_grad={e_g:.2e}")
        assert e_n < STATED["nll_max"] and e_g < STATED["grad_max"]


def test_batch_many_vectors_split3(pwa):
    """2050 vectors (65 vector groups, the last one ragged) in one split-3 pass:
    flag words and recomputation across many groups, 1e-6 for every vector."""
    k, nv = 16, 2050
    s = synth.make_sample(2, n_data=1501, n_mc=4507, k=k, seed=61)
    Vs = synth.eval_vectors(2, nv, k, seed=61)
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        nll, grad = c.nll_batch(Vs, split=3)
    _check(s.A_data, s.A_mc, Vs, nll, grad, label=f"split 3, {nv} vectors")


def test_batch_edge_cases(pwa):
    s = synth.make_sample(2, n_data=500, n_mc=1500, k=8)
    Vs = synth.eval_vectors(2, 3, 8)
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        # a zero vector among valid ones: domain error for it, the others still computed
        V2 = Vs.copy()
        V2[1] = 0
        with pytest.raises(pwa.DomainError):
            c.nll_batch(V2, split=2)
        # empty data in the Eq. 2 form
        c.set_amplitudes("data", s.A_data[:0])
        nll, grad = c.nll_batch(Vs, split=2)
        assert np.all(nll == 0) and np.all(grad == 0)
        c.set_amplitudes("data", s.A_data)
        with pytest.raises(pwa.PwaError) as ei:
            c.nll_batch(Vs, split=4)
        assert ei.value.status == 6
        # split 3: a zero vector among valid ones, empty data
        with pytest.raises(pwa.DomainError):
            c.nll_batch(V2, split=3)
        c.set_amplitudes("data", s.A_data[:0])
        nll, grad = c.nll_batch(Vs, split=3)
        assert np.all(nll == 0) and np.all(grad == 0)
        c.set_amplitudes("data", s.A_data)
        assert c.nll_batch(Vs[:0], split=2)[0].shape == (0,)
    with pwa.Context(0, "f64") as c:
        c.set_amplitudes("data", s.A_data.astype(np.complex128))
        c.set_amplitudes("mc", s.A_mc.astype(np.complex128))
        for split in (2, 3):
            with pytest.raises(pwa.PwaError) as ei:
                c.nll_batch(Vs, split=split)
            assert ei.value.status == 6
        nll, grad = c.nll_batch(Vs, split=0)
        _check(s.A_data, s.A_mc, Vs, nll, grad, tol=1e-12, label="f64 split 0")


def test_batch_fit_descends_to_the_minimum(pwa):
    """Device multi-start L-BFGS on the matrix-core pass with exact recomputation
    of small coherent sums (split 3; one graph per iteration).

    Every start ends below its starting NLL; the reported NLL is the split-3
    value at the returned V (oracle within 1e-6 of the term scale); the best
    start reaches the minimum of an FP64 fit on the oracle (SciPy L-BFGS-B)
    within 1e-6 of the term scale.
    """
    import scipy.optimize as so
    k, nv = 8, 48
    s = synth.make_sample(2, n_data=4000, n_mc=16000, k=k, seed=5)
    V0 = synth.eval_vectors(2, nv, k, seed=6)
    _say("case batch_fit k=8 nv=48 iters=150")
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        V, nll, st, ms = c.batch_fit(V0, 150)
        # zero iterations: the starts come back unevaluated
        Vz, nz, sz, _ = c.batch_fit(V0[:3], 0)
        # one iteration: the starts, evaluated by the split-3 pass
        V1, n1, _, _ = c.batch_fit(V0[:5], 1)
        nb, _ = c.nll_batch(V0[:5], split=3)
    assert np.array_equal(Vz, V0[:3]) and np.all(np.isnan(nz)) and np.all(sz == 0)
    assert np.array_equal(V1, V0[:5]) and np.allclose(n1, nb, rtol=0, atol=1e-9 * np.abs(nb).max())
    assert set(np.unique(st)) <= {0, 1, 2}
    _say(f"  {ms:.3f} ms / iteration; status counts {np.bincount(st, minlength=3)}")
    f0 = np.array([oracle.nll_grad(s.A_data, s.A_mc, V0[b])[0] for b in range(nv)])
    f = np.array([oracle.nll_grad(s.A_data, s.A_mc, V[b])[0] for b in range(nv)])
    assert np.all(f < f0)
    for b in range(nv):
        e_n, _ = errors(reference(s.A_data, s.A_mc, V[b]), nll[b], np.zeros(2 * k))
        assert e_n < 1e-6, b
    best = int(np.argmin(f))

    def fun(x):
        v = x[0::2] + 1j * x[1::2]
        val, g = oracle.nll_grad(s.A_data, s.A_mc, v)
        return val, g
    x0 = np.empty(2 * k)
    x0[0::2], x0[1::2] = V[best].real, V[best].imag
    res = so.minimize(fun, x0, jac=True, method="L-BFGS-B", options=dict(maxiter=500, ftol=1e-15, gtol=1e-10))
    scale = reference(s.A_data, s.A_mc, V[best])["s_nll"]
    _say(f"  best start NLL {f[best]:.6f}, FP64 minimum {res.fun:.6f}, gap {(f[best] - res.fun) / scale:.2e} scaled")
    assert (f[best] - res.fun) / scale < 1e-6


def test_batch_fit_polar(pwa):
    """The batched minimiser in polar parameters (|V_a| >= rmin, periodic phases,
    arg V_0 = 0): it follows the FP64 reference L-BFGS in the same parameters
    for the first iterations, and its best start reaches the Cartesian FP64
    minimum within 1e-5 of the term scale; every returned V has V_0 real."""
    import scipy.optimize as so

    from oracle.lbfgs import LbfgsOracle
    k, nv = 8, 32
    s = synth.make_sample(2, n_data=4000, n_mc=16000, k=k, seed=5)
    V0 = synth.eval_vectors(2, nv, k, seed=8)
    _say("case batch_fit polar k=8 nv=32")
    T = 10
    with pwa.Context(0, "f32") as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        VT, fT, _, _ = c.batch_fit(V0, T, polar=True)
        V, nll, st, ms = c.batch_fit(V0, 300, polar=True)
        # a bound above every start magnitude: every returned magnitude respects it
        rmin = 1.01 * float(np.max(np.abs(V0)))
        Vb, _, _, _ = c.batch_fit(V0[:4], 40, polar=True, rmin=rmin)
    assert np.all(np.abs(Vb) >= rmin * (1 - 1e-12))
    assert np.all(V[:, 0].imag == 0.0) and np.all(V[:, 0].real >= 0.0)

    def fun(x):
        return oracle.nll_grad(s.A_data, s.A_mc, x[0::2] + 1j * x[1::2])
    for b in range(3):
        v0 = V0[b]
        ph0 = math.atan2(v0[0].imag, v0[0].real)
        p0 = np.empty(2 * k)
        p0[0::2] = np.abs(v0)
        p0[1::2] = [0.0] + [math.remainder(math.atan2(z.imag, z.real) - ph0, 2 * math.pi) for z in v0[1:]]
        ref = LbfgsOracle(fun, p0, polar=True)
        for _ in range(T):
            ref.step()
        Vr = ref.x[0::2] * np.exp(1j * ref.x[1::2])
        scale = reference(s.A_data, s.A_mc, Vr)["s_nll"]
        _say(f"  start {b}: after {T} steps f gpu {fT[b]:.10g} ref {ref.f:.10g} "
             f"dV {np.max(np.abs(VT[b] - Vr)) / np.max(np.abs(Vr)):.2e}")
        assert abs(fT[b] - ref.f) < 1e-6 * scale
        assert np.max(np.abs(VT[b] - Vr)) < 1e-4 * np.max(np.abs(Vr))
    f = np.array([oracle.nll_grad(s.A_data, s.A_mc, V[b])[0] for b in range(nv)])
    best = int(np.argmin(f))
    x0 = np.empty(2 * k)
    x0[0::2], x0[1::2] = V[best].real, V[best].imag
    res = so.minimize(fun, x0, jac=True, method="L-BFGS-B", options=dict(maxiter=500, ftol=1e-15, gtol=1e-10))
    scale = reference(s.A_data, s.A_mc, V[best])["s_nll"]
    _say(f"  polar: {ms:.3f} ms / iteration; status {np.bincount(st, minlength=3)}; best {f[best]:.6f}, "
         f"FP64 minimum {res.fun:.6f}, gap {(f[best] - res.fun) / scale:.2e} scaled")
    assert (f[best] - res.fun) / scale < 1e-5
