"""Pins of the FP64 oracle: facts fixed by the paper or by mathematics, not by the oracle.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
if the oracle disagrees with the fact.  test_oracle_pins.py runs them on the
oracle; test_oracle_mutants.py runs them on deliberately broken builds of the
oracle to show that each plausible mistake is caught by at least one pin.

Citations are to Berger, "Partial Wave Analysis using Graphics Cards":
Eq. 1 (coherent intensity), Eq. 2 (likelihood with MC normalisation),
Eq. 3 (expanded form), Section 2 (MC footnote, precompute remark).
"""
from __future__ import annotations

import cmath
import json
import math
import os
from fractions import Fraction

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _cplx_rows(rows):
    return np.array([[complex(r, i) for r, i in row] for row in rows], dtype=np.complex128)


def _rel(a, b, scale=None):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    s = scale if scale is not None else max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / s)


def _small_case(seed=1, nd=40, nm=120, k=3, weighted=False):
    g = np.random.default_rng(seed)
    Ad = synth.random_amplitudes(g, nd, k, np.complex128)
    Am = synth.random_amplitudes(g, nm, k, np.complex128)
    V = synth.draw_v(g, 1, k)[0]
    w = g.uniform(0.2, 3.0, nm) if weighted else None
    return Ad, Am, V, w


# ------------------------------------------------------------------ golden
def pin_golden_hand_example(orc):
    """Hand-worked K=2 example (tests/golden/hand_k2.json): Eq. 1, 2, 3 and the Eq. 3 bracket."""
    with open(os.path.join(GOLDEN, "hand_k2.json")) as f:
        gd = json.load(f)
    Ad, Am = _cplx_rows(gd["A_data"]), _cplx_rows(gd["A_mc"])
    V = np.array([complex(r, i) for r, i in gd["V"]])
    ng = gd["n_gen"]
    assert np.array_equal(orc.intensity(Ad, V), np.array(gd["intensity_data"], float))
    assert np.array_equal(orc.intensity(Am, V), np.array(gd["intensity_mc"], float))
    nll, grad = orc.nll_grad(Ad, Am, V, n_gen=ng)
    assert abs(nll - (-math.log(2) + 3 * math.log(1.25))) < 1e-15
    assert _rel(grad, gd["grad"]) < 1e-15
    nll, grad = orc.nll_grad(Ad, Am, V, n_gen=ng, extended=True)
    assert abs(nll - (-math.log(2) + 1.25)) < 1e-15
    assert _rel(grad, gd["grad_ext"]) < 1e-15
    M = orc.gram(Am, n_gen=ng)
    assert np.allclose(M, _cplx_rows(gd["gram"]), rtol=0, atol=1e-15)
    nll_g, grad_g = orc.nll_grad_gram(Ad, M, V)
    assert abs(nll_g - (-math.log(2) + 3 * math.log(1.25))) < 1e-15
    assert _rel(grad_g, gd["grad"]) < 1e-15


# ------------------------------------------------------------- closed forms
def pin_single_wave_closed_form(orc):
    """K=1: I = |V|^2 |A|^2, so NLL = -sum ln|A_i|^2 + N_D ln((1/N_gen) sum w |A_j|^2),
    independent of V, and the gradient vanishes (Eq. 1, 2)."""
    g = np.random.default_rng(7)
    Ad = synth.random_amplitudes(g, 50, 1, np.complex128)
    Am = synth.random_amplitudes(g, 200, 1, np.complex128)
    w = g.uniform(0.5, 2.0, 200)
    ng = 333.0
    expect = (-math.fsum(math.log(abs(a) ** 2) for a in Ad[:, 0])
              + 50 * math.log(math.fsum(wj * abs(a) ** 2 for wj, a in zip(w, Am[:, 0])) / ng))
    for V in (np.array([1.0 + 0j]), np.array([0.3 - 2.2j]), np.array([-7.5 + 0.01j])):
        nll, grad = orc.nll_grad(Ad, Am, V, w=w, n_gen=ng)
        assert abs(nll - expect) < 1e-12 * (abs(expect) + 50)
        assert np.max(np.abs(grad)) < 1e-12 * 50 / abs(V[0])
        # single-event intensities equal |V|^2 |A|^2
        assert _rel(orc.intensity(Ad, V), np.abs(V[0]) ** 2 * np.abs(Ad[:, 0]) ** 2) < 1e-14


def pin_jensen_equal_samples(orc):
    """Data and MC the same rows, w = 1, N_gen = N: NLL = N ln(mean I) - sum ln I >= 0 (Jensen),
    with equality exactly when I is constant over the sample (Eq. 2)."""
    g = np.random.default_rng(11)
    A = synth.random_amplitudes(g, 64, 3, np.complex128)
    V = synth.draw_v(g, 1, 3)[0]
    nll, _ = orc.nll_grad(A, A, V)
    assert nll > 0
    # constant intensity: every row is a phase times the same row
    base = A[0]
    Ac = np.exp(1j * g.uniform(0, 2 * math.pi, 64))[:, None] * base[None, :]
    nll_c, grad_c = orc.nll_grad(Ac, Ac, V)
    assert abs(nll_c) < 1e-12 * 64
    assert np.max(np.abs(grad_c)) < 1e-9


def pin_n_gen_shift(orc):
    """Changing N_gen (generated MC count, acceptance remark of Section 2) shifts the Eq. 2
    NLL by N_D ln(N_gen/N_gen') and leaves the gradient unchanged."""
    Ad, Am, V, w = _small_case(3, weighted=True)
    n1, g1 = orc.nll_grad(Ad, Am, V, w=w, n_gen=120.0)
    n2, g2 = orc.nll_grad(Ad, Am, V, w=w, n_gen=480.0)
    assert abs((n1 - n2) - 40 * math.log(4.0)) < 1e-11
    assert _rel(g1, g2) < 1e-14


def pin_weights(orc):
    """Integer weights are repeated MC rows; N_gen given explicitly (footnote on weighted MC)."""
    Ad, Am, V, _ = _small_case(5, nm=30)
    wi = np.random.default_rng(5).integers(1, 4, 30)
    rep = np.repeat(Am, wi, axis=0)
    n1, g1 = orc.nll_grad(Ad, Am, V, w=wi.astype(float), n_gen=100.0)
    n2, g2 = orc.nll_grad(Ad, rep, V, n_gen=100.0)
    assert abs(n1 - n2) < 1e-12 * (abs(n1) + 40)
    assert _rel(g1, g2) < 1e-12


# --------------------------------------------------------------- invariants
def pin_global_phase(orc):
    """NLL(e^{i phi} V) = NLL(V); complex gradient rotates by e^{i phi} (Eq. 1: I depends on |z|)."""
    Ad, Am, V, w = _small_case(13, weighted=True)
    n0, g0 = orc.nll_grad(Ad, Am, V, w=w)
    c0 = g0[0::2] + 1j * g0[1::2]
    for phi in (0.3, 2.0, -1.1):
        r = cmath.exp(1j * phi)
        n1, g1 = orc.nll_grad(Ad, Am, r * V, w=w)
        assert abs(n1 - n0) < 1e-12 * (abs(n0) + 40)
        c1 = g1[0::2] + 1j * g1[1::2]
        assert np.max(np.abs(c1 - r * c0)) < 1e-11 * np.max(np.abs(c0))
        assert _rel(orc.intensity(Ad, r * V), orc.intensity(Ad, V)) < 1e-14


def pin_scale_invariance(orc):
    """Eq. 2 form: NLL(cV) = NLL(V) for every complex c != 0 (the N_D ln S term
    cancels |c|^2); the complex gradient scales as g(cV) = g(V)/conj(c)."""
    Ad, Am, V, w = _small_case(17, weighted=True)
    n0, g0 = orc.nll_grad(Ad, Am, V, w=w, n_gen=500.0)
    c0 = g0[0::2] + 1j * g0[1::2]
    for c in (3.0, 0.05 - 0.2j, -12 + 5j):
        n1, g1 = orc.nll_grad(Ad, Am, c * V, w=w, n_gen=500.0)
        assert abs(n1 - n0) < 1e-11 * (abs(n0) + 40)
        c1 = g1[0::2] + 1j * g1[1::2]
        assert np.max(np.abs(c1 - c0 / np.conj(c))) < 1e-10 * np.max(np.abs(c0 / np.conj(c)))


def pin_euler_identities(orc):
    """Homogeneity: sum_a conj(V_a) sum_i conj(A_ia) z_i / I_i = N_D exactly, and
    sum_a conj(V_a) sum_j w_j conj(A_ja) z_j = sum_j w_j I_j; hence the full
    Eq. 2 gradient has V^H g = 0 (radial and phase directions are flat)."""
    Ad, Am, V, w = _small_case(19, weighted=True)
    nll, grad, parts = orc.nll_grad(Ad, Am, V, w=w, parts=True)
    GD = parts["GD"][0::2] + 1j * parts["GD"][1::2]
    HM = parts["HM"][0::2] + 1j * parts["HM"][1::2]
    assert abs(np.vdot(V, GD) - 40) < 1e-12 * 40
    assert abs(np.vdot(V, HM) - parts["s_raw"]) < 1e-12 * parts["s_raw"]
    # s_raw is the weighted sum of the Eq. 1 intensities of the MC rows
    s_direct = math.fsum(w * orc.intensity(Am, V))
    assert abs(parts["s_raw"] - s_direct) < 1e-13 * s_direct
    # sum_i ln I_i of the Eq. 1 intensities of the data rows
    sl = math.fsum(np.log(orc.intensity(Ad, V)))
    assert abs(parts["sum_log"] - sl) < 1e-12 * (abs(sl) + 40)
    cg = grad[0::2] + 1j * grad[1::2]
    assert abs(np.vdot(V, cg)) < 1e-11 * np.linalg.norm(V) * np.max(np.abs(cg))


def pin_extended_vs_shape(orc):
    """Eq. 3 (linear S) vs Eq. 2 (N_D ln S): min over lambda > 0 of NLL_ext(sqrt(lambda) V)
    equals NLL(V) + N_D - N_D ln N_D, at lambda = N_D / S(V)."""
    Ad, Am, V, w = _small_case(23, weighted=True)
    ng = 200.0
    nll, _, parts = orc.nll_grad(Ad, Am, V, w=w, n_gen=ng, parts=True)
    S = parts["s_raw"] / ng
    lam = 40 / S
    ne, ge = orc.nll_grad(Ad, Am, math.sqrt(lam) * V, w=w, n_gen=ng, extended=True)
    assert abs(ne - (nll + 40 - 40 * math.log(40))) < 1e-11 * (abs(nll) + 40)
    # stationary along the radial direction at that lambda
    cg = ge[0::2] + 1j * ge[1::2]
    assert abs(np.vdot(V, cg).real) < 1e-10 * np.linalg.norm(V) * np.max(np.abs(cg))
    # and strictly larger away from it
    for f in (0.8, 1.25):
        nf, _ = orc.nll_grad(Ad, Am, math.sqrt(lam * f) * V, w=w, n_gen=ng, extended=True)
        assert nf > ne


def pin_gram_identity(orc):
    """Eq. 3 bracket: M_ab = (1/N_gen) sum_j w_j conj(A_ja) A_jb, Hermitian PSD with
    trace (1/N_gen) sum w |A|^2, and V^H M V equals the streamed MC estimate S;
    per event, the Eq. 3 double sum sum_ab V_a V_b^* A_a A_b^* equals Eq. 1's I."""
    Ad, Am, V, w = _small_case(29, weighted=True)
    ng = 150.0
    M = orc.gram(Am, w=w, n_gen=ng)
    Mref = (Am.conj().T * w) @ Am / ng          # library matmul
    assert np.max(np.abs(M - Mref)) < 1e-13 * np.max(np.abs(Mref))
    assert np.max(np.abs(M - M.conj().T)) < 1e-14 * np.max(np.abs(M))
    assert np.min(np.linalg.eigvalsh(M)) > -1e-12 * np.max(np.abs(M))
    assert abs(np.trace(M).real - math.fsum(w * np.sum(np.abs(Am) ** 2, axis=1)) / ng) < 1e-12 * np.trace(M).real
    _, _, parts = orc.nll_grad(Ad, Am, V, w=w, n_gen=ng, parts=True)
    S = parts["s_raw"] / ng
    assert abs(np.vdot(V, M @ V).real - S) < 1e-12 * S
    # per-event: I_i = sum_ab V_a (A_ia conj(A_ib)) conj(V_b)
    Ii = np.einsum("a,ia,ib,b->i", V, Ad, Ad.conj(), V.conj()).real
    assert _rel(orc.intensity(Ad, V), Ii) < 1e-13
    # Gram-form likelihood equals the streamed one
    n1, g1 = orc.nll_grad(Ad, Am, V, w=w, n_gen=ng)
    n2, g2 = orc.nll_grad_gram(Ad, M, V)
    assert abs(n1 - n2) < 1e-12 * (abs(n1) + 40)
    assert _rel(g1, g2) < 1e-11
    n1, g1 = orc.nll_grad(Ad, Am, V, w=w, n_gen=ng, extended=True)
    n2, g2 = orc.nll_grad_gram(Ad, M, V, extended=True)
    assert abs(n1 - n2) < 1e-12 * (abs(n1) + 40)
    assert _rel(g1, g2) < 1e-11


def pin_permutation(orc):
    """Events are independent (Section 3): shuffling rows changes only the summation order."""
    Ad, Am, V, w = _small_case(31, nd=200, nm=500, weighted=True)
    g = np.random.default_rng(31)
    pd, pm = g.permutation(200), g.permutation(500)
    n1, g1 = orc.nll_grad(Ad, Am, V, w=w)
    n2, g2 = orc.nll_grad(Ad[pd], Am[pm], V, w=w[pm])
    assert abs(n1 - n2) < 1e-13 * (abs(n1) + 200)
    assert _rel(g1, g2) < 1e-12


def pin_shard_combination(orc):
    """Events shard (Section 3): raw sums (sum ln I, sum w I, the data and MC gradient
    sums) of disjoint chunks of the data and MC rows add to those of the whole sample,
    and the nonlinear combine of the added sums gives the whole-sample NLL and gradient."""
    Ad, Am, V, w = _small_case(37, nd=301, nm=907, weighted=True)
    whole_n, whole_g, whole_p = orc.nll_grad(Ad, Am, V, w=w, parts=True)
    cd, cm = [0, 97, 210, 301], [0, 400, 555, 907]
    tot = None
    for i in range(3):
        _, _, p = orc.nll_grad(Ad[cd[i]:cd[i + 1]], Am[cm[i]:cm[i + 1]], V, w=w[cm[i]:cm[i + 1]],
                               n_gen=Am.shape[0], parts=True)
        tot = dict(p) if tot is None else {k: tot[k] + p[k] for k in tot}
    for key in ("sum_log", "s_raw"):
        assert abs(tot[key] - whole_p[key]) < 1e-12 * (abs(whole_p[key]) + 1), key
    for key in ("GD", "HM"):
        assert _rel(tot[key], whole_p[key]) < 1e-12, key
    nd, ng = Ad.shape[0], Am.shape[0]
    nll = -tot["sum_log"] + nd * np.log(tot["s_raw"] / ng)
    grad = 2 * (-tot["GD"] + nd / tot["s_raw"] * tot["HM"])
    assert abs(nll - whole_n) < 1e-12 * (abs(whole_n) + nd)
    assert _rel(grad, whole_g) < 1e-11


# ---------------------------------------------------------- exact arithmetic
def _frac_c(z):
    return (Fraction(z.real), Fraction(z.imag))


def pin_gaussian_integers_exact(orc):
    """Integer amplitudes and V: Eq. 1 intensities are integers, and the oracle's must
    equal exact integer arithmetic bit for bit."""
    g = np.random.default_rng(37)
    A = synth.gaussian_integer_amplitudes(g, 300, 48, 4, np.complex128)
    V = (g.integers(-4, 5, 48) + 1j * g.integers(-4, 5, 48))
    I = orc.intensity(A, V)
    Ai = [[(int(a.real), int(a.imag)) for a in row] for row in A]
    Vi = [(int(v.real), int(v.imag)) for v in V]
    for i, row in enumerate(Ai):
        zr = sum(vr * ar - vi * ai for (ar, ai), (vr, vi) in zip(row, Vi))
        zi = sum(vr * ai + vi * ar for (ar, ai), (vr, vi) in zip(row, Vi))
        assert I[i] == float(zr * zr + zi * zi)


def _brute(Ad, Am, V, w, ng, extended):
    """Exact rational z, I, S and gradient sums; logs of the correctly rounded I."""
    k = len(V)
    Vf = [_frac_c(v) for v in V]

    def zrow(row):
        r = sum(vr * ar - vi * ai for (ar, ai), (vr, vi) in zip(row, Vf))
        i = sum(vr * ai + vi * ar for (ar, ai), (vr, vi) in zip(row, Vf))
        return r, i

    rowsd = [[_frac_c(a) for a in row] for row in Ad]
    rowsm = [[_frac_c(a) for a in row] for row in Am]
    logs = []
    GD = [[Fraction(0), Fraction(0)] for _ in range(k)]
    for row in rowsd:
        zr, zi = zrow(row)
        I = zr * zr + zi * zi
        logs.append(math.log(float(I)))
        ur, ui = zr / I, zi / I
        for a, (ar, ai) in enumerate(row):
            GD[a][0] += ar * ur + ai * ui
            GD[a][1] += ar * ui - ai * ur
    sraw = Fraction(0)
    HM = [[Fraction(0), Fraction(0)] for _ in range(k)]
    for j, row in enumerate(rowsm):
        zr, zi = zrow(row)
        wj = Fraction(w[j]) if w is not None else Fraction(1)
        sraw += wj * (zr * zr + zi * zi)
        for a, (ar, ai) in enumerate(row):
            HM[a][0] += wj * (ar * zr + ai * zi)
            HM[a][1] += wj * (ar * zi - ai * zr)
    nd = len(rowsd)
    S = sraw / Fraction(ng)
    if extended:
        nll = -math.fsum(logs) + float(S)
        c = Fraction(1) / Fraction(ng)
    else:
        nll = -math.fsum(logs) + nd * math.log(float(S))
        c = Fraction(nd) / sraw
    grad = []
    for a in range(k):
        grad += [float(2 * (-GD[a][0] + c * HM[a][0])), float(2 * (-GD[a][1] + c * HM[a][1]))]
    return nll, np.array(grad)


def pin_brute_force(orc):
    """Tiny inputs (N <= 8, K <= 4): exact rational arithmetic for z, I, S and the gradient
    sums, math.fsum for the log sum, against the oracle at 1e-14 (Eq. 1-3)."""
    g = np.random.default_rng(41)
    for k in (1, 2, 3, 4):
        for extended in (False, True):
            nd, nm = int(g.integers(1, 9)), int(g.integers(1, 9))
            Ad = synth.random_amplitudes(g, nd, k, np.complex128)
            Am = synth.random_amplitudes(g, nm, k, np.complex128)
            V = synth.draw_v(g, 1, k)[0]
            w = g.uniform(0.1, 2.0, nm)
            ng = float(nm + int(g.integers(0, 5)))
            nb, gb = _brute(Ad, Am, V, w, ng, extended)
            no, go = orc.nll_grad(Ad, Am, V, w=w, n_gen=ng, extended=extended)
            assert abs(no - nb) < 1e-14 * (abs(nb) + nd)
            # K = 1 has an exactly zero gradient: compare on an absolute floor of 1
            assert _rel(go, gb, scale=max(np.max(np.abs(gb)), 1.0)) < 1e-13


# ------------------------------------------------------------ differentiation
def _fd_grad(f, V, h):
    """Central differences with one Richardson step, in the real coordinates (Re V_a, Im V_a)."""
    k = len(V)
    out = np.empty(2 * k)
    for a in range(k):
        for part, e in ((0, 1.0), (1, 1j)):
            def d(hh):
                dv = np.zeros(k, complex)
                dv[a] = e * hh
                return (f(V + dv) - f(V - dv)) / (2 * hh)
            out[2 * a + part] = (4 * d(h / 2) - d(h)) / 3
    return out


def pin_finite_differences(orc):
    """The returned gradient is dNLL/d(Re V_a, Im V_a): central differences, h = 1e-4
    (FP64), with one Richardson step, for both likelihood forms and the Gram form."""
    Ad, Am, V, w = _small_case(43, nd=30, nm=90, k=4, weighted=True)
    for extended in (False, True):
        f = lambda v: orc.nll_grad(Ad, Am, v, w=w, n_gen=123.0, extended=extended)[0]
        _, grad = orc.nll_grad(Ad, Am, V, w=w, n_gen=123.0, extended=extended)
        fd = _fd_grad(f, V, 1e-4)
        assert _rel(grad, fd) < 1e-7, (extended, grad, fd)
    M = orc.gram(Am, w=w, n_gen=123.0)
    f = lambda v: orc.nll_grad_gram(Ad, M, v)[0]
    _, grad = orc.nll_grad_gram(Ad, M, V)
    assert _rel(grad, _fd_grad(f, V, 1e-4)) < 1e-7


# --------------------------------------------------------------- edge cases
def pin_edge_cases(orc):
    """No data: Eq. 2 gives ln L = 0 (empty product).  A data intensity of 0 or V = 0
    makes -ln L infinite.  No MC rows with data present is invalid."""
    Ad, Am, V, w = _small_case(47)
    nll, grad = orc.nll_grad(Ad[:0], Am, V)
    assert nll == 0.0 and np.all(grad == 0)
    nll, _ = orc.nll_grad(Ad, Am, np.zeros_like(V))
    assert nll == math.inf
    Az = Ad.copy()
    Az[5] = 0
    nll, _ = orc.nll_grad(Az, Am, V)
    assert nll == math.inf
    try:
        orc.nll_grad(Ad, Am[:0], V)
    except ValueError:
        pass
    else:
        raise AssertionError("no MC rows accepted")


def pin_summation_accuracy(orc):
    """Sums over events must not lose small terms next to a large one (the paper's
    remark that the double-precision final sum depends on the summation
    algorithm): with K = 1, A = V = 1 and MC weights (1e16, 1, ..., 1) the raw MC
    sum is exactly 1e16 + n, and the data log-sum of I = (e^30, 1, ..., 1) keeps
    every term."""
    n = 10000
    Am = np.ones((n + 1, 1), complex)
    w = np.ones(n + 1)
    w[0] = 1e16
    Ad = np.ones((n + 1, 1), complex)
    Ad[0, 0] = math.exp(15.0)
    V = np.array([1.0 + 0j])
    _, _, parts = orc.nll_grad(Ad, Am, V, w=w, parts=True)
    assert parts["s_raw"] == 1e16 + n
    assert parts["HM"][0] == 1e16 + n
    assert abs(parts["sum_log"] - math.log(math.exp(15.0) ** 2)) < 1e-14 * 30
    # with K = 1 and V = 1 every data term conj(A) z / I is exactly 1
    assert parts["GD"][0] == n + 1


# ---------------------------------------------------------- statistical pin
def pin_fit_recovers_truth(orc):
    """The likelihood is maximised near the vector the data were drawn at: fit the
    K=4 J/psi -> gamma K+K- stand-in (5000 data, 50000 flat MC) from a perturbed
    start with V_0 fixed to 1 (the Eq. 2 likelihood cannot see a complex scale)
    and check, with the curvature of the fitted NLL, that the truth is a
    statistically acceptable point: 2 (NLL(truth) - NLL(fit)) below the 99.9%
    quantile of chi^2 with 6 degrees of freedom, every pull below 4 (Eq. 2 used
    as a fit, Section 2)."""
    from scipy.optimize import minimize
    s = synth.make_sample(0, scale=0.5)
    vt = s.V_true / s.V_true[0]
    k = s.k

    def unpack(x):
        return np.concatenate([[1.0 + 0j], x[0::2] + 1j * x[1::2]])

    def fun(x):
        nll, grad = orc.nll_grad(s.A_data, s.A_mc, unpack(x))
        return nll, grad[2:]

    xt = np.empty(2 * (k - 1))
    xt[0::2], xt[1::2] = vt[1:].real, vt[1:].imag
    g = np.random.default_rng(53)
    x0 = xt * (1 + 0.3 * g.standard_normal(xt.shape))
    res = minimize(fun, x0, jac=True, method="L-BFGS-B", options=dict(maxiter=500, gtol=1e-9))
    n_fit, n_true = fun(res.x)[0], fun(xt)[0]
    assert n_fit <= n_true + 1e-6
    assert 2 * (n_true - n_fit) < 22.46, (n_true, n_fit)
    # covariance from the finite-difference Hessian of the analytic gradient
    x = res.x
    h = 1e-4 * np.maximum(1.0, np.abs(x))
    H = np.empty((x.size, x.size))
    for i in range(x.size):
        e = np.zeros(x.size)
        e[i] = h[i]
        H[i] = (fun(x + e)[1] - fun(x - e)[1]) / (2 * h[i])
    H = 0.5 * (H + H.T)
    assert np.min(np.linalg.eigvalsh(H)) > 0
    sigma = np.sqrt(np.diag(np.linalg.inv(H)))
    pulls = (x - xt) / sigma
    assert np.max(np.abs(pulls)) < 4.0, pulls


PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
