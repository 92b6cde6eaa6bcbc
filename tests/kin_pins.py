"""Pins of the kinematic-amplitude oracle (oracle/kin.c): facts fixed by the
mathematics of the lineshape and the angular functions, or by an independent
implementation, not by the oracle itself.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError if the
oracle disagrees.  test_kin_oracle.py runs them on the oracle and on planted
mistakes in copies of kin.c (each mistake must fail some pin).

The amplitude model (stand-in lineshape of the J/psi -> gamma K+K- example in
Section 2 of Berger, "Partial Wave Analysis using Graphics Cards"; the section
notes that amplitudes are precomputed only while masses and widths are fixed):
A_a(m, x) = BW_a(m) Y_{J_a}^0(x), BW_a = 1 / (m_a^2 - m^2 - i m_a Gamma_a),
Y_J^0(x) = sqrt((2J+1)/(4 pi)) P_J(x).
"""
from __future__ import annotations

import math

import numpy as np

import synth

FOUR_PI = 4.0 * math.pi


def _y_closed(J, x):
    """Y_J^0 at x in {-1, 0, 1} from the closed forms P_J(1) = 1, P_J(-1) = (-1)^J,
    P_J(0) = 0 for odd J and (-1)^(J/2) (J-1)!! / J!! for even J."""
    norm = math.sqrt((2 * J + 1) / FOUR_PI)
    if x == 1.0:
        return norm
    if x == -1.0:
        return norm * (-1) ** J
    if J % 2:
        return 0.0
    num = math.prod(range(J - 1, 0, -2)) if J > 1 else 1
    den = math.prod(range(J, 0, -2)) if J > 0 else 1
    return norm * (-1) ** (J // 2) * num / den


def pin_peak_value_and_angular_closed_forms(orc):
    """At m = m_a the Breit-Wigner is i / (m_a Gamma_a); Y_J^0 at cos theta = -1, 0, 1
    takes its closed-form values (J = 0 .. 4)."""
    spins = np.array([0, 1, 2, 3, 4], dtype=np.int32)
    res = np.array([1.5, 0.05, 1.7, 0.1, 2.0, 0.15, 2.3, 0.2, 1.9, 0.3])
    for xv in (-1.0, 0.0, 1.0):
        for a, J in enumerate(spins):
            ma, ga = res[2 * a], res[2 * a + 1]
            A = orc.kin_amplitudes(np.array([[ma, xv]]), spins, res)[0, a]
            expect = 1j / (ma * ga) * _y_closed(int(J), xv)
            assert abs(A - expect) <= 1e-13 * max(abs(expect), 1.0 / (ma * ga)), (J, xv, A, expect)


def pin_angular_orthonormality(orc):
    """2 pi int_{-1}^{1} Y_J^0 Y_J'^0 dx = delta_JJ' (Gauss-Legendre, exact for these degrees)."""
    spins = np.arange(5, dtype=np.int32)
    res = np.tile([2.0, 0.1], 5)
    xg, wg = np.polynomial.legendre.leggauss(12)
    mx = np.stack([np.full_like(xg, 2.0), xg], axis=1)
    Y = (orc.kin_amplitudes(mx, spins, res) * (2.0 * 0.1) / 1j).real     # divide out BW(m_a)
    G = 2.0 * math.pi * (Y * wg[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(5))) < 1e-13


def pin_lineshape_integral(orc):
    """int_0^inf |BW|^2 d(m^2) = (pi/2 + atan(m_a / Gamma_a)) / (m_a Gamma_a): the Lorentzian
    in s = m^2 with half-width m_a Gamma_a, centred at m_a^2 (fixes where the width enters)."""
    from scipy.integrate import quad
    for ma, ga in ((1.5, 0.05), (2.3, 0.2)):
        res = np.array([ma, ga])

        def f(m):
            A = orc.kin_amplitudes(np.array([[m, 1.0]]), np.array([0], dtype=np.int32), res)[0, 0]
            return abs(A) ** 2 * FOUR_PI * 2.0 * m      # Y_0^0 = 1/sqrt(4 pi); d(m^2) = 2 m dm
        val = 0.0
        for lo, hi in ((0.0, ma - 20 * ga), (ma - 20 * ga, ma + 20 * ga), (ma + 20 * ga, 60.0)):
            val += quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-12, points=[ma] if lo < ma < hi else None)[0]
        tail = 1.0 / (60.0 ** 2 - ma * ma)           # int_{60^2}^inf ds / (s - m_a^2)^2, Gamma negligible
        expect = (math.pi / 2 + math.atan(ma / ga)) / (ma * ga)
        assert abs(val + tail - expect) < 1e-7 * expect, (ma, ga, val + tail, expect)


def pin_matches_precomputed_amplitudes(orc):
    """With masses and widths fixed, the kinematic NLL and V gradient equal those of the
    precomputed-amplitude oracle fed with amplitude rows from the independent numpy
    lineshape of the input generator (both forms, weighted MC)."""
    s = synth.make_kin_sample(1, n_data=400, n_mc=1500, k=7, weighted=True)
    m_d, x_d = s.mx_data[:, 0].astype(np.float64), s.mx_data[:, 1].astype(np.float64)
    m_m, x_m = s.mx_mc[:, 0].astype(np.float64), s.mx_mc[:, 1].astype(np.float64)
    Ad = synth.amplitudes(m_d, x_d, s.waves)
    Am = synth.amplitudes(m_m, x_m, s.waves)
    V = synth.eval_vectors(1, 1, s.k, stream=9)[0]
    for ext in (False, True):
        n1, g1, _ = orc.kin_nll_grad(s.mx_data, s.mx_mc, V, s.res, s.waves.J, w=s.w_mc, n_gen=1700, extended=ext)
        n2, g2 = orc.nll_grad(Ad, Am, V, w=s.w_mc, n_gen=1700, extended=ext)
        assert abs(n1 - n2) < 1e-12 * abs(n2), (ext, n1, n2)
        assert np.max(np.abs(g1 - g2)) < 1e-11 * np.max(np.abs(g2)), ext


def pin_resonance_gradient_richardson(orc):
    """dNLL/dm_a and dNLL/dGamma_a against Richardson-extrapolated central differences
    (h = 1e-5 and h/2), every wave, both likelihood forms."""
    s = synth.make_kin_sample(1, n_data=300, n_mc=1200, k=5, weighted=True)
    V = synth.eval_vectors(1, 1, s.k, stream=4)[0]
    for ext in (False, True):
        f0, _, gr = orc.kin_nll_grad(s.mx_data, s.mx_mc, V, s.res, s.waves.J, w=s.w_mc, extended=ext)
        fd = np.empty_like(gr)
        for i in range(gr.size):
            def d(h):
                rp, rm = s.res.copy(), s.res.copy()
                rp[i] += h
                rm[i] -= h
                fp = orc.kin_nll_grad(s.mx_data, s.mx_mc, V, rp, s.waves.J, w=s.w_mc, extended=ext)[0]
                fm = orc.kin_nll_grad(s.mx_data, s.mx_mc, V, rm, s.waves.J, w=s.w_mc, extended=ext)[0]
                return (fp - fm) / (2 * h)
            fd[i] = (4 * d(0.5e-5) - d(1e-5)) / 3
        assert np.max(np.abs(fd - gr)) < 1e-6 * np.max(np.abs(gr)), (ext, fd, gr)


def pin_v_gradient_central_difference(orc):
    """dNLL/dRe V_a and dNLL/dIm V_a of the kinematic form against central differences."""
    s = synth.make_kin_sample(1, n_data=300, n_mc=1000, k=4)
    V = synth.eval_vectors(1, 1, s.k, stream=5)[0]
    _, gv, _ = orc.kin_nll_grad(s.mx_data, s.mx_mc, V, s.res, s.waves.J)
    for i in range(2 * s.k):
        dv = np.zeros(s.k, dtype=complex)
        dv[i // 2] = 1e-6 if i % 2 == 0 else 1e-6j
        fp = orc.kin_nll_grad(s.mx_data, s.mx_mc, V + dv, s.res, s.waves.J)[0]
        fm = orc.kin_nll_grad(s.mx_data, s.mx_mc, V - dv, s.res, s.waves.J)[0]
        assert abs((fp - fm) / 2e-6 - gv[i]) < 1e-5 * np.max(np.abs(gv))


PINS = [pin_peak_value_and_angular_closed_forms, pin_angular_orthonormality, pin_lineshape_integral,
        pin_matches_precomputed_amplitudes, pin_resonance_gradient_richardson, pin_v_gradient_central_difference]
