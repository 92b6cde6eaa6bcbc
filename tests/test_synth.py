"""The seeded input generator: determinism, shapes, and the physics stand-in."""
import math

import numpy as np

import synth


def test_deterministic_and_shapes():
    a = synth.make_sample(0, scale=0.2)
    b = synth.make_sample(0, scale=0.2)
    assert a.A_data.shape == (2000, 4) and a.A_mc.shape == (20000, 4)
    assert a.A_data.dtype == np.complex128
    assert np.array_equal(a.A_data, b.A_data) and np.array_equal(a.A_mc, b.A_mc)
    c = synth.make_sample(1, scale=0.002)
    assert c.A_data.dtype == np.complex64 and c.A_data.shape == (2000, 16)
    assert c.A_mc.shape == (10000, 16)
    assert abs(np.angle(c.V_true[0])) < 1e-12 and c.V_true[0].real > 0


def test_spherical_harmonic_normalisation():
    # integral over the sphere of |Y_J^0|^2 is 1: 2 pi int_{-1}^{1} Y^2 dx
    x, wq = np.polynomial.legendre.leggauss(40)
    for J in (0, 2, 4, 6):
        assert abs(2 * math.pi * np.sum(wq * synth.y_j0(J, x) ** 2) - 1.0) < 1e-12


def test_breit_wigner_peak():
    m = np.array([1.5])
    assert abs(abs(synth.breit_wigner(m, 1.5, 0.05)[0]) - 1 / (1.5 * 0.05)) < 1e-12


def test_weighted_mc_estimates_flat_integral():
    # the weighted (peaked) MC sample and the flat one estimate the same integral
    s_flat = synth.make_sample(1, scale=0.02)
    s_w = synth.make_sample(1, scale=0.02, weighted=True)
    v = s_flat.V_true
    i_flat = np.abs(s_flat.A_mc.astype(np.complex128) @ v) ** 2
    i_w = np.abs(s_w.A_mc.astype(np.complex128) @ v) ** 2 * s_w.w_mc
    m1, e1 = i_flat.mean(), i_flat.std() / math.sqrt(i_flat.size)
    m2, e2 = i_w.mean(), i_w.std() / math.sqrt(i_w.size)
    assert abs(m1 - m2) < 5 * math.hypot(e1, e2)
    assert e2 < e1          # importance weighting reduces the sampling error


def test_acceptance_keeps_ngen():
    s = synth.make_sample(0, scale=0.1, accept_fraction=0.6)
    assert s.n_gen == 10000.0 and 5000 < s.A_mc.shape[0] < 7000


def test_multifit_table():
    t = synth.multifit_table(64)
    assert len(t) == 64
    for nd, k, nm in t:
        assert 10_000 <= nd <= 1_000_000 and 4 <= k <= 48 and nm == 5 * nd
