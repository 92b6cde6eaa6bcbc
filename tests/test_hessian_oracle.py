"""The Hessian oracle against what the mathematics fixes (CPU), and broken
copies of it against the same pins.

Pins: central differences of the independent C oracle's gradient (step 1e-4,
Richardson-extrapolated); symmetry; the exact identities that follow from the
invariances of the Eq. 2 form (NLL(cV) = NLL(V) for any complex c):
  H x = -g  (real scale)   and   H (J x) = J g  (phase; J x is the direction of iV)
at any V, not only at a minimum; K = 1 gives H = 0 in the Eq. 2 form; and the
Eq. 3 form's normalisation term is the constant 2 x (the real form of M)."""
import importlib.util
import os

import numpy as np
import pytest

import oracle
import oracle.hessian as HESS
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sample(k=4, nd=400, nm=1500, seed=3):
    s = synth.make_sample(2, n_data=nd, n_mc=nm, k=k, seed=seed)
    V = synth.eval_vectors(2, 1, k, seed=seed)[0]
    return s.A_data.astype(np.complex128), s.A_mc.astype(np.complex128), V


def _x(V):
    x = np.empty(2 * V.shape[0])
    x[0::2], x[1::2] = V.real, V.imag
    return x


def _V(x):
    return x[0::2] + 1j * x[1::2]


def _fd(Ad, Am, V, extended, h=1e-4, w=None):
    """Columns of the Hessian by central differences of the C oracle's gradient,
    Richardson-extrapolated from steps h and h/2."""
    x = _x(V)
    n = x.size
    scale = np.abs(x) + 1e-3

    def col(m, step):
        e = np.zeros(n)
        e[m] = step * scale[m]
        gp = oracle.nll_grad(Ad, Am, _V(x + e), w=w, extended=extended)[1]
        gm = oracle.nll_grad(Ad, Am, _V(x - e), w=w, extended=extended)[1]
        return (gp - gm) / (2 * e[m])

    return np.stack([(4 * col(m, h / 2) - col(m, h)) / 3 for m in range(n)], axis=1)


def pin_finite_differences(M):
    for extended in (False, True):
        Ad, Am, V = _sample()
        w = np.linspace(0.5, 1.5, Am.shape[0])
        H = M.hessian(Ad, Am, V, w=w, extended=extended)
        F = _fd(Ad, Am, V, extended, w=w)
        err = np.max(np.abs(H - F)) / np.max(np.abs(H))
        assert err < 1e-7, (extended, err)


def pin_symmetric(M):
    Ad, Am, V = _sample(k=5)
    H = M.hessian(Ad, Am, V)
    assert np.max(np.abs(H - H.T)) <= 1e-12 * np.max(np.abs(H))


def pin_invariance_identities(M):
    Ad, Am, V = _sample(k=6, seed=7)
    H = M.hessian(Ad, Am, V)
    g = oracle.nll_grad(Ad, Am, V)[1]
    x = _x(V)
    Jx = _x(1j * V)
    Jg = _x(1j * _V(g))
    sc = np.max(np.abs(H)) * np.max(np.abs(x))
    assert np.max(np.abs(H @ x + g)) < 1e-10 * sc
    assert np.max(np.abs(H @ Jx - Jg)) < 1e-10 * sc


def pin_k1_zero(M):
    Ad, Am, V = _sample(k=1, seed=9)
    H = M.hessian(Ad, Am, V)
    assert np.max(np.abs(H)) < 1e-9 * Ad.shape[0]


def pin_extended_mc_term_constant(M):
    Ad, Am, V = _sample(k=3, seed=11)
    w = np.linspace(0.2, 2.0, Am.shape[0])
    _, _, h1 = M.hessian(Ad, Am, V, w=w, extended=True, parts=True)
    _, _, h2 = M.hessian(Ad, Am, 3.7 * V[::-1].copy(), w=w, extended=True, parts=True)
    assert np.max(np.abs(h1 - h2)) < 1e-12 * np.max(np.abs(h1))
    # its quadratic form at x is 2 S
    x = _x(V)
    S = oracle.nll_grad(Ad, Am, V, w=w, extended=True, parts=True)[2]["s_raw"] / Am.shape[0]
    assert abs(x @ h1 @ x - 2 * S) < 1e-10 * abs(2 * S)


PINS = [pin_finite_differences, pin_symmetric, pin_invariance_identities, pin_k1_zero,
        pin_extended_mc_term_constant]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(HESS)


MUTANTS = {
    "no_outer_term": ("h_log = d2 - outer", "h_log = d2"),
    "outer_sign": ("h_log = d2 - outer", "h_log = d2 + outer"),
    "no_factor_two_d2I": ("d2 = 2.0 * np.einsum", "d2 = 1.0 * np.einsum"),
    "outer_one_power_of_I": ("1.0 / Id ** 2)", "1.0 / Id)"),
    "mc_no_nd": ("h_mc = nd * (d2S / S - np.outer(dS, dS) / S ** 2)", "h_mc = (d2S / S - np.outer(dS, dS) / S ** 2)"),
    "mc_no_dS_term": ("h_mc = nd * (d2S / S - np.outer(dS, dS) / S ** 2)", "h_mc = nd * (d2S / S)"),
    "conj_b_dropped": ("np.einsum(\"im,in,i->mn\", np.conj(bd), bd", "np.einsum(\"im,in,i->mn\", bd, bd"),
    "b_im_not_rotated": ("b[:, 1::2] = 1j * A", "b[:, 1::2] = A"),
    "weights_dropped": ("dS = (wm[:, None] * dIm).sum(axis=0) / ng", "dS = dIm.sum(axis=0) / ng"),
    "data_sign": ("h_data = -h_log", "h_data = h_log"),
}


def _mutant(name):
    src = open(os.path.join(ROOT, "oracle", "hessian.py")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    spec = importlib.util.spec_from_loader(f"hess_mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    M = _mutant(name)
    caught = []
    for pin in PINS:
        try:
            pin(M)
        except Exception:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passes every pin"
