"""Pins of the reference L-BFGS: the two-loop recursion is the BFGS inverse-Hessian
product, the method minimises a convex quadratic, and it reaches the same likelihood
minimum as SciPy's L-BFGS-B on the K=4 stand-in."""
import numpy as np

import oracle
import synth
from oracle.lbfgs import LbfgsOracle, two_loop


def test_two_loop_equals_explicit_bfgs():
    g = np.random.default_rng(1)
    n = 7
    S, Y = [], []
    for _ in range(5):
        s = g.standard_normal(n)
        y = s + 0.3 * g.standard_normal(n)
        assert s @ y > 0
        S.append(s)
        Y.append(y)
    gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):              # H <- (I - r s y^T) H (I - r y s^T) + r s s^T
        r = 1.0 / (s @ y)
        E = np.eye(n) - r * np.outer(s, y)
        H = E @ H @ E.T + r * np.outer(s, s)
    v = g.standard_normal(n)
    assert np.allclose(two_loop(v, S, Y), -H @ v, rtol=1e-12, atol=1e-12)


def test_quadratic_minimum():
    g = np.random.default_rng(2)
    n = 10
    Bm = g.standard_normal((n, n))
    Q = Bm @ Bm.T + n * np.eye(n)
    b = g.standard_normal(n)
    opt = LbfgsOracle(lambda x: (0.5 * x @ Q @ x - b @ x, Q @ x - b), g.standard_normal(n), ftol=1e-15)
    for _ in range(400):
        opt.step()
    assert np.allclose(opt.x, np.linalg.solve(Q, b), rtol=1e-6, atol=1e-8)


def test_likelihood_minimum_matches_scipy():
    from scipy.optimize import minimize
    s = synth.make_sample(0, scale=0.3)
    k = s.k

    def fun(x):
        V = x[0::2] + 1j * x[1::2]
        return oracle.nll_grad(s.A_data, s.A_mc, V)

    x0 = np.empty(2 * k)
    v0 = synth.eval_vectors(0, 1, k)[0]
    x0[0::2], x0[1::2] = v0.real, v0.imag
    opt = LbfgsOracle(fun, x0)
    for _ in range(600):
        opt.step()
        if opt.status:
            break
    ref = minimize(fun, x0, jac=True, method="L-BFGS-B", options=dict(maxiter=2000, gtol=1e-10, ftol=1e-15))
    assert opt.f <= ref.fun + 1e-6 * abs(ref.fun)
    assert abs(opt.f - ref.fun) < 1e-6 * abs(ref.fun)
