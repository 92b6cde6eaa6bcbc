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


# ---------------------------------------------------------------- polar form
from oracle.lbfgs import polar_gradient, polar_start, polar_to_cartesian  # noqa: E402


def _small_problem(seed=3):
    s = synth.make_sample(0, scale=0.3)
    V = synth.eval_vectors(0, 1, s.k, seed=seed)[0]
    return s, V


def _polar_f(s, p):
    return oracle.nll_grad(s.A_data, s.A_mc, polar_to_cartesian(p)[0::2] + 1j * polar_to_cartesian(p)[1::2])


def test_polar_chain_rule_against_richardson_differences():
    """The polar gradient (chain rule of V = r e^{i phi}) against Richardson-extrapolated
    central differences of the oracle NLL in (r_a, phi_a), every component."""
    s, V = _small_problem()
    p = np.empty(2 * s.k)
    p[0::2], p[1::2] = np.abs(V), np.angle(V)
    f0, g = _polar_f(s, p)
    gp = polar_gradient(p, g)
    fd = np.empty_like(gp)
    for i in range(p.size):
        def d(h):
            e = np.zeros_like(p)
            e[i] = h
            return (_polar_f(s, p + e)[0] - _polar_f(s, p - e)[0]) / (2 * h)
        h = 1e-4 * max(1.0, abs(p[i]))
        fd[i] = (4 * d(h / 2) - d(h)) / 3
    scale = np.max(np.abs(gp))
    assert np.max(np.abs(fd - gp)) < 1e-7 * scale


def test_polar_invariants():
    """Global phase and complex scale: the NLL (Eq. 2 form) does not change under
    V -> c V, so the phase derivatives sum to zero and sum_a r_a d/dr_a = 0;
    shifting every phase by 2 pi changes nothing (periodicity)."""
    s, V = _small_problem(5)
    p = np.empty(2 * s.k)
    p[0::2], p[1::2] = np.abs(V), np.angle(V)
    f, g = _polar_f(s, p)
    gp = polar_gradient(p, g)
    scale = np.max(np.abs(gp[1::2])) + np.max(np.abs(p[0::2] * gp[0::2]))
    assert abs(np.sum(gp[1::2])) < 1e-10 * scale
    assert abs(np.sum(p[0::2] * gp[0::2])) < 1e-10 * scale
    q = p.copy()
    q[1::2] += 2 * np.pi
    f2, g2 = _polar_f(s, q)
    assert abs(f2 - f) <= 1e-12 * abs(f)
    assert np.allclose(polar_gradient(q, g2), gp, rtol=1e-9, atol=1e-9 * np.max(np.abs(gp)))
    # the start map: V_0 rotated onto the positive real axis, magnitudes kept
    ps = polar_start(V)
    assert ps[1] == 0.0 and np.allclose(ps[0::2], np.abs(V))
    Vs = polar_to_cartesian(ps)
    assert abs(_polar_f(s, ps)[0] - f) < 1e-12 * abs(f) and Vs[1] == 0.0


def _cartesian_minimum(s, V0, extended=False):
    from scipy.optimize import minimize

    def fun(x):
        return oracle.nll_grad(s.A_data, s.A_mc, x[0::2] + 1j * x[1::2], extended=extended)
    x0 = np.empty(2 * s.k)
    x0[0::2], x0[1::2] = V0.real, V0.imag
    return minimize(fun, x0, jac=True, method="L-BFGS-B", options=dict(maxiter=3000, gtol=1e-11, ftol=1e-16))


def test_polar_lbfgs_reaches_the_cartesian_minimum():
    s, V0 = _small_problem(7)

    def fun(x):
        return oracle.nll_grad(s.A_data, s.A_mc, x[0::2] + 1j * x[1::2])
    opt = LbfgsOracle(fun, polar_start(V0), polar=True, ftol=1e-14)
    for _ in range(1500):
        opt.step()
        if opt.status:
            break
    ref = _cartesian_minimum(s, V0)
    assert opt.status == 1
    assert np.all(np.abs(opt.x[1::2]) <= np.pi) and opt.x[1] == 0.0
    assert abs(opt.f - ref.fun) < 1e-9 * abs(ref.fun)


def test_polar_bound_is_kept_and_active_at_the_optimum():
    """Eq. 3 form (no scale freedom): with rmin above a wave's magnitude at the
    minimum, every trial point keeps the bound, the fit ends on it with a
    non-negative magnitude derivative there (a boundary minimum), and its NLL
    is not below the unbounded minimum.  In the Eq. 2 form the same bound
    cannot bind (the common scale of V is free) and the unbounded minimum is
    reached."""
    s, V0 = _small_problem(7)
    for extended in (True, False):
        ref = _cartesian_minimum(s, V0, extended=True)
        Vm = ref.x[0::2] + 1j * ref.x[1::2]
        a = int(np.argmin(np.abs(Vm)))
        rmin = 1.5 * abs(Vm[a])

        def fun(x):
            return oracle.nll_grad(s.A_data, s.A_mc, x[0::2] + 1j * x[1::2], extended=extended)
        opt = LbfgsOracle(fun, polar_start(V0, rmin), polar=True, rmin=rmin, ftol=1e-14)
        seen_min = np.inf
        for _ in range(3000):
            opt.step()
            seen_min = min(seen_min, np.min(opt.xt[0::2]))
            if opt.status:
                break
        assert opt.status == 1 and seen_min >= rmin
        if extended:
            assert opt.f >= ref.fun - 1e-9 * abs(ref.fun)
            at = opt.x[0::2] <= rmin
            assert at.any()
            assert np.all(opt.g[0::2][at] >= -1e-6 * np.max(np.abs(opt.g)))
        else:
            free = _cartesian_minimum(s, V0)
            assert abs(opt.f - free.fun) < 1e-9 * abs(free.fun)
