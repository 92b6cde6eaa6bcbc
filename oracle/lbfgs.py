"""FP64 reference L-BFGS (test infrastructure only; same import rules as the oracle).

The minimiser the device runs for many fits at once, written out plainly:
L-BFGS with the two-loop recursion (Nocedal & Wright, Numerical Optimization,
Algorithm 7.4), history m, initial inverse Hessian (s.y / y.y) I from the
newest pair, Armijo backtracking by halving, and the same per-evaluation
state machine (one function evaluation per step):

  start:   accept the first trial point, choose a direction;
  search:  f_t <= f + c1 alpha g.d accepts (pair enters the history if
           s.y > 0), otherwise alpha halves;
  first trial step of an empty history moves x by 1% of |x|;
  stop:    status 1 if an accepted step changes f by <= ftol (1 + |f|),
           status 2 if alpha |d|_max <= 1e-15 (1 + |x|_max).

Parameters are the real vector x = (Re V_0, Im V_0, ...), or with polar=True
(the other representation Section 4 of the paper discusses for complex fit
parameters) x = (|V_0|, arg V_0, |V_1|, arg V_1, ...) with:
  - the gradient from the Cartesian one by the chain rule of V_a = r_a e^{i phi_a};
  - arg V_0 held at 0 (its gradient component set to zero);
  - the bound r_a >= rmin kept by projecting every trial point onto it, by
    dropping direction components that push a magnitude at the bound further
    down, and by the Armijo test along the projected step,
    f_t <= f + c1 g.(x_t - x);
  - phases wrapped into [-pi, pi] after each accepted step (the history keeps
    the step taken); a direction with no descent left after dropping the
    bound components ends the fit (status 1).
"""
from __future__ import annotations

import math

import numpy as np


def two_loop(g, S, Y):
    """-H g for the pairs (oldest first) in S, Y."""
    q = np.array(g, dtype=float)
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        a = (s @ q) / (s @ y)
        alphas.append(a)
        q = q - a * y
    if S:
        q = q * ((S[-1] @ Y[-1]) / (Y[-1] @ Y[-1]))
    for (s, y), a in zip(zip(S, Y), reversed(alphas)):
        b = (y @ q) / (s @ y)
        q = q + s * (a - b)
    return -q


def polar_to_cartesian(p):
    """(r_0, phi_0, r_1, phi_1, ...) -> (Re V_0, Im V_0, ...)."""
    p = np.asarray(p, dtype=float)
    x = np.empty_like(p)
    x[0::2] = p[0::2] * np.cos(p[1::2])
    x[1::2] = p[0::2] * np.sin(p[1::2])
    return x


def polar_gradient(p, g):
    """Gradient in (r_a, phi_a) from the gradient g in (Re V_a, Im V_a) at p."""
    r, ph = p[0::2], p[1::2]
    out = np.empty_like(np.asarray(g, dtype=float))
    out[0::2] = np.cos(ph) * g[0::2] + np.sin(ph) * g[1::2]
    out[1::2] = r * (-np.sin(ph) * g[0::2] + np.cos(ph) * g[1::2])
    return out


def polar_start(V0, rmin=0.0):
    """Polar parameters of the complex start V0 with V_0 rotated to the real axis
    (arg V_0 = 0) and magnitudes raised to rmin."""
    V = np.asarray(V0, dtype=complex) * np.exp(-1j * np.angle(V0[0]))
    p = np.empty(2 * V.size)
    p[0::2] = np.maximum(np.abs(V), rmin)
    p[1::2] = np.angle(V)
    p[1] = 0.0
    return p


class LbfgsOracle:
    def __init__(self, fun, x0, m=8, c1=1e-4, ftol=1e-12, polar=False, rmin=0.0):
        """fun(x) -> (f, g) in (Re V_a, Im V_a); with polar, x0 holds polar parameters."""
        self.fun, self.m, self.c1, self.ftol = fun, m, c1, ftol
        self.polar, self.rmin = polar, rmin
        self.xt = np.array(x0, dtype=float)
        if polar:
            self.xt = self._project(self.xt)
        self.phase, self.status, self.iter = 0, 0, 0
        self.S, self.Y = [], []
        self.x = self.g = self.d = None
        self.f = self.alpha = self.gtd = None

    def _project(self, p):
        p = p.copy()
        p[0::2] = np.maximum(p[0::2], self.rmin)
        p[1] = 0.0
        return p

    def _eval(self, x):
        if not self.polar:
            ft, gt = self.fun(x)
            return ft, np.asarray(gt, dtype=float)
        ft, gt = self.fun(polar_to_cartesian(x))
        gp = polar_gradient(x, np.asarray(gt, dtype=float))
        gp[1] = 0.0
        return ft, gp

    def _trial(self):
        self.xt = self.x + self.alpha * self.d
        if self.polar:
            self.xt = self._project(self.xt)
            self.slope = self.g @ (self.xt - self.x)

    def _direction(self):
        fresh = not self.S
        d = two_loop(self.g, self.S, self.Y)
        gtd = self.g @ d
        if not gtd < 0:
            self.S, self.Y = [], []
            d = -self.g
            gtd = self.g @ d
            fresh = True
        if self.polar:
            at = np.zeros(d.size, dtype=bool)
            at[0::2] = self.x[0::2] <= self.rmin
            d = np.where(at & (d < 0), 0.0, d)
            gtd = self.g @ d
            if not gtd < 0:
                self.S, self.Y = [], []
                d = np.where(at & (self.g > 0), 0.0, -self.g)
                gtd = self.g @ d
                fresh = True
                if not gtd < 0:
                    self.status = 1
                    self.xt = self.x.copy()
                    return
        self.d, self.gtd = d, gtd
        if fresh:
            xn, dn = np.linalg.norm(self.x), np.linalg.norm(d)
            self.alpha = 0.01 * (xn if xn > 0 else 1.0) / dn if dn > 0 else 0.0
        else:
            self.alpha = 1.0
        self.phase = 1
        self._trial()

    def _armijo(self, ft):
        slope = self.slope if self.polar else self.alpha * self.gtd
        return np.isfinite(ft) and ft <= self.f + self.c1 * slope

    def step(self):
        if self.status:
            return
        ft, gt = self._eval(self.xt)
        if self.phase == 0:
            self.x, self.f, self.g = self.xt.copy(), ft, gt
            self._direction()
            return
        if self._armijo(ft):
            s, y = self.xt - self.x, gt - self.g
            if s @ y > 0:
                self.S.append(s)
                self.Y.append(y)
                if len(self.S) > self.m:
                    self.S.pop(0)
                    self.Y.pop(0)
            fold = self.f
            self.x, self.f, self.g = self.xt.copy(), ft, gt
            if self.polar:
                self.x[1::2] = [math.remainder(v, 2 * math.pi) for v in self.x[1::2]]
            self.iter += 1
            if abs(fold - ft) <= self.ftol * (1 + abs(ft)):
                self.status = 1
                self.xt = self.x.copy()
                return
            self._direction()
        else:
            self.alpha *= 0.5
            if self.alpha * np.max(np.abs(self.d)) <= 1e-15 * (1 + np.max(np.abs(self.x))):
                self.status = 2
                self.xt = self.x.copy()
                return
            self._trial()
