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

Parameters are the real vector x = (Re V_0, Im V_0, ...).
"""
from __future__ import annotations

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


class LbfgsOracle:
    def __init__(self, fun, x0, m=8, c1=1e-4, ftol=1e-12):
        self.fun, self.m, self.c1, self.ftol = fun, m, c1, ftol
        self.xt = np.array(x0, dtype=float)
        self.phase, self.status, self.iter = 0, 0, 0
        self.S, self.Y = [], []
        self.x = self.g = self.d = None
        self.f = self.alpha = self.gtd = None

    def _direction(self):
        fresh = not self.S
        d = two_loop(self.g, self.S, self.Y)
        gtd = self.g @ d
        if not gtd < 0:
            self.S, self.Y = [], []
            d = -self.g
            gtd = self.g @ d
            fresh = True
        self.d, self.gtd = d, gtd
        if fresh:
            xn, dn = np.linalg.norm(self.x), np.linalg.norm(d)
            self.alpha = 0.01 * (xn if xn > 0 else 1.0) / dn if dn > 0 else 0.0
        else:
            self.alpha = 1.0
        self.phase = 1
        self.xt = self.x + self.alpha * d

    def step(self):
        if self.status:
            return
        ft, gt = self.fun(self.xt)
        gt = np.asarray(gt, dtype=float)
        if self.phase == 0:
            self.x, self.f, self.g = self.xt.copy(), ft, gt
            self._direction()
            return
        if np.isfinite(ft) and ft <= self.f + self.c1 * self.alpha * self.gtd:
            s, y = self.xt - self.x, gt - self.g
            if s @ y > 0:
                self.S.append(s)
                self.Y.append(y)
                if len(self.S) > self.m:
                    self.S.pop(0)
                    self.Y.pop(0)
            fold = self.f
            self.x, self.f, self.g = self.xt.copy(), ft, gt
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
            self.xt = self.x + self.alpha * self.d
