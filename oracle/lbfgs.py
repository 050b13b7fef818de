"""Limited-memory BFGS and the multi-level registration driver (FP64).

Sec. 2.1 solves Eq. 1 with L-BFGS (Nocedal, 1980) inside a coarse-to-fine
scheme.  The paper fixes no memory size, initial scaling, line search or
stopping rule; the reading used here (textbook choices) is:

* Memory m_L pairs (s_k, t_k) with s_k = y_{k+1} - y_k and
  t_k = grad_{k+1} - grad_k; a pair is stored only if s^T t > 1e-10 |s| |t|.
* Direction d = -H g by the two-loop recursion, initial matrix
  H0 = gamma I with gamma = s^T t / t^T t of the newest pair.
* With no stored pair, d = -g * (h_min / |g|_inf): the first step moves no node
  component by more than the finest image spacing of the level.
* If g^T d >= 0 the memory is dropped and the first-step direction is used.
* Armijo backtracking: t = 1, 1/2, ... (at most 10 halvings), accept when
  J(y + t d) <= J(y) + c1 t g^T d with c1 = 1e-4; otherwise the iteration
  fails and y is left unchanged.
* A level stops after max_iter iterations, on a failed line search, on a zero
  gradient, or (if enabled) when J decreases by at most tol (1 + |J|).
* Levels run from the coarsest to the finest; the coarsest starts at the
  identity, every finer level at the prolongated result of the level below.
"""

from __future__ import annotations

import numpy as np

from .grids import identity, level_shapes, prolongate, pyramid
from .objective import Problem, eval_J_grad

INFO = {"OK": 0, "CONVERGED": 1, "MAX_ITER": 2, "LINESEARCH_FAIL": 3, "NONFINITE": 4}


class LBFGS:
    """L-BFGS state for one level; ``fun(y) -> (J, grad)``."""

    def __init__(self, fun, y0, mem=5, h_min=1.0, c1=1e-4, max_halvings=10):
        self.fun = fun
        self.mem = mem
        self.h_min = float(h_min)
        self.c1 = c1
        self.max_halvings = max_halvings
        self.y = np.asarray(y0, dtype=np.float64).copy()
        self.J, self.g = fun(self.y)
        self.S, self.Tp = [], []
        self.evals = 1

    def reset(self):
        self.S, self.Tp = [], []

    def first_direction(self, g):
        gmax = float(np.max(np.abs(g)))
        return -g * (self.h_min / gmax)

    def two_loop(self, g):
        """d = -H g (two-loop recursion, newest pair last in the lists)."""
        q = g.copy()
        a = [0.0] * len(self.S)
        rho = [1.0 / float(np.vdot(s, t)) for s, t in zip(self.S, self.Tp)]
        for i in reversed(range(len(self.S))):
            a[i] = rho[i] * float(np.vdot(self.S[i], q))
            q = q - a[i] * self.Tp[i]
        s, t = self.S[-1], self.Tp[-1]
        gamma = float(np.vdot(s, t)) / float(np.vdot(t, t))
        r = gamma * q
        for i in range(len(self.S)):
            b = rho[i] * float(np.vdot(self.Tp[i], r))
            r = r + (a[i] - b) * self.S[i]
        return -r

    def direction(self, g):
        if not self.S:
            return self.first_direction(g)
        return self.two_loop(g)

    def descent_direction(self, g):
        """(d, g^T d) for this iteration: the quasi-Newton direction, or, if it
        does not descend (g^T d >= 0), the first-step direction after the
        memory is dropped."""
        d = self.direction(g)
        gtd = float(np.vdot(g, d))
        if not gtd < 0.0:
            self.reset()
            d = self.first_direction(g)
            gtd = float(np.vdot(g, d))
        return d, gtd

    @staticmethod
    def keep_pair(s, tv) -> bool:
        """Curvature test of a new pair: stored only if s^T t > 1e-10 |s| |t|."""
        st = float(np.vdot(s, tv))
        return st > 1e-10 * float(np.linalg.norm(s)) * float(np.linalg.norm(tv))

    def store_pair(self, s, tv):
        """Append the newest pair; beyond m_L pairs the oldest is dropped."""
        self.S.append(s)
        self.Tp.append(tv)
        if len(self.S) > self.mem:
            self.S.pop(0)
            self.Tp.pop(0)

    def step(self):
        """One iteration; returns (info, t)."""
        g = self.g
        if not np.all(np.isfinite(g)) or not np.isfinite(self.J):
            return INFO["NONFINITE"], 0.0
        if float(np.max(np.abs(g))) == 0.0:
            return INFO["CONVERGED"], 0.0
        d, gtd = self.descent_direction(g)
        t = 1.0
        for _ in range(self.max_halvings + 1):
            yt = self.y + t * d
            Jt, gt = self.fun(yt)
            self.evals += 1
            if np.isfinite(Jt) and Jt <= self.J + self.c1 * t * gtd:
                s = yt - self.y
                tv = gt - g
                if self.keep_pair(s, tv):
                    self.store_pair(s, tv)
                self.y, self.J, self.g = yt, float(Jt), gt
                return INFO["OK"], t
            t *= 0.5
        return INFO["LINESEARCH_FAIL"], 0.0


def early_stop_met(J_old: float, J_new: float, tol: float) -> bool:
    """Early-stop test of a level: the accepted step lowered J by at most
    tol (1 + |J|), measured at the objective before the step."""
    return (J_old - J_new) <= tol * (1.0 + abs(J_old))


def register(R, T, h, levels=3, ratio=2, alpha=0.1, tau=1.0, rho=1.0, max_iter=50,
             mem=5, tol=1e-6, early_stop=False, record=None, my0=None):
    """Multi-level registration (Sec. 2.1): returns the finest-level y and a
    per-level list of (iterations, evaluations, final J, final info).

    ``record``, if given, is a list that receives one (level, J) tuple per
    accepted iteration.  ``my0``: deformation-grid node counts of level 0
    (default m / ratio + 1 per axis), see ``level_shapes``.
    """
    m = R.shape
    shapes = level_shapes(m, h, levels, ratio, my0)
    Rs, Ts = pyramid(R, T, levels)
    y = None
    report = []
    for lev in reversed(range(levels)):
        ml, hl, myl = shapes[lev]
        prob = Problem(Rs[lev], Ts[lev], hl, myl, alpha, tau, rho)
        if y is None:
            y = identity(ml, hl, myl)
        else:
            y = prolongate(y)
        opt = LBFGS(lambda v, p=prob: eval_J_grad(p, v)[:2], y, mem=mem, h_min=min(hl))
        info, it = INFO["MAX_ITER"], 0
        while it < max_iter:
            J_old = opt.J
            st, _ = opt.step()
            if st != INFO["OK"]:
                info = st
                break
            it += 1
            if record is not None:
                record.append((lev, opt.J))
            if early_stop and early_stop_met(J_old, opt.J, tol):
                info = INFO["CONVERGED"]
                break
        y = opt.y
        report.append((lev, it, opt.evals, opt.J, info))
    return y, report
