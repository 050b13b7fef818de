"""Pins of the oracle's L-BFGS and multi-level driver."""

import numpy as np
import pytest

import oracle as O
from paper_1812_06765_amd import synth


def _dense_bfgs_inverse(S, Tp, n):
    """Inverse-Hessian BFGS recursion H_{k+1} = V^T H_k V + rho s s^T with
    V = I - rho t s^T, started from gamma I of the newest pair."""
    s, t = S[-1], Tp[-1]
    H = (s @ t) / (t @ t) * np.eye(n)
    for s, t in zip(S, Tp):
        rho = 1.0 / (s @ t)
        V = np.eye(n) - rho * np.outer(t, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("n,k", [(7, 1), (20, 3), (50, 5)])
def test_two_loop_equals_dense_bfgs(n, k):
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(k)]
    Tp = [A @ s for s in S]
    opt = O.LBFGS(lambda v: (0.0, np.zeros(n)), np.zeros(n), mem=k)
    opt.S, opt.Tp = list(S), list(Tp)
    g = rng.standard_normal(n)
    H = _dense_bfgs_inverse(S, Tp, n)
    assert np.max(np.abs(opt.two_loop(g) + H @ g)) < 1e-10 * np.abs(H @ g).max()


def test_lbfgs_solves_convex_quadratic():
    rng = np.random.default_rng(2)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + 0.5 * np.eye(n)
    b = rng.standard_normal(n)

    def fun(x):
        return 0.5 * x @ A @ x - b @ x, A @ x - b

    opt = O.LBFGS(fun, np.zeros(n), mem=5, h_min=1.0)
    for _ in range(400):
        info, _ = opt.step()
        if info != O.INFO["OK"]:
            break
    x = np.linalg.solve(A, b)
    assert np.max(np.abs(opt.y - x)) < 1e-6 * np.abs(x).max()


def test_lbfgs_first_step_and_armijo():
    n = 4
    A = np.diag([1.0, 10.0, 100.0, 1000.0])

    def fun(x):
        return 0.5 * x @ A @ x, A @ x

    x0 = np.ones(n)
    opt = O.LBFGS(fun, x0, mem=3, h_min=0.5)
    J0, g0 = fun(x0)
    info, t = opt.step()
    assert info == O.INFO["OK"]
    d = -g0 * (0.5 / np.abs(g0).max())
    assert np.max(np.abs(opt.y - (x0 + t * d))) < 1e-15
    assert opt.J <= J0 + 1e-4 * t * (g0 @ d)
    # a failed line search leaves the iterate unchanged
    stuck = O.LBFGS(lambda v: (float(np.sum(v)) if np.all(v == 1.0) else 1e9, np.ones(n)),
                    np.ones(n), mem=3)
    info, _ = stuck.step()
    assert info == O.INFO["LINESEARCH_FAIL"] and np.array_equal(stuck.y, np.ones(n))


def test_register_reduces_objective_and_error():
    """Two-level registration of a small blob pair: J falls on every level and
    the deformation moves towards the known inverse of the generating field."""
    m = (16, 16, 16)
    pr = synth.blob_phantom_pair(m, seed_R=1, seed_u=2, max_disp=1.5)
    rec = []
    y, rep = O.register(pr.R, pr.T, (1.0, 1.0, 1.0), levels=2, alpha=0.1, tau=0.1, rho=0.1,
                        max_iter=15, mem=5, record=rec)
    assert y.shape == (3, 9, 9, 9)
    for lev in (1, 0):
        Js = [J for (lv, J) in rec if lv == lev]
        assert len(Js) >= 3 and all(b <= a for a, b in zip(Js, Js[1:]))
    # ground truth on the image grid: y*(x) solves z + u(z) = x (voxel units)
    x = synth.voxel_centres(m)
    zstar = synth.invert_displacement(pr.field, x)
    yhat = O.apply_P(y, m, (9, 9, 9))
    ident = O.apply_P(O.identity(m, (1.0, 1.0, 1.0), (9, 9, 9)), m, (9, 9, 9))
    inner = (slice(None), slice(3, 13), slice(3, 13), slice(3, 13))
    err0 = np.sqrt(((ident - zstar)[inner] ** 2).sum(0)).mean()
    err1 = np.sqrt(((yhat - zstar)[inner] ** 2).sum(0)).mean()
    assert err1 < 0.8 * err0
