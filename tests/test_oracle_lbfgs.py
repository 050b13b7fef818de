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


def _diag_quadratic(diag):
    A = np.diag(np.asarray(diag, dtype=np.float64))

    def fun(x):
        return 0.5 * float(x @ A @ x), A @ x

    return A, fun


def _armijo_t(fun, x0, d, c1=1e-4, halvings=10):
    """First t in 1, 1/2, 1/4, ... that satisfies the Armijo condition."""
    J0, g0 = fun(x0)
    gtd = float(g0 @ d)
    t = 1.0
    for _ in range(halvings + 1):
        if fun(x0 + t * d)[0] <= J0 + c1 * t * gtd:
            return t
        t *= 0.5
    return None


def test_lbfgs_non_descent_direction_drops_memory():
    """A stored pair of negative curvature (s^T t < 0, which the pair test
    never admits but a resumed or corrupted history can hold) makes the
    two-loop matrix negative definite: with s = e1, t = -e1 it is H = -I, so
    d = -H g = g ascends.  The iteration must then drop the memory and take
    the first-step direction -g h_min / |g|_inf instead."""
    A, fun = _diag_quadratic([1.0, 2.0, 3.0, 4.0])
    x0 = np.ones(4)
    opt = O.LBFGS(fun, x0, mem=5, h_min=1.0)
    e1 = np.eye(4)[0]
    opt.S, opt.Tp = [e1.copy()], [-e1.copy()]
    g0 = A @ x0
    assert np.allclose(opt.two_loop(g0), g0)        # H = -I: an ascent direction
    info, t = opt.step()
    assert info == O.INFO["OK"]
    d = -g0 * (1.0 / np.abs(g0).max())
    assert t == _armijo_t(fun, x0, d) == 1.0
    assert np.array_equal(opt.y, x0 + t * d)
    # the old pair is gone; only the pair of this step is held
    assert len(opt.S) == 1
    assert np.array_equal(opt.S[0], opt.y - x0)
    assert np.array_equal(opt.Tp[0], A @ opt.y - g0)


def _crafted_pair_case(cos_target):
    """One L-BFGS step from y0 = 0 on a function whose value drops to 0 off
    y0 and whose gradient change t = g1 - g0 has the prescribed cosine with
    the step s (s = d exactly, since y0 = 0 and the first trial is taken)."""
    n = 6
    g0 = np.array([0.5, -1.0, 2.0, 0.25, -0.75, 1.5])
    d = -g0 * (1.0 / np.abs(g0).max())
    dn = d / np.linalg.norm(d)
    p = np.zeros(n)
    p[0], p[1] = d[1], -d[0]                      # orthogonal to d
    p /= np.linalg.norm(p)
    kappa = cos_target / np.sqrt(1.0 - cos_target ** 2)
    tv = kappa * dn + p

    def fun(y):
        if not np.any(y):
            return 1.0, g0.copy()
        return 0.0, g0 + tv

    opt = O.LBFGS(fun, np.zeros(n), mem=5, h_min=1.0)
    info, t = opt.step()
    assert info == O.INFO["OK"] and t == 1.0 and np.array_equal(opt.y, d)
    s = opt.y
    cos = float(s @ tv) / (np.linalg.norm(s) * np.linalg.norm(tv))
    return opt, cos


@pytest.mark.parametrize("cos_target,kept", [(2e-10, True), (0.5e-10, False), (0.0, False),
                                             (-0.3, False), (0.3, True)])
def test_lbfgs_pair_curvature_test(cos_target, kept):
    """A pair is stored only when s^T t > 1e-10 |s| |t| (cosine above 1e-10):
    cases just above and below the threshold, orthogonal, negative and
    plainly positive curvature."""
    opt, cos = _crafted_pair_case(cos_target)
    assert abs(cos - cos_target) < 1e-14
    assert len(opt.S) == (1 if kept else 0)


def test_lbfgs_memory_keeps_newest_pairs():
    """With more accepted steps than memory slots, the held pairs are the last
    m_L differences of the iterates and gradients, oldest first."""
    A, fun = _diag_quadratic([1.0, 3.0, 7.0, 20.0, 45.0, 100.0])
    opt = O.LBFGS(fun, np.ones(6), mem=3, h_min=0.5)
    ys, gs = [opt.y.copy()], [opt.g.copy()]
    for _ in range(6):
        info, _ = opt.step()
        assert info == O.INFO["OK"]
        ys.append(opt.y.copy())
        gs.append(opt.g.copy())
    assert len(opt.S) == 3
    for k in range(3):
        i = len(ys) - 4 + k
        assert np.array_equal(opt.S[k], ys[i + 1] - ys[i])
        assert np.array_equal(opt.Tp[k], gs[i + 1] - gs[i])


def test_early_stop_rule_on_hand_made_sequence():
    """A level stops when an accepted step lowers J by at most tol (1 + |J|)
    with |J| taken before the step.  At J = 1e6 and tol = 1e-6 the threshold
    is 1.000001; a decrease of 1.0000005 stops, one of 1.000002 does not, and
    the same decrease near J = 0 does not either.  The case J_old = 1e6,
    J_new = 1e6 - 1.0000005 separates J_old from J_new in the tolerance:
    tol (1 + J_new) = 1.0000000 < 1.0000005."""
    tol = 1e-6
    assert O.early_stop_met(1e6, 1e6 - 1.0000005, tol)
    assert not O.early_stop_met(1e6, 1e6 - 1.000002, tol)
    assert not O.early_stop_met(0.0, -1.0000005, tol)
    assert O.early_stop_met(0.0, -0.5e-6, tol)
    assert O.early_stop_met(-1e6, -1e6 - 1.0000005, tol)   # |J| for a negative J
    assert not O.early_stop_met(-1e6, -1e6 - 1.000002, tol)
    assert O.early_stop_met(5.0, 5.0, tol)                  # no decrease at all


def test_register_stops_at_first_small_decrease():
    """The driver ends a level with CONVERGED right after the first accepted
    step whose decrease meets the early-stop rule, and not before."""
    m = (8, 8, 8)
    pr = synth.blob_phantom_pair(m, seed_R=1, seed_u=2, max_disp=1.0)
    rec = []
    _, rep = O.register(pr.R, pr.T, (1.0, 1.0, 1.0), levels=1, alpha=0.1, tau=0.1, rho=0.1,
                        max_iter=60, mem=5, tol=2e-3, early_stop=True, record=rec)
    (lev, it, ev, Jf, info), = rep
    assert info == O.INFO["CONVERGED"] and 1 < it < 60
    p = O.Problem(pr.R, pr.T, (1.0, 1.0, 1.0), (5, 5, 5), 0.1, 0.1, 0.1)
    J0 = O.eval_J_grad(p, p.identity())[0]
    Js = [J0] + [J for (_, J) in rec]
    dec = [(a - b) <= 2e-3 * (1.0 + abs(a)) for a, b in zip(Js, Js[1:])]
    assert dec[-1] and not any(dec[:-1]) and len(dec) == it
