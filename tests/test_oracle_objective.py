"""Pins of the oracle's full objective J = D + alpha S and its gradients:
central finite differences of J over every y entry on small grids, the
template derivative against finite differences and against the transpose of
scipy's trilinear warp."""

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from oracle.objective import crossing_mask
from paper_1812_06765_amd import synth


def _problem(m, h, seed=1, alpha=0.1, eps=0.1):
    pr = synth.blob_phantom_pair(m, h, seed_R=seed, seed_u=seed + 1, max_disp=1.0)
    my = tuple(v // 2 + 1 for v in m)
    return O.Problem(pr.R, pr.T, h, my, alpha, eps, eps)


@pytest.mark.parametrize("m,h", [((8, 8, 8), (1.0, 1.0, 1.0)), ((8, 12, 6), (1.0, 0.5, 2.0))])
def test_gradient_matches_central_fd_everywhere(m, h):
    p = _problem(m, h)
    rng = np.random.default_rng(4)
    y = p.identity() + 0.35 * rng.standard_normal((3,) + p.my) * min(h)
    J, g, _ = O.eval_J_grad(p, y)
    eps = 1e-6
    bad = crossing_mask(p, y, eps)
    assert bad.sum() < 0.05 * bad.size
    fd = np.zeros_like(y)
    for idx in np.ndindex(*y.shape):
        if bad[idx]:
            continue
        yp = y.copy()
        yp[idx] += eps
        ym = y.copy()
        ym[idx] -= eps
        fd[idx] = (O.eval_J_grad(p, yp)[0] - O.eval_J_grad(p, ym)[0]) / (2 * eps)
    err = np.abs(fd - g)[~bad]
    assert err.max() < 1e-6 * np.abs(g).max()


def test_template_gradient_matches_fd():
    m, h = (8, 8, 8), (1.0, 1.0, 1.0)
    p = _problem(m, h, seed=5)
    rng = np.random.default_rng(6)
    y = p.identity() + 0.35 * rng.standard_normal((3,) + p.my)
    J, g, gT, _ = O.eval_J_grad_T(p, y)
    J2, g2, _ = O.eval_J_grad(p, y)
    assert J == J2 and np.array_equal(g, g2)
    eps = 1e-6
    T0 = p.T.astype(np.float64)
    for k in [(0, 0, 0), (3, 4, 5), (7, 7, 7), (2, 6, 1), (5, 0, 3), (4, 4, 4)]:
        out = []
        for sgn in (1.0, -1.0):
            Tk = T0.copy()
            Tk[k] += sgn * eps
            q = O.Problem(p.R, Tk, h, p.my, p.alpha, p.tau, p.rho)
            out.append(O.eval_J_grad(q, y)[0])
        fd = (out[0] - out[1]) / (2 * eps)
        assert abs(fd - gT[k]) < 1e-6 * max(1.0, np.abs(gT).max())


def test_template_adjoint_is_transpose_of_map_coordinates():
    """The warp is linear in T for fixed points, so <W T', e> = <T', W^T e>
    with W taken from scipy's trilinear map_coordinates (nearest mode)."""
    rng = np.random.default_rng(7)
    m, h = (9, 8, 7), (1.0, 2.0, 0.5)
    x = np.stack(np.meshgrid(*[O.image_coords_1d(m[d], h[d]) for d in range(3)],
                             indexing="ij"))
    yhat = x + 1.5 * rng.standard_normal(x.shape) * np.asarray(h).reshape(3, 1, 1, 1)
    _, _, cells = O.warp(np.zeros(m), h, yhat)
    e = rng.standard_normal(m)
    Tp = rng.standard_normal(m)
    coords = np.stack([yhat[d] / h[d] - 0.5 for d in range(3)])
    lhs = float(np.vdot(ndimage.map_coordinates(Tp, coords, order=1, mode="nearest"), e))
    rhs = float(np.vdot(Tp, O.warp_T_adjoint(e, m, cells)))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_objective_parts_and_alpha():
    p = _problem((8, 8, 8), (1.0, 1.0, 1.0), alpha=0.0)
    rng = np.random.default_rng(8)
    y = p.identity() + 0.3 * rng.standard_normal((3,) + p.my)
    J0, g0, (D0, S0) = O.eval_J_grad(p, y)
    q = O.Problem(p.R, p.T, p.h, p.my, 2.5, p.tau, p.rho)
    J1, g1, (D1, S1) = O.eval_J_grad(q, y)
    assert D0 == D1 and S0 == S1 and J0 == D0
    assert abs(J1 - (D1 + 2.5 * S1)) < 1e-12 * J1
    _, gS = O.curvature(y - p.identity(), p.hy)
    assert np.max(np.abs(g1 - (g0 + 2.5 * gS))) < 1e-12 * np.abs(g1).max()


def _cut_gradient(R, T, y, n0, B, margin):
    """grad J of the objective on the images cut out around a box of B^3
    nodes at n0 (a margin of ``margin`` node cells, clipped at the faces), at
    y shifted to the cut's origin; returned at the box's nodes."""
    my = y.shape[1:]
    lo = [max(n0[d] - margin, 0) for d in range(3)]
    hi = [min(n0[d] + B + margin, my[d] - 1) for d in range(3)]
    cut = tuple(slice(2 * lo[d], 2 * hi[d]) for d in range(3))
    ys = y[(slice(None),) + tuple(slice(lo[d], hi[d] + 1) for d in range(3))].copy()
    for d in range(3):
        ys[d] -= 2.0 * lo[d]
    p = O.Problem(R[cut], T[cut], (1.0, 1.0, 1.0), ys.shape[1:], 0.1, 10.0, 10.0)
    _, g, _ = O.eval_J_grad(p, ys)
    return g[(slice(None),) + tuple(slice(n0[d] - lo[d], n0[d] - lo[d] + B) for d in range(3))]


def test_gradient_is_local_to_a_cut():
    """A node's gradient depends only on the image points of its index sets
    (Eq. 3), their difference stencils, the template where they are warped
    to and the nodes two cells around it.  So the objective on the images
    cut out with a margin of 6 node cells around a box (clipped at the
    faces), at y shifted to the cut's origin, gives the full problem's
    gradient at the box's nodes exactly; with a margin of one cell it does
    not (the cut's replicated ends and the clamped warp reach the box).
    This is what lets the full-resolution GPU test compare its finest level
    with the oracle on cuts."""
    m = (48, 40, 64)
    pr = synth.ct_phantom_pair(m, seed_R=5, seed_u=6)
    my = tuple(v // 2 + 1 for v in m)
    p = O.Problem(pr.R, pr.T, (1.0, 1.0, 1.0), my, 0.1, 10.0, 10.0)
    j = [np.arange(n, dtype=np.float64) / (n - 1) for n in my]
    w = (np.sin(2 * np.pi * j[0])[:, None, None] * np.sin(np.pi * j[1])[None, :, None]
         * np.cos(np.pi * j[2])[None, None, :])
    y = (p.identity() + np.stack([2 * w, -2 * w, w])).astype(np.float32).astype(np.float64)
    _, g, _ = O.eval_J_grad(p, y)
    B = 6
    for n0 in ((9, 7, 12), (0, 0, 0), (my[0] - B, my[1] - B, my[2] - B)):
        box = (slice(None),) + tuple(slice(n0[d], n0[d] + B) for d in range(3))
        assert np.array_equal(_cut_gradient(pr.R, pr.T, y, n0, B, 6), g[box])
    n0 = (9, 7, 12)
    box = (slice(None),) + tuple(slice(n0[d], n0[d] + B) for d in range(3))
    assert not np.allclose(_cut_gradient(pr.R, pr.T, y, n0, B, 1), g[box], rtol=1e-6)
