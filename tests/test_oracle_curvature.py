"""Pins of the oracle's curvature regulariser."""

import numpy as np
import pytest
from scipy import ndimage

import oracle as O


@pytest.mark.parametrize("hy", [(1.0, 1.0, 1.0), (2.0, 0.5, 1.5)])
def test_laplacian_equals_correlate1d_nearest(hy):
    rng = np.random.default_rng(0)
    u = rng.standard_normal((6, 7, 5))
    want = sum(ndimage.correlate1d(u, [1.0, -2.0, 1.0], axis=d, mode="nearest") / hy[d] ** 2
               for d in range(3))
    assert np.max(np.abs(O.laplacian(u, hy) - want)) < 1e-13
    if hy == (1.0, 1.0, 1.0):
        assert np.max(np.abs(O.laplacian(u, hy) - ndimage.laplace(u, mode="nearest"))) < 1e-13


def test_laplacian_symmetric_dense():
    shp = (3, 4, 3)
    n = int(np.prod(shp))
    A = np.stack([O.laplacian(np.eye(n)[k].reshape(shp), (1.0, 2.0, 0.5)).ravel()
                  for k in range(n)], axis=1)
    assert np.max(np.abs(A - A.T)) < 1e-14


def test_curvature_zero_on_shift_and_affine_interior():
    my = (7, 6, 8)
    m = tuple(2 * (v - 1) for v in my)
    h = (1.0, 1.5, 0.5)
    X = O.identity(m, h, my)
    hy = tuple(O.node_spacing(m[d], h[d], my[d]) for d in range(3))
    # a constant shift u = c (y = X + c) is not penalised at all
    c = np.broadcast_to(np.array([0.3, -2.0, 1.0])[:, None, None, None], (3,) + my).copy()
    S, g = O.curvature(c, hy)
    assert S == 0.0 and np.max(np.abs(g)) == 0.0
    S, g = O.curvature((X + c) - X, hy)
    assert S < 1e-25 and np.max(np.abs(g)) < 1e-12
    # an affine displacement has zero Laplacian at interior nodes
    A = np.array([[0.1, 0.2, -0.3], [0.05, -0.1, 0.1], [0.0, -0.2, 0.2]])
    u = np.einsum("cd,d...->c...", A, X)
    Au = np.stack([O.laplacian(u[c], hy) for c in range(3)])
    assert np.max(np.abs(Au[:, 1:-1, 1:-1, 1:-1])) < 1e-13


def test_curvature_quadratic_closed_form():
    my = (9, 9, 9)
    hy = (2.0, 1.0, 0.5)
    j = np.arange(9) * hy[0]
    c = 0.7
    u = np.zeros((3,) + my)
    u[0] = c * (j ** 2)[:, None, None]
    Au = O.laplacian(u[0], hy)
    assert np.max(np.abs(Au[1:-1] - 2.0 * c)) < 1e-12


def test_curvature_gradient_homogeneity_and_fd():
    rng = np.random.default_rng(1)
    my = (5, 6, 4)
    hy = (1.0, 2.0, 0.5)
    u = rng.standard_normal((3,) + my)
    S, g = O.curvature(u, hy)
    # S is a quadratic form: <grad S(u), u> = 2 S(u)
    assert abs(float(np.vdot(g, u)) - 2.0 * S) < 1e-10 * S
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 1), (2, 4, 5, 3), (0, 2, 2, 2)]:
        up = u.copy()
        up[idx] += eps
        um = u.copy()
        um[idx] -= eps
        fd = (O.curvature(up, hy)[0] - O.curvature(um, hy)[0]) / (2 * eps)
        assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))
