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


def _gaussian_bump_field(hy, amps, s=1.0, extent=10.0):
    """Node field u_c = amps[c] * exp(-|X - centre|^2 / (2 s^2)) on a nodal grid
    of spacing hy spanning [0, extent]^3, centred in the box."""
    my = [int(round(extent / hy[d])) + 1 for d in range(3)]
    x = [np.arange(my[d]) * hy[d] - 0.5 * extent for d in range(3)]
    r2 = x[0][:, None, None] ** 2 + x[1][None, :, None] ** 2 + x[2][None, None, :] ** 2
    g = np.exp(-r2 / (2.0 * s * s))
    return np.stack([a * g for a in amps])


def test_curvature_absolute_weight_converges_to_continuous_functional():
    """The discrete S approximates (1/2) int (Laplace u)^2 dx.  For a Gaussian
    bump u = a exp(-r^2 / (2 s^2)) in 3D, Laplace u = (r^2/s^4 - 3/s^2) u, and
    the integral has the closed form int (Laplace u)^2 dx = 15 pi^(3/2) a^2 / (4 s)
    (moments of the normal distribution of variance s^2/2 per axis:
    E r^2 = 3 s^2 / 2, E r^4 = 15 s^4 / 4).  The bump is 5 s from every face,
    so the replicated boundary rows play no part, the nodal sum of a smooth
    decaying integrand is exact to far below the stencil error, and the
    seven-point stencil makes the error O(h^2): it must fall fourfold when h
    halves, and the Richardson extrapolation must hit the closed form.  This
    fixes the absolute weight (the node volume hbar^y and the factor 1/2)
    that the relative pins (FD of S, <grad S, u> = 2 S) leave free."""
    s = 1.0
    amps = (1.0, -0.5, 2.0)
    exact = sum(a * a for a in amps) * 15.0 * np.pi ** 1.5 / (8.0 * s)
    hy1 = (0.25, 0.2, 0.125)                    # anisotropic node spacing
    hy2 = tuple(v / 2 for v in hy1)
    S1, _ = O.curvature(_gaussian_bump_field(hy1, amps, s), hy1)
    S2, _ = O.curvature(_gaussian_bump_field(hy2, amps, s), hy2)
    e1, e2 = S1 - exact, S2 - exact
    assert abs(e1) < 0.03 * exact and abs(e2) < 0.01 * exact
    assert 3.5 < e1 / e2 < 4.5                  # second order
    rich = (4.0 * S2 - S1) / 3.0
    assert abs(rich - exact) < 2e-4 * exact


def test_curvature_gradient_absolute_weight():
    """With S pinned absolutely, <grad S, w> must equal the directional
    derivative of S along w; for the quadratic S that is (S(u + w) - S(u - w)) / 2
    exactly (no step error), here with u and w two different bumps."""
    hy = (0.25, 0.2, 0.125)
    u = _gaussian_bump_field(hy, (1.0, 0.3, -0.7), s=1.0)
    w = _gaussian_bump_field(hy, (0.2, -1.0, 0.5), s=1.5)
    S, g = O.curvature(u, hy)
    dd = (O.curvature(u + w, hy)[0] - O.curvature(u - w, hy)[0]) / 2.0
    assert abs(float(np.vdot(g, w)) - dd) < 1e-10 * abs(dd)
