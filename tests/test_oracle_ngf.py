"""Pins of the oracle's warp, finite differences and NGF distance."""

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from paper_1812_06765_amd import synth


def _rand_points(m, h, rng, spread=2.0):
    x = np.stack(np.meshgrid(*[O.image_coords_1d(m[d], h[d]) for d in range(3)],
                             indexing="ij"))
    return x + spread * rng.standard_normal(x.shape) * np.asarray(h).reshape(3, 1, 1, 1)


@pytest.mark.parametrize("m,h", [((10, 12, 8), (1.0, 1.0, 1.0)), ((9, 7, 11), (0.5, 2.0, 1.5))])
def test_warp_equals_map_coordinates_nearest(m, h):
    rng = np.random.default_rng(1)
    T = rng.standard_normal(m)
    yhat = _rand_points(m, h, rng)  # includes points outside the domain
    Ty, _, _ = O.warp(T, h, yhat)
    coords = np.stack([yhat[d] / h[d] - 0.5 for d in range(3)])
    want = ndimage.map_coordinates(T, coords, order=1, mode="nearest")
    assert np.max(np.abs(Ty - want)) < 1e-13


def test_warp_identity_is_exact():
    pr = synth.blob_phantom_pair((16, 12, 8))
    m, h, my = (16, 12, 8), (1.0, 1.0, 1.0), (9, 7, 5)
    yhat = O.apply_P(O.identity(m, h, my), m, my)
    Ty, _, _ = O.warp(pr.T.astype(np.float64), h, yhat)
    assert np.array_equal(Ty, pr.T.astype(np.float64))


def test_warp_derivative_matches_finite_differences():
    rng = np.random.default_rng(2)
    m, h = (9, 8, 10), (1.0, 0.5, 2.0)
    T = rng.standard_normal(m)
    yhat = _rand_points(m, h, rng, spread=1.0)
    Ty, dT, _ = O.warp(T, h, yhat)
    eps = 1e-7
    for d in range(3):
        xi = yhat[d] / h[d] - 0.5
        frac = xi - np.floor(xi)
        ok = (frac > 1e-5) & (frac < 1 - 1e-5) & (np.abs(xi + 0.0) > 1e-5) \
            & (np.abs(xi - (m[d] - 1)) > 1e-5)
        yp = yhat.copy()
        yp[d] += eps
        ym = yhat.copy()
        ym[d] -= eps
        fd = (O.warp(T, h, yp)[0] - O.warp(T, h, ym)[0]) / (2 * eps)
        assert ok.sum() > 0.9 * ok.size
        assert np.max(np.abs(fd - dT[d])[ok]) < 1e-6


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cdiff_equals_correlate1d_nearest(axis):
    rng = np.random.default_rng(3)
    u = rng.standard_normal((7, 9, 6))
    h = 0.75
    want = ndimage.correlate1d(u, [-0.5, 0.0, 0.5], axis=axis, mode="nearest") / h
    assert np.max(np.abs(O.cdiff(u, h, axis) - want)) < 1e-14


@pytest.mark.parametrize("m", [3, 4, 7])
def test_cdiff_adj_is_dense_transpose(m):
    h = 1.3
    G = np.stack([O.cdiff(np.eye(m)[:, k], h, 0) for k in range(m)], axis=1)
    rng = np.random.default_rng(m)
    w = rng.standard_normal(m)
    assert np.max(np.abs(O.cdiff_adj(w, h, 0) - G.T @ w)) < 1e-14
    # and in 3D along each axis
    u = rng.standard_normal((m, m + 1, m + 2))
    for axis in range(3):
        w3 = rng.standard_normal(u.shape)
        lhs = np.vdot(O.cdiff(u, h, axis), w3)
        rhs = np.vdot(u, O.cdiff_adj(w3, h, axis))
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def _ramp_closed_form(m, h, a, b, tau, rho):
    """D for R = <a, x>, T = <b, x> at the identity: the replicated central
    difference gives a_d at interior voxels and a_d / 2 at the two end voxels
    of each axis, so every voxel falls in one of 8 classes (interior or end
    per axis) with a constant r."""
    hbar = h[0] * h[1] * h[2]
    D = 0.0
    for kx in (1.0, 0.5):
        for ky in (1.0, 0.5):
            for kz in (1.0, 0.5):
                k = (kx, ky, kz)
                count = 1
                for d in range(3):
                    count *= (m[d] - 2) if k[d] == 1.0 else 2
                gR = [a[d] * k[d] for d in range(3)]
                gT = [b[d] * k[d] for d in range(3)]
                c = sum(gT[d] * gR[d] for d in range(3)) + tau * rho
                nT = np.sqrt(sum(g * g for g in gT) + tau * tau)
                nR = np.sqrt(sum(g * g for g in gR) + rho * rho)
                D += count * (1.0 - (c / (nT * nR)) ** 2)
    return 0.5 * hbar * D


@pytest.mark.parametrize("a,b", [((1.0, 0.0, 0.0), (0.0, 1.0, 0.0)),
                                 ((0.3, -1.2, 0.8), (2.0, 0.5, -0.4))])
def test_ngf_linear_ramp_closed_form(a, b):
    m, h = (8, 10, 6), (1.0, 0.5, 2.0)
    my = (5, 6, 4)
    x = np.stack(np.meshgrid(*[O.image_coords_1d(m[d], h[d]) for d in range(3)],
                             indexing="ij"))
    R = sum(a[d] * x[d] for d in range(3))
    T = sum(b[d] * x[d] for d in range(3))
    p = O.Problem(R, T, h, my, 0.0, 0.7, 1.3)
    J, _, (D, S) = O.eval_J_grad(p, p.identity())
    want = _ramp_closed_form(m, h, a, b, 0.7, 1.3)
    assert abs(D - want) < 1e-12 * want
    assert S == 0.0 and J == D


def test_ngf_identical_images_zero_and_bounds():
    pr = synth.blob_phantom_pair((16, 16, 16))
    m, h, my = (16, 16, 16), (1.0, 1.0, 1.0), (9, 9, 9)
    p = O.Problem(pr.R, pr.R, h, my, 0.0, 0.1, 0.1)
    J, g, (D, S) = O.eval_J_grad(p, p.identity())
    assert abs(D) < 1e-12 * np.prod(m)
    assert np.max(np.abs(g)) < 1e-10
    q = O.Problem(pr.R, pr.T, h, my, 0.0, 0.1, 0.1)
    rng = np.random.default_rng(0)
    for _ in range(3):
        y = q.identity() + rng.standard_normal((3,) + my)
        _, _, (D, _) = O.eval_J_grad(q, y)
        assert 0.0 <= D <= 0.5 * np.prod(h) * np.prod(m)


def test_ngf_scale_invariance():
    pr = synth.blob_phantom_pair((12, 12, 12))
    m, h, my = (12, 12, 12), (1.0, 1.0, 1.0), (7, 7, 7)
    rng = np.random.default_rng(1)
    base = O.Problem(pr.R, pr.T, h, my, 0.0, 0.1, 0.2)
    y = base.identity() + 0.5 * rng.standard_normal((3,) + my)
    s, t = 3.0, 0.25
    scaled = O.Problem(s * pr.R.astype(np.float64), t * pr.T.astype(np.float64), h, my,
                       0.0, t * 0.1, s * 0.2)
    D0 = O.eval_J_grad(base, y)[2][0]
    D1 = O.eval_J_grad(scaled, y)[2][0]
    assert abs(D0 - D1) < 1e-12 * abs(D0)
