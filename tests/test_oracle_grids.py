"""Pins of the oracle's grids, index maps, P, P^T, pyramid and prolongation.

Each check compares the oracle against something other than itself: exact
rationals, numpy's linear interpolation, brute-force dense matrices,
closed forms and adjoint identities.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O

SIZES = [8, 16, 32, 64, 96, 128, 160, 192, 256]


def _check_index_map(m, my):
    j0, r, den, w0, w1 = O.index_map(m, my)
    j0f, w0f, w1f = O.index_map_f32(m, my)
    hy = Fraction(m, my - 1)  # in units of h
    for i in range(m):
        pos = Fraction(2 * i + 1, 2) / hy  # node coordinate of voxel centre i
        jj = pos.numerator // pos.denominator
        frac = pos - jj
        assert j0[i] == jj and j0f[i] == jj
        assert Fraction(int(r[i]), den) == frac
        assert w1[i] == float(frac) and w0[i] == float(1 - frac)
        # float32 weights: nearest float32 to the exact rational
        for wf, exact in ((w1f[i], frac), (w0f[i], 1 - frac)):
            lo = np.nextafter(wf, np.float32(-1))
            hi = np.nextafter(wf, np.float32(2))
            err = abs(Fraction(float(wf)) - exact)
            assert err <= abs(Fraction(float(lo)) - exact)
            assert err <= abs(Fraction(float(hi)) - exact)
        assert 0 <= jj <= my - 2


@pytest.mark.parametrize("m", SIZES)
def test_index_map_exact_ratio2(m):
    _check_index_map(m, m // 2 + 1)


@pytest.mark.parametrize("m,my", [(32, 9), (64, 17), (100, 26), (30, 7), (9, 4), (12, 12)])
def test_index_map_exact_other_ratios(m, my):
    _check_index_map(m, my)


@pytest.mark.parametrize("m", [8, 16, 64])
def test_omega_ratio2_ranges_and_weights(m):
    my = m // 2 + 1
    idx, wt = O.omega_sets(m, my)
    for j in range(my):
        pairs = sorted((int(i), float(w)) for i, w in zip(idx[j], wt[j]) if w != 0.0)
        want = [(i, w) for i, w in zip(range(2 * j - 2, 2 * j + 2), (0.25, 0.75, 0.75, 0.25))
                if 0 <= i <= m - 1]
        assert pairs == want


def _interp_matrix(m, h, my):
    """Dense 1D interpolation matrix from numpy's np.interp of unit vectors."""
    X = np.arange(my) * (m * h / (my - 1))
    x = (np.arange(m) + 0.5) * h
    M = np.zeros((m, my))
    for j in range(my):
        e = np.zeros(my)
        e[j] = 1.0
        M[:, j] = np.interp(x, X, e)
    return M


@pytest.mark.parametrize("m,h,my", [((8, 8, 8), (1, 1, 1), (5, 5, 5)),
                                     ((8, 12, 6), (1.0, 0.5, 2.0), (5, 7, 4)),
                                     ((12, 8, 10), (1.0, 1.0, 1.0), (4, 3, 6))])
def test_P_equals_kronecker_of_np_interp(m, h, my):
    rng = np.random.default_rng(11)
    y = rng.standard_normal((3,) + my)
    Mx, My, Mz = (_interp_matrix(m[d], h[d], my[d]) for d in range(3))
    want = np.einsum("xi,yj,zk,cijk->cxyz", Mx, My, Mz, y)
    got = O.apply_P(y, m, my)
    assert np.max(np.abs(got - want)) < 1e-13
    # P^T is the transpose of the same dense operator
    z = rng.standard_normal((3,) + m)
    wantT = np.einsum("xi,yj,zk,cxyz->cijk", Mx, My, Mz, z)
    assert np.max(np.abs(O.apply_PT(z, m, my) - wantT)) < 1e-12


@pytest.mark.parametrize("m,h,my", [((16, 16, 16), (1, 1, 1), (9, 9, 9)),
                                     ((16, 24, 8), (0.7, 1.3, 2.0), (9, 13, 5)),
                                     ((20, 16, 12), (1, 1, 1), (6, 5, 4))])
def test_P_reproduces_constants_and_affine(m, h, my):
    X = O.identity(m, h, my)
    ones = np.ones((1,) + my)
    assert np.max(np.abs(O.apply_P(ones, m, my) - 1.0)) < 1e-15
    x = np.stack(np.meshgrid(*[O.image_coords_1d(m[d], h[d]) for d in range(3)],
                             indexing="ij"))
    assert np.max(np.abs(O.apply_P(X, m, my) - x)) < 1e-12 * max(m) * max(h)
    # affine map A X + b is reproduced too
    A = np.array([[1.1, 0.2, -0.3], [0.05, 0.9, 0.1], [0.0, -0.2, 1.2]])
    b = np.array([0.3, -1.0, 2.0])
    yA = np.einsum("cd,d...->c...", A, X) + b[:, None, None, None]
    xA = np.einsum("cd,d...->c...", A, x) + b[:, None, None, None]
    assert np.max(np.abs(O.apply_P(yA, m, my) - xA)) < 1e-11


@pytest.mark.parametrize("m,my", [((16, 12, 20), (9, 7, 11)), ((32, 32, 32), (17, 17, 17)),
                                  ((24, 16, 8), (7, 5, 3))])
def test_P_adjoint_identity(m, my):
    rng = np.random.default_rng(5)
    y = rng.standard_normal((3,) + my)
    z = rng.standard_normal((3,) + m)
    lhs = float(np.vdot(O.apply_P(y, m, my), z))
    rhs = float(np.vdot(y, O.apply_PT(z, m, my)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_PT_of_ones_closed_form():
    # ratio 2: an interior node collects 1/4+3/4+3/4+1/4 = 2 per axis, an end
    # node 3/4+1/4 = 1 per axis -> 8, 4, 2, 1 in 3D
    m = (16, 16, 16)
    my = (9, 9, 9)
    out = O.apply_PT(np.ones((1,) + m), m, my)[0]
    per_axis = np.array([1.0] + [2.0] * 7 + [1.0])
    want = per_axis[:, None, None] * per_axis[None, :, None] * per_axis[None, None, :]
    assert np.array_equal(out, want)


def test_downsample_equals_reshape_mean():
    rng = np.random.default_rng(3)
    u = (rng.standard_normal((16, 12, 8)) * 300.0).astype(np.float32)
    want = u.astype(np.float64).reshape(8, 2, 6, 2, 4, 2).mean(axis=(1, 3, 5)).astype(np.float32)
    assert np.array_equal(O.downsample(u), want)


def test_pyramid_levels_and_shapes():
    rng = np.random.default_rng(4)
    R = rng.standard_normal((32, 16, 64)).astype(np.float32)
    Rs, Ts = O.pyramid(R, R, 3)
    assert [a.shape for a in Rs] == [(32, 16, 64), (16, 8, 32), (8, 4, 16)]
    assert all(a.dtype == np.float32 for a in Rs)
    sh = O.level_shapes((32, 16, 64), (1.0, 2.0, 0.5), 3)
    assert sh[2] == ((8, 4, 16), (4.0, 8.0, 2.0), (5, 3, 9))


@pytest.mark.parametrize("mc", [(5, 5, 5), (9, 7, 4)])
def test_prolongate_matches_np_interp_and_identity(mc):
    rng = np.random.default_rng(9)
    yc = rng.standard_normal((3,) + mc)
    got = O.prolongate(yc)
    mf = tuple(2 * n - 1 for n in mc)
    # separable np.interp on node indices: fine node k sits at coarse index k/2
    want = yc
    for axis in (1, 2, 3):
        n = want.shape[axis]
        xf = np.arange(2 * n - 1) / 2.0
        want = np.apply_along_axis(lambda v: np.interp(xf, np.arange(n), v), axis, want)
    assert got.shape == (3,) + mf
    assert np.max(np.abs(got - want)) < 1e-14
    # the coarse identity prolongates to the fine identity exactly
    m = tuple(4 * (n - 1) for n in mc)
    h = (1.0, 2.0, 0.5)
    Xc = O.identity(tuple(v // 2 for v in m), tuple(2 * v for v in h), mc)
    Xf = O.identity(m, h, mf)
    assert np.array_equal(O.prolongate(Xc), Xf)


def test_level_shapes_with_node_counts():
    """Node counts given at level 0 halve their cells per level; with
    m/ratio + 1 they reproduce the ratio rule; on a general grid the coarse
    identity still prolongates to the fine identity (node positions j h^y of
    the halved grid are the even fine nodes)."""
    m, h = (48, 64, 96), (1.0, 0.5, 2.0)
    assert O.level_shapes(m, h, 3, 2, my0=(25, 33, 49)) == O.level_shapes(m, h, 3, 2)
    sh = O.level_shapes(m, h, 3, my0=(17, 33, 25))  # ratios 3, 2, 4
    assert [s[2] for s in sh] == [(17, 33, 25), (9, 17, 13), (5, 9, 7)]
    # non-integer ratios: 64 / 26 and 40 / 18 image cells per node cell
    sh = O.level_shapes((64, 40, 64), (1.0, 1.0, 1.0), 2, my0=(27, 19, 33))
    for lev in (1,):
        (mc, hc, nc), (mf, hf, nf) = sh[lev], sh[lev - 1]
        Xc, Xf = O.identity(mc, hc, nc), O.identity(mf, hf, nf)
        assert np.allclose(O.prolongate(Xc), Xf, rtol=0, atol=1e-12)
    # brute force: P of the identity is the cell centres on these grids too
    (mf, hf, nf) = sh[0]
    yh = O.apply_P(O.identity(mf, hf, nf), mf, nf)
    for d in range(3):
        c = (np.arange(mf[d]) + 0.5) * hf[d]
        shp = [1, 1, 1]
        shp[d] = mf[d]
        assert np.max(np.abs(yh[d] - c.reshape(shp))) < 1e-12
