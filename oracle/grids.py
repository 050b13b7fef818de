"""Grids, grid conversion P and its adjoint, pyramid and prolongation (FP64).

Readings (the paper gives grid dimensions only, Sec. 2.1 and the paragraph
"Grid conversion" of Sec. 2.2):

* The image grid is cell-centred: voxel i along an axis of m cells and spacing
  h has its centre at (i + 1/2) h; the domain is [0, m h].
* The deformation grid is nodal over the same domain: node j of m^y nodes sits
  at j * h^y with h^y = m h / (m^y - 1).  With m^y = m/2 + 1 this gives
  h^y = 2 h and the dyadic trilinear weights 1/4, 3/4.
* y holds positions (a transformation), so the template is sampled at P y
  (Sec. 2.1, Eq. 1: T(P(y))); the identity deformation is y = node positions.

Arrays are indexed [x][y][z] with z fastest; a deformation is stored as
(3, m^y_x, m^y_y, m^y_z), component-major.
"""

from __future__ import annotations

import numpy as np


def image_coords_1d(m: int, h: float) -> np.ndarray:
    """Cell-centred image coordinates along one axis: (i + 1/2) h."""
    return (np.arange(m, dtype=np.float64) + 0.5) * h


def node_spacing(m: int, h: float, my: int) -> float:
    """Deformation-grid spacing h^y = m h / (m^y - 1) (nodal grid over [0, m h])."""
    return m * h / (my - 1)


def node_coords_1d(m: int, h: float, my: int) -> np.ndarray:
    """Nodal deformation-grid coordinates along one axis: j h^y."""
    return np.arange(my, dtype=np.float64) * node_spacing(m, h, my)


def identity(m, h, my) -> np.ndarray:
    """Identity deformation y = X: the node positions, shape (3, *my)."""
    ax = [node_coords_1d(m[d], h[d], my[d]) for d in range(3)]
    return np.stack(np.meshgrid(*ax, indexing="ij"))


def index_map(m: int, my: int):
    """Per-axis index map of the grid conversion (Sec. 2.2, "Grid conversion":
    the index sets and weights are fixed beforehand, separately per dimension).

    Image point i lies at (i + 1/2) h = (j0 + w1) h^y, i.e. at node coordinate
    num/den with num = (2 i + 1)(m^y - 1) and den = 2 m.  In exact integers:
    j0 = num div den, r = num mod den, and the two trilinear weights along this
    axis are w0 = (den - r)/den (node j0) and w1 = r/den (node j0 + 1).

    Returns (j0 int64, r int64, den int, w0 float64, w1 float64).
    """
    i = np.arange(m, dtype=np.int64)
    num = (2 * i + 1) * (my - 1)
    den = 2 * m
    j0 = num // den
    r = num - j0 * den
    w1 = r.astype(np.float64) / den
    w0 = (den - r).astype(np.float64) / den
    return j0, r, den, w0, w1


def index_map_f32(m: int, my: int):
    """The index map in the storage precision of the GPU path: int32 node index
    and float32 weights rounded to nearest from the exact rationals.

    float32(float64(r/den)) is correctly rounded here: r/den is a ratio of
    integers below 2^24, and rounding first to 53 bits then to 24 bits cannot
    create a double-rounding error when 53 >= 2*24 + 2 (Figueroa, 1995).
    """
    j0, r, den, w0, w1 = index_map(m, my)
    return j0.astype(np.int32), w0.astype(np.float32), w1.astype(np.float32)


def omega_sets(m: int, my: int):
    """Index sets Omega(j) and weights omega of Eq. 3, for one axis.

    Omega(j) = { i : j0(i) = j } with weight w0(i), together with
    { i : j0(i) + 1 = j } with weight w1(i): the image points whose
    interpolation uses node j.  Built by scanning every image point (brute
    force).  Returned padded to a common length with (index 0, weight 0).
    """
    j0, _, _, w0, w1 = index_map(m, my)
    lists = [[] for _ in range(my)]
    for i in range(m):
        lists[j0[i]].append((i, w0[i]))
        lists[j0[i] + 1].append((i, w1[i]))
    k = max(len(v) for v in lists)
    idx = np.zeros((my, k), dtype=np.int64)
    wt = np.zeros((my, k), dtype=np.float64)
    for j, v in enumerate(lists):
        for n, (i, w) in enumerate(v):
            idx[j, n] = i
            wt[j, n] = w
    return idx, wt


def apply_P(y: np.ndarray, m, my) -> np.ndarray:
    """Grid conversion y_hat = P y (Sec. 2.1 and Sec. 2.2, "Grid conversion"):
    trilinear interpolation of each component from the 8 surrounding nodes,

        y_hat[i] = sum_{a,b,c in {0,1}} W_x^a W_y^b W_z^c y[j0_x + a, j0_y + b, j0_z + c]

    with W^0 = w0 and W^1 = w1 of the per-axis index maps.
    y: (C, *my) -> (C, *m).
    """
    (jx, _, _, w0x, w1x), (jy, _, _, w0y, w1y), (jz, _, _, w0z, w1z) = (
        index_map(m[d], my[d]) for d in range(3))
    out = np.zeros((y.shape[0],) + tuple(m), dtype=np.float64)
    for a, wx in ((0, w0x), (1, w1x)):
        for b, wy in ((0, w0y), (1, w1y)):
            for c, wz in ((0, w0z), (1, w1z)):
                w = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
                out += w * y[:, (jx + a)[:, None, None], (jy + b)[None, :, None],
                             (jz + c)[None, None, :]]
    return out


def apply_PT(z: np.ndarray, m, my) -> np.ndarray:
    """Adjoint grid conversion, Eq. 3: for every deformation node j,

        (P^T z)[j] = sum_{i_x in Omega_x(j_x)} sum_{i_y in Omega_y(j_y)}
                     sum_{i_z in Omega_z(j_z)} omega_x omega_y omega_z z[i_x, i_y, i_z]

    one node at a time (gather form, free of write conflicts).
    z: (C, *m) -> (C, *my).
    """
    (ix, wx), (iy, wy), (iz, wz) = (omega_sets(m[d], my[d]) for d in range(3))
    out = np.zeros((z.shape[0],) + tuple(my), dtype=np.float64)
    for kx in range(ix.shape[1]):
        for ky in range(iy.shape[1]):
            for kz in range(iz.shape[1]):
                w = (wx[:, kx][:, None, None] * wy[:, ky][None, :, None]
                     * wz[:, kz][None, None, :])
                out += w * z[:, ix[:, kx][:, None, None], iy[:, ky][None, :, None],
                             iz[:, kz][None, None, :]]
    return out


def downsample(u: np.ndarray) -> np.ndarray:
    """One pyramid step (Sec. 2.2, "Generating the multi-level pyramid"; the
    filter is not stated, read as the 2x2x2 box mean).

    Coarse voxel I is the mean of its 8 children 2I + (dx, dy, dz), summed in
    float64 in the fixed order ((000+001)+(010+011)) + ((100+101)+(110+111)),
    scaled by 1/8 and rounded once to float32.
    """
    v = u.astype(np.float64)

    def c(dx, dy, dz):
        return v[dx::2, dy::2, dz::2]

    s = ((c(0, 0, 0) + c(0, 0, 1)) + (c(0, 1, 0) + c(0, 1, 1))) + \
        ((c(1, 0, 0) + c(1, 0, 1)) + (c(1, 1, 0) + c(1, 1, 1)))
    return (0.125 * s).astype(np.float32)


def level_shapes(m, h, levels: int, ratio: int = 2, my0=None):
    """Image shape, spacing and deformation-grid shape of every pyramid level.

    Level 0 is the input; level l has m / 2^l cells and spacing h 2^l, and a
    deformation grid of m_l / ratio + 1 nodes per axis.  With ``my0`` (node
    counts of level 0 per axis) level l instead has (my0 - 1) / 2^l + 1
    nodes: every coarser level halves the node cells as it halves the image
    cells, so the nodal prolongation between levels stays exact (the
    multi-level scheme of Sec. 2.1 with the grid conversion of Sec. 2.2 on
    any grid).
    """
    out = []
    for lev in range(levels):
        ml = tuple(int(m[d]) >> lev for d in range(3))
        hl = tuple(float(h[d]) * (1 << lev) for d in range(3))
        if my0 is None:
            myl = tuple(ml[d] // ratio + 1 for d in range(3))
        else:
            myl = tuple(((int(my0[d]) - 1) >> lev) + 1 for d in range(3))
        out.append((ml, hl, myl))
    return out


def pyramid(R: np.ndarray, T: np.ndarray, levels: int):
    """Reference and template pyramids; each level is built from the stored
    float32 level above it."""
    Rs, Ts = [R.astype(np.float32)], [T.astype(np.float32)]
    for _ in range(1, levels):
        Rs.append(downsample(Rs[-1]))
        Ts.append(downsample(Ts[-1]))
    return Rs, Ts


def prolongate(yc: np.ndarray) -> np.ndarray:
    """Deformation prolongation between levels (implied by the multi-level
    scheme of Sec. 2.1, not described): along each axis fine node 2j takes
    coarse node j and fine node 2j+1 the mean of coarse nodes j and j+1; the
    3D operator is the tensor product of the three 1D operators.
    (C, a, b, c) -> (C, 2a-1, 2b-1, 2c-1)."""
    out = yc.astype(np.float64)
    for axis in (1, 2, 3):
        n = out.shape[axis]
        shp = list(out.shape)
        shp[axis] = 2 * n - 1
        fine = np.zeros(shp, dtype=np.float64)
        sl_even = [slice(None)] * 4
        sl_even[axis] = slice(0, 2 * n - 1, 2)
        fine[tuple(sl_even)] = out
        sl_odd = [slice(None)] * 4
        sl_odd[axis] = slice(1, 2 * n - 2, 2)
        lo = [slice(None)] * 4
        lo[axis] = slice(0, n - 1)
        hi = [slice(None)] * 4
        hi[axis] = slice(1, n)
        fine[tuple(sl_odd)] = 0.5 * (out[tuple(lo)] + out[tuple(hi)])
        out = fine
    return out
