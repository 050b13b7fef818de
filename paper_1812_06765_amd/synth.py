"""Seeded synthetic registration inputs.

This module is shared by the oracle tests, the GPU tests and the benchmark.  It
holds only input generation: analytic phantoms sampled at voxel centres, smooth
random displacement fields, and the ground-truth inverse of a displacement.  It
contains none of the registration method's arithmetic (no grid conversion, no
interpolation of images, no distance or regulariser terms), so neither side of a
parity test can inherit a mistake from it.

The workloads stand in for the paper's data (Section 3: follow-up thorax-abdomen
CT at about 256^3, lung 4DCT); neither data set is available, so every input
here is a seeded phantom of the same shape, spacing and intensity range.

Coordinates: arrays are indexed ``[x][y][z]`` with z fastest.  A point is given
in voxel units of its grid, where voxel ``i`` has its centre at ``i + 0.5``.
All draws use numpy's PCG64 generator with the seed passed in; the order of the
draws is fixed by the code below.
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Pair",
    "voxel_centres",
    "SinusoidField",
    "BSplineField",
    "blob_phantom_pair",
    "ct_phantom_pair",
    "ct_phantom_pair_slabs",
    "ct_phantom_value",
    "invert_displacement",
    "smooth_node_perturbation",
    "batch_shapes",
    "sha256",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sha256(a: np.ndarray) -> str:
    """SHA-256 of an array's bytes (C order), to freeze generated inputs."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def voxel_centres(m) -> np.ndarray:
    """(3, mx, my, mz) float64 voxel-centre positions in voxel units."""
    ax = [np.arange(n, dtype=np.float64) + 0.5 for n in m]
    g = np.meshgrid(*ax, indexing="ij")
    return np.stack(g)


# ---------------------------------------------------------------------------
# smooth displacement fields (continuous: evaluable at arbitrary points)
# ---------------------------------------------------------------------------


class SinusoidField:
    """u_c(p) = A * sum_k sin(2*pi*<f_ck, p>/m + phi_ck), three terms per component.

    ``p`` is in voxel units of a grid of extent ``m``; frequencies are in cycles
    per extent, drawn from U[0.5, 1.5]^3; phases from U[0, 2 pi).  ``A`` is set
    so that the largest Euclidean norm of u over the grid's voxel centres equals
    ``max_amp`` voxels.
    """

    def __init__(self, m, max_amp: float, seed: int, terms: int = 3):
        rng = _rng(seed)
        self.m = np.asarray(m, dtype=np.float64)
        self.freq = rng.uniform(0.5, 1.5, size=(3, terms, 3))
        self.phase = rng.uniform(0.0, 2.0 * np.pi, size=(3, terms))
        self.amp = 1.0
        raw = self(voxel_centres(m))
        self.amp = max_amp / float(np.sqrt((raw**2).sum(0)).max())

    def __call__(self, p: np.ndarray) -> np.ndarray:
        q = p / self.m.reshape((3,) + (1,) * (p.ndim - 1))
        out = np.zeros_like(p, dtype=np.float64)
        for c in range(3):
            for k in range(self.freq.shape[1]):
                arg = sum(self.freq[c, k, d] * q[d] for d in range(3))
                out[c] += np.sin(2.0 * np.pi * arg + self.phase[c, k])
        return self.amp * out


def _cubic_bspline(t: np.ndarray) -> np.ndarray:
    """Uniform cubic B-spline kernel, support (-2, 2)."""
    a = np.abs(t)
    out = np.zeros_like(a)
    m1 = a < 1.0
    m2 = (a >= 1.0) & (a < 2.0)
    out[m1] = (4.0 - 6.0 * a[m1] ** 2 + 3.0 * a[m1] ** 3) / 6.0
    out[m2] = (2.0 - a[m2]) ** 3 / 6.0
    return out


class BSplineField:
    """Cubic B-spline displacement with i.i.d. N(0,1) control coefficients.

    Control points sit every ``spacing`` voxels, starting one spacing before
    the grid and ending at least one spacing after it, so the field is smooth
    up to the boundary.  The coefficients are scaled so that the largest
    Euclidean norm over the grid's voxel centres equals ``max_amp`` voxels.
    """

    def __init__(self, m, spacing: float, max_amp: float, seed: int):
        rng = _rng(seed)
        self.m = tuple(int(v) for v in m)
        self.spacing = float(spacing)
        self.ncp = [int(np.ceil(n / self.spacing)) + 4 for n in self.m]
        self.coef = rng.standard_normal(size=(3,) + tuple(self.ncp))
        self.scale = 1.0
        peak, step = 0.0, max(1, (1 << 24) // (self.m[1] * self.m[2]))
        for x0 in range(0, self.m[0], step):  # in slabs: bounded memory
            raw = self.on_grid(x0, min(self.m[0], x0 + step))
            peak = max(peak, float(np.sqrt((raw**2).sum(0)).max()))
        self.scale = max_amp / peak

    def _basis(self, d: int, p: np.ndarray) -> np.ndarray:
        # control point k sits at (k - 1) * spacing
        k = np.arange(self.ncp[d], dtype=np.float64)
        return _cubic_bspline(p[..., None] / self.spacing - (k - 1.0))

    def on_grid(self, x0: int = 0, x1: int | None = None) -> np.ndarray:
        """Field at the voxel centres of the grid, (3, mx, my, mz), or of the
        x-slab [x0, x1) of it."""
        x1 = self.m[0] if x1 is None else x1
        bx = self._basis(0, np.arange(x0, x1, dtype=np.float64) + 0.5)
        by, bz = (self._basis(d, np.arange(self.m[d], dtype=np.float64) + 0.5) for d in (1, 2))
        out = np.einsum("cijk,xi,yj,zk->cxyz", self.coef, bx, by, bz, optimize=True)
        return np.ascontiguousarray(self.scale * out)

    def __call__(self, p: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
        """Field at arbitrary points p (3, ...).  A point sees the 4 x 4 x 4
        control points whose basis functions cover it; outside the control
        lattice the missing ones contribute nothing."""
        shp = p.shape[1:]
        flat = p.reshape(3, -1)
        out = np.empty((3, flat.shape[1]))
        for a in range(0, flat.shape[1], chunk):
            q = flat[:, a:a + chunk]
            ks, ws = [], []
            for d in range(3):
                t = q[d] / self.spacing
                k = np.floor(t).astype(np.int64)[:, None] + np.arange(4)  # (n, 4)
                w = _cubic_bspline(t[:, None] - (k - 1.0))  # control point k sits at (k-1) s
                ok = (k >= 0) & (k < self.ncp[d])
                ks.append(np.clip(k, 0, self.ncp[d] - 1))
                ws.append(np.where(ok, w, 0.0))
            c = self.coef[:, ks[0][:, :, None, None], ks[1][:, None, :, None],
                          ks[2][:, None, None, :]]  # (3, n, 4, 4, 4)
            out[:, a:a + chunk] = np.einsum("cnijk,ni,nj,nk->cn", c, ws[0], ws[1], ws[2],
                                            optimize=True)
        return (self.scale * out).reshape((3,) + shp)


def invert_displacement(field, points: np.ndarray, iters: int = 60) -> np.ndarray:
    """Solve z + u(z) = x for z by the fixed point z <- x - u(z).

    Used for the ground-truth correspondence of a pair built as
    T(x) = R(x + u(x)): the deformation that maps the template back onto the
    reference is y(x) = z(x).  Converges for smooth u with |grad u| < 1.
    """
    z = points.copy()
    for _ in range(iters):
        z = points - field(z)
    return z


# ---------------------------------------------------------------------------
# phantoms
# ---------------------------------------------------------------------------


@dataclass
class Pair:
    R: np.ndarray  # float32 (mx, my, mz)
    T: np.ndarray  # float32 (mx, my, mz)
    field: object  # displacement used to build T, in voxel units
    m: tuple
    h: tuple
    seeds: tuple


EDGE_WIDTH = 1.0  # voxels; smooth edges keep the sampled phantom band-limited


def _soft(dist_vox):
    """Smooth indicator of a region from an (approximate) signed distance in
    voxels, positive inside: a tanh edge of width EDGE_WIDTH.  A hard 0/1
    edge would alias differently in R and T and make the generating
    displacement a poor minimiser of any image distance."""
    return 0.5 * (1.0 + np.tanh(dist_vox / EDGE_WIDTH))


def _ellipsoid(q, centre, semi, m):
    """Smooth ellipsoid indicator; q in fractions of the extent, semi-axes in
    fractions; the signed distance is approximated by (1 - radius) times the
    shortest semi-axis in voxels."""
    rad = np.sqrt(sum(((q[d] - centre[d]) / semi[d]) ** 2 for d in range(3)))
    return _soft((1.0 - rad) * min(semi[d] * m[d] for d in range(3)))


def _blob_phantom_value(p, m, blobs):
    q = p / np.asarray(m, dtype=np.float64).reshape((3,) + (1,) * (p.ndim - 1))
    val = _ellipsoid(q, (0.5, 0.5, 0.5), (0.35, 0.28, 0.22), m)
    for c, sig, amp in blobs:
        r2 = sum((p[d] - c[d]) ** 2 for d in range(3))
        val = val + amp * np.exp(-0.5 * r2 / sig**2)
    return val


def blob_phantom_pair(m=(32, 32, 32), h=(1.0, 1.0, 1.0), seed_R=1, seed_u=2,
                      max_disp=2.0, noise=0.01) -> Pair:
    """Ellipsoid of value 1 with six Gaussian blobs, plus Gaussian noise.

    The ellipsoid has semi-axes (0.35, 0.28, 0.22) of the extent and a smooth
    edge about one voxel wide.  Blob centres
    are uniform inside it, sigma ~ U[2, 5] voxels, amplitude +-0.5.  T is the
    same analytic phantom evaluated at x + u(x), with u a sum of three random
    sinusoids per component of ``max_disp`` voxels peak norm, and independent
    noise.
    """
    rng = _rng(seed_R)
    mm = np.asarray(m, dtype=np.float64)
    blobs = []
    while len(blobs) < 6:
        c = rng.uniform(0.0, 1.0, size=3)
        if (((c - 0.5) / np.array([0.35, 0.28, 0.22])) ** 2).sum() <= 1.0:
            sig = rng.uniform(2.0, 5.0)
            amp = 0.5 if rng.uniform() < 0.5 else -0.5
            blobs.append((c * mm, sig, amp))
    x = voxel_centres(m)
    R = _blob_phantom_value(x, m, blobs) + rng.normal(0.0, noise, size=tuple(m))
    field = SinusoidField(m, max_disp, seed_u)
    T = _blob_phantom_value(x + field(x), m, blobs) + rng.normal(0.0, noise, size=tuple(m))
    return Pair(np.ascontiguousarray(R, dtype=np.float32),
                np.ascontiguousarray(T, dtype=np.float32), field, tuple(m), tuple(h),
                (seed_R, seed_u))


def ct_phantom_value(p: np.ndarray, m) -> np.ndarray:
    """CT-like thorax phantom in Hounsfield units at points p (voxel units).

    Every region has a smooth edge about one voxel wide.  Air -1000 HU; body ellipsoid 40 HU with semi-axes (0.42, 0.32, 0.45) of
    the extent; two lung ellipsoids -850 HU centred at (0.5 +- 0.18, 0.47, 0.5)
    with semi-axes (0.14, 0.18, 0.30); a spine cylinder of 700 HU along z at
    (0.5, 0.72) of radius 0.06 * min(mx, my) voxels, clipped to the body.
    """
    mm = np.asarray(m, dtype=np.float64).reshape((3,) + (1,) * (p.ndim - 1))
    q = p / mm
    body = _ellipsoid(q, (0.5, 0.5, 0.5), (0.42, 0.32, 0.45), m)
    val = -1000.0 + 1040.0 * body
    for sx in (-0.18, 0.18):
        lung = _ellipsoid(q, (0.5 + sx, 0.47, 0.5), (0.14, 0.18, 0.30), m)
        val = val + (-850.0 - 40.0) * lung * body
    rad = 0.06 * min(m[0], m[1])
    spine = _soft(rad - np.sqrt((p[0] - 0.5 * m[0]) ** 2 + (p[1] - 0.72 * m[1]) ** 2))
    val = val + (700.0 - 40.0) * spine * body
    return val


def ct_phantom_pair_slabs(m, seed_R=5, seed_u=6, max_disp=6.0, cp_spacing=16.0, noise=20.0,
                          slab=32, progress=None, workers=8):
    """The CT pair recipe of ``ct_phantom_pair`` generated in x-slabs of
    ``slab`` planes, for volumes too large to form in one piece (bounded
    memory, a progress callback per slab).  The noise of slab k is drawn
    from PCG64 seeded with (seed_R, k) for R and (seed_R, k, 1) for T, so the
    values differ from ``ct_phantom_pair`` of the same seeds; the recipe is
    the same."""
    m = tuple(int(v) for v in m)
    field = BSplineField(m, cp_spacing, max_disp, seed_u)
    R = np.empty(m, dtype=np.float32)
    T = np.empty(m, dtype=np.float32)
    ax = [np.arange(n, dtype=np.float64) + 0.5 for n in m]

    def one(k):
        x0 = k * slab
        x1 = min(m[0], x0 + slab)
        x = np.stack(np.meshgrid(ax[0][x0:x1], ax[1], ax[2], indexing="ij"))
        shp = (x1 - x0, m[1], m[2])
        rng_r = np.random.Generator(np.random.PCG64([seed_R, k]))
        rng_t = np.random.Generator(np.random.PCG64([seed_R, k, 1]))
        R[x0:x1] = ct_phantom_value(x, m) + rng_r.normal(0.0, noise, size=shp)
        T[x0:x1] = ct_phantom_value(x + field.on_grid(x0, x1), m) + rng_t.normal(0.0, noise,
                                                                                  size=shp)
        return x1

    from concurrent.futures import ThreadPoolExecutor
    nslab = (m[0] + slab - 1) // slab
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        done = 0
        for _ in ex.map(one, range(nslab)):
            done += 1
            if progress is not None:
                progress(min(m[0], done * slab), m[0])
    return Pair(R, T, field, m, (1.0, 1.0, 1.0), (seed_R, seed_u))


def ct_phantom_pair(m=(128, 128, 128), h=(1.0, 1.0, 1.0), seed_R=3, seed_u=4,
                    max_disp=6.0, cp_spacing=16.0, noise=20.0) -> Pair:
    """CT-like pair: R is the phantom plus N(0, noise) HU; T(x) = phantom(x + u(x))
    plus independent noise, with u a cubic B-spline field of control spacing
    ``cp_spacing`` voxels and ``max_disp`` voxels peak norm."""
    rng = _rng(seed_R)
    x = voxel_centres(m)
    R = ct_phantom_value(x, m) + rng.normal(0.0, noise, size=tuple(m))
    field = BSplineField(m, cp_spacing, max_disp, seed_u)
    T = ct_phantom_value(x + field.on_grid(), m) + rng.normal(0.0, noise, size=tuple(m))
    return Pair(np.ascontiguousarray(R, dtype=np.float32),
                np.ascontiguousarray(T, dtype=np.float32), field, tuple(m), tuple(h),
                (seed_R, seed_u))


def smooth_node_perturbation(my, spacing_nodes: float, max_amp: float, seed: int) -> np.ndarray:
    """Smooth random field on a node grid of shape ``my``: (3, *my) float64.

    ``max_amp`` is the peak Euclidean norm in the caller's units; the caller
    adds it to the identity deformation (node positions) to get a perturbed y.
    The field is a cubic B-spline evaluated at node indices (not voxel centres).
    """
    f = BSplineField(my, spacing_nodes, 1.0, seed)
    nodes = np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in my],
                                 indexing="ij"))
    v = f(nodes)
    return v * (max_amp / float(np.sqrt((v**2).sum(0)).max()))


def batch_shapes(count=64, choices=(96, 128, 160, 192, 256), seed=8):
    """Uneven batch shapes: each axis drawn uniformly and independently."""
    rng = _rng(seed)
    return [tuple(int(c) for c in rng.choice(choices, size=3)) for _ in range(count)]
