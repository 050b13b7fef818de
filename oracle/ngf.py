"""Template warp, central differences and the NGF distance with its
derivatives (FP64).

Sec. 2.2, paragraph "Distance measure and gradient computation", Eq. 2:

    D(y) = (hbar / 2) * sum_i ( 1 - r_i^2 ),
    r_i  = ( <grad T_i(P y), grad R_i> + tau rho ) / ( ||grad T_i||_tau ||grad R_i||_rho ),
    ||v||_eps = sqrt(<v, v> + eps^2),  hbar = h_x h_y h_z.

Readings:

* "grad T_i(P(y))" is the finite-difference gradient of the warped template
  T_y = T(P y) on the image grid (discretise, then optimise), not the analytic
  gradient of T at y_hat.
* The differences are central with a replicated ghost cell at each end:
  (G u)[i] = (u[min(i+1, m-1)] - u[max(i-1, 0)]) / (2 h).
* The warp is trilinear with clamping at the domain edge (replicate), slope 0
  outside the domain; at an integer coordinate the cell to the right is used
  (right-sided derivative) except at the upper edge (left-sided).
* The gradient is assembled matrix-free by the chain rule (same paragraph):
  grad_y D = P^T diag(dT_y/dy_hat) G^T v with v = dD/d(grad T).
"""

from __future__ import annotations

import numpy as np


def warp(T: np.ndarray, h, yhat: np.ndarray):
    """Trilinear warp of T at the physical points y_hat (3, *m_out).

    Continuous index xi_d = y_hat_d / h_d - 1/2.  Outside [0, m_d - 1] the
    coordinate is clamped to the edge and the slope mask s_d is 0.  The cell
    is i0_d = min(floor(xi_d), m_d - 2) and the fraction f_d = xi_d - i0_d.

    Returns T_y, dT_y/dy_hat (3, ...) and the cell data (i0, f) used by the
    template adjoint.
    """
    m = T.shape
    i0, f, s = [], [], []
    for d in range(3):
        xi = yhat[d] / h[d] - 0.5
        sd = ((xi >= 0.0) & (xi <= m[d] - 1)).astype(np.float64)
        xi = np.clip(xi, 0.0, m[d] - 1.0)
        i0d = np.minimum(np.floor(xi), m[d] - 2).astype(np.int64)
        i0.append(i0d)
        f.append(xi - i0d)
        s.append(sd)
    Ty = np.zeros(yhat.shape[1:], dtype=np.float64)
    dT = np.zeros((3,) + yhat.shape[1:], dtype=np.float64)
    Tv = T.astype(np.float64)
    for a in (0, 1):
        wa = f[0] if a else 1.0 - f[0]
        da = 1.0 if a else -1.0
        for b in (0, 1):
            wb = f[1] if b else 1.0 - f[1]
            db = 1.0 if b else -1.0
            for c in (0, 1):
                wc = f[2] if c else 1.0 - f[2]
                dc = 1.0 if c else -1.0
                val = Tv[i0[0] + a, i0[1] + b, i0[2] + c]
                Ty += wa * wb * wc * val
                dT[0] += da * wb * wc * val
                dT[1] += wa * db * wc * val
                dT[2] += wa * wb * dc * val
    for d in range(3):
        dT[d] *= s[d] / h[d]
    return Ty, dT, (i0, f)


def warp_T_adjoint(e: np.ndarray, m, cells) -> np.ndarray:
    """Derivative with respect to the template voxels: for a sensitivity e on
    the output points, dD/dT[k] = sum_i e[i] W(i -> k), where W(i -> k) is the
    trilinear weight voxel k receives in the (clamped) warp of point i.
    Written as a plain scatter-add of every corner of every point."""
    i0, f = cells
    out = np.zeros(m, dtype=np.float64)
    for a in (0, 1):
        wa = f[0] if a else 1.0 - f[0]
        for b in (0, 1):
            wb = f[1] if b else 1.0 - f[1]
            for c in (0, 1):
                wc = f[2] if c else 1.0 - f[2]
                np.add.at(out, (i0[0] + a, i0[1] + b, i0[2] + c), wa * wb * wc * e)
    return out


def cdiff(u: np.ndarray, h: float, axis: int) -> np.ndarray:
    """Central difference along one axis with a replicated ghost cell."""
    m = u.shape[axis]
    k = np.arange(m)
    ip = np.minimum(k + 1, m - 1)
    im = np.maximum(k - 1, 0)
    return (np.take(u, ip, axis=axis) - np.take(u, im, axis=axis)) / (2.0 * h)


def cdiff_adj(w: np.ndarray, h: float, axis: int) -> np.ndarray:
    """Transpose of ``cdiff`` along one axis (m >= 3):

        (G^T w)[k] = (w[k-1] - w[k+1]) / (2h)     for 1 <= k <= m-2,
        (G^T w)[0] = -(w[0] + w[1]) / (2h),
        (G^T w)[m-1] = (w[m-2] + w[m-1]) / (2h).
    """
    m = w.shape[axis]
    wm = np.moveaxis(w, axis, 0)
    out = np.zeros_like(wm, dtype=np.float64)
    out[1:m - 1] = (wm[0:m - 2] - wm[2:m]) / (2.0 * h)
    out[0] = -(wm[0] + wm[1]) / (2.0 * h)
    out[m - 1] = (wm[m - 2] + wm[m - 1]) / (2.0 * h)
    return np.moveaxis(out, 0, axis)


def ngf_terms(gT, gR, tau: float, rho: float):
    """Per-point quantities of Eq. 2: r, ||grad T||_tau, ||grad R||_rho and the
    smoothed inner product c = <grad T, grad R> + tau rho."""
    nT = np.sqrt(gT[0] ** 2 + gT[1] ** 2 + gT[2] ** 2 + tau * tau)
    nR = np.sqrt(gR[0] ** 2 + gR[1] ** 2 + gR[2] ** 2 + rho * rho)
    c = gT[0] * gR[0] + gT[1] * gR[1] + gT[2] * gR[2] + tau * rho
    r = c / (nT * nR)
    return r, nT, nR, c


def ngf_dgT(gT, gR, tau: float, rho: float, hbar: float) -> np.ndarray:
    """Derivative of D with respect to the template gradient at each point:
    v = -hbar r / (nT nR) * (grad R - (c / nT^2) grad T)."""
    r, nT, nR, c = ngf_terms(gT, gR, tau, rho)
    k = -hbar * r / (nT * nR)
    return np.stack([k * (gR[d] - (c / (nT * nT)) * gT[d]) for d in range(3)])
