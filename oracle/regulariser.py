"""Curvature regulariser (FP64).

Sec. 2.1 names the curvature regulariser, which penalises the squared
Laplacian of every deformation component.  Readings (the discretisation is not
given in the paper):

* It acts on the displacement u = y - X (X = node positions), which equals the
  Laplacian of y at interior nodes and does not penalise the identity at the
  boundary.
* Seven-point Laplacian with a replicated ghost node (Neumann):
  (A u)[j] = sum_d (u[j + e_d]* - 2 u[j] + u[j - e_d]*) / (h^y_d)^2,
  where * clamps the index to the grid.
* Midpoint quadrature with node volume hbar^y = h^y_x h^y_y h^y_z:
  S = (hbar^y / 2) sum_c sum_j (A u_c)[j]^2, so grad S = hbar^y A^T A u_c,
  and A is symmetric.
"""

from __future__ import annotations

import numpy as np


def laplacian(u: np.ndarray, hy) -> np.ndarray:
    """Seven-point Laplacian of a scalar node field with replicated ghosts."""
    out = np.zeros_like(u, dtype=np.float64)
    for d in range(3):
        m = u.shape[d]
        k = np.arange(m)
        up = np.take(u, np.minimum(k + 1, m - 1), axis=d)
        um = np.take(u, np.maximum(k - 1, 0), axis=d)
        out += (up - 2.0 * u + um) / (hy[d] * hy[d])
    return out


def curvature(u: np.ndarray, hy):
    """S(u) and grad S for a displacement u of shape (3, *my)."""
    hbar_y = float(hy[0] * hy[1] * hy[2])
    Au = np.stack([laplacian(u[c], hy) for c in range(3)])
    S = 0.5 * hbar_y * float(np.sum(Au * Au))
    grad = hbar_y * np.stack([laplacian(Au[c], hy) for c in range(3)])
    return S, grad
