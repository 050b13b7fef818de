"""Objective J = D + alpha S and its gradient (Sec. 2.1, Eq. 1), evaluated in
the three steps of Sec. 2.2, "Evaluating the objective function":

1. y_hat = P y (grid conversion to the image grid);
2. D and its derivative with respect to y_hat (Eq. 2 and the chain rule);
3. back to the deformation grid with P^T (Eq. 3).  Only the derivative is
   converted back; y_hat needs no conversion (reading of an ambiguous step).

Every sum is taken in float64.  Inputs given in float32 are widened exactly.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .regulariser import curvature
from .grids import apply_P, apply_PT, identity, node_spacing
from .ngf import cdiff, cdiff_adj, ngf_dgT, ngf_terms, warp, warp_T_adjoint


@dataclass
class Problem:
    """One registration level: images on an m grid with spacing h, and a
    deformation grid of my nodes spanning the same domain."""

    R: np.ndarray
    T: np.ndarray
    h: tuple
    my: tuple
    alpha: float
    tau: float
    rho: float

    @property
    def m(self):
        return tuple(self.R.shape)

    @property
    def hy(self):
        return tuple(node_spacing(self.m[d], self.h[d], self.my[d]) for d in range(3))

    def identity(self) -> np.ndarray:
        return identity(self.m, self.h, self.my)


def _forward(p: Problem, y: np.ndarray):
    y = np.asarray(y, dtype=np.float64)
    R = np.asarray(p.R, dtype=np.float64)
    T = np.asarray(p.T, dtype=np.float64)
    yhat = apply_P(y, p.m, p.my)
    Ty, dT, cells = warp(T, p.h, yhat)
    gT = [cdiff(Ty, p.h[d], d) for d in range(3)]
    gR = [cdiff(R, p.h[d], d) for d in range(3)]
    hbar = float(p.h[0] * p.h[1] * p.h[2])
    r, _, _, _ = ngf_terms(gT, gR, p.tau, p.rho)
    D = float(0.5 * hbar * np.sum(1.0 - r * r))
    v = ngf_dgT(gT, gR, p.tau, p.rho, hbar)
    e = sum(cdiff_adj(v[d], p.h[d], d) for d in range(3))
    return y, D, dT, e, cells


def eval_J_grad(p: Problem, y: np.ndarray):
    """J(y), grad_y J, and the parts (D, S).

    grad_y D = P^T( e * dT_y/dy_hat ) with e = sum_d G_d^T v_d;
    grad_y S = hbar^y A(A(y - X)).
    """
    y, D, dT, e, _ = _forward(p, y)
    dDdyhat = e[None] * dT
    gradD = apply_PT(dDdyhat, p.m, p.my)
    S, gradS = curvature(y - p.identity(), p.hy)
    J = D + p.alpha * S
    return J, gradD + p.alpha * gradS, (D, S)


def eval_J_grad_T(p: Problem, y: np.ndarray):
    """As ``eval_J_grad``, plus the derivative of J with respect to the
    template voxels: dJ/dT = dD/dT = W^T e (S does not depend on T)."""
    y, D, dT, e, cells = _forward(p, y)
    gradD = apply_PT(e[None] * dT, p.m, p.my)
    S, gradS = curvature(y - p.identity(), p.hy)
    gT = warp_T_adjoint(e, p.m, cells)
    return D + p.alpha * S, gradD + p.alpha * gradS, gT, (D, S)


def crossing_mask(p: Problem, y: np.ndarray, step: float) -> np.ndarray:
    """Flag the y entries whose finite-difference stencil of half-width
    ``step`` can move an affected warp coordinate across an integer (a kink of
    the trilinear warp), where a central difference does not approximate the
    one-sided derivative the method uses.  Returns a bool mask shaped like y.
    A node influences image points through weights <= 1, so a change of
    ``step`` in a node component moves xi of those points by at most step/h."""
    yhat = apply_P(np.asarray(y, dtype=np.float64), p.m, p.my)
    bad_img = np.zeros((3,) + p.m, dtype=bool)
    for d in range(3):
        xi = yhat[d] / p.h[d] - 0.5
        dist = np.abs(xi - np.round(xi))
        bad_img[d] = dist <= 2.0 * step / p.h[d]
        bad_img[d] |= (xi < 0.0) & (xi > -2.0 * step / p.h[d])
        bad_img[d] |= np.abs(xi - (p.m[d] - 1)) <= 2.0 * step / p.h[d]
    # a node component is affected if any image point in its support is flagged
    # on that component; the support is where P^T of the indicator is nonzero
    out = apply_PT(bad_img.astype(np.float64), p.m, p.my) > 0.0
    return out
