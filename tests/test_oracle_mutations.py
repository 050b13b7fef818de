"""Planted mistakes in the oracle must each fail at least one pin.

Each case patches one oracle function with a plausible slip (a dropped term,
a wrong sign or index, swapped operands) and runs the pins that should catch
it; the test passes only if a pin raises.  This shows the pins are sensitive
to the mistakes they are meant to exclude.
"""

import numpy as np
import pytest

import oracle as O
import oracle.regulariser as OC
import oracle.grids as OG
import oracle.lbfgs as OL
import oracle.ngf as ON
import oracle.objective as OO
import test_oracle_curvature as tc
import test_oracle_grids as tg
import test_oracle_lbfgs as tl
import test_oracle_ngf as tn
import test_oracle_objective as to


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _cdiff_adj_bad_end(w, h, axis):
    out = np.moveaxis(_orig["cdiff_adj"](w, h, axis), axis, 0).copy()
    out[0] = -out[0]
    return np.moveaxis(out, 0, axis)


def _ngf_terms_no_tau_rho(gT, gR, tau, rho):
    r, nT, nR, c = _orig["ngf_terms"](gT, gR, tau, rho)
    c2 = c - tau * rho
    return c2 / (nT * nR), nT, nR, c2


def _index_map_swapped(m, my):
    j0, r, den, w0, w1 = _orig["index_map"](m, my)
    return j0, r, den, w1, w0


def _omega_bad(m, my):
    idx, wt = _orig["omega_sets"](m, my)
    return idx, np.where(wt > 0, 0.5, 0.0)


def _laplacian_bad(u, hy):
    return _orig["laplacian"](u, (hy[0], hy[1], 1.0))


def _warp_bad(T, h, yhat):
    Ty, dT, cells = _orig["warp"](T, h, yhat)
    return Ty, dT[[1, 0, 2]], cells


def _two_loop_bad_gamma(self, g):
    s, t = self.S[-1], self.Tp[-1]
    d = _orig["two_loop"](self, g)
    gamma = float(np.vdot(s, t)) / float(np.vdot(t, t))
    return d / gamma**2


_orig = {
    "cdiff_adj": ON.cdiff_adj,
    "ngf_terms": ON.ngf_terms,
    "index_map": OG.index_map,
    "omega_sets": OG.omega_sets,
    "laplacian": OC.laplacian,
    "warp": ON.warp,
    "two_loop": OL.LBFGS.two_loop,
}


def test_mutation_gradient_adjoint_end_sign(monkeypatch):
    monkeypatch.setattr(ON, "cdiff_adj", _cdiff_adj_bad_end)
    monkeypatch.setattr(OO, "cdiff_adj", _cdiff_adj_bad_end)
    monkeypatch.setattr(O, "cdiff_adj", _cdiff_adj_bad_end)
    assert _fails(tn.test_cdiff_adj_is_dense_transpose, 4)
    assert _fails(to.test_gradient_matches_central_fd_everywhere, (8, 8, 8), (1.0, 1.0, 1.0))


def test_mutation_dropped_tau_rho(monkeypatch):
    monkeypatch.setattr(ON, "ngf_terms", _ngf_terms_no_tau_rho)
    monkeypatch.setattr(OO, "ngf_terms", _ngf_terms_no_tau_rho)
    assert _fails(tn.test_ngf_linear_ramp_closed_form, (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))


def test_mutation_swapped_interpolation_weights(monkeypatch):
    monkeypatch.setattr(OG, "index_map", _index_map_swapped)
    monkeypatch.setattr(O, "index_map", _index_map_swapped)
    assert _fails(tg.test_P_equals_kronecker_of_np_interp, (8, 8, 8), (1, 1, 1), (5, 5, 5))
    assert _fails(tg.test_P_reproduces_constants_and_affine, (16, 16, 16), (1, 1, 1), (9, 9, 9))


def test_mutation_wrong_adjoint_weights(monkeypatch):
    monkeypatch.setattr(OG, "omega_sets", _omega_bad)
    assert _fails(tg.test_P_adjoint_identity, (16, 12, 20), (9, 7, 11))
    # (P^T 1 is unchanged by this slip: 4 x 0.5 = 2 per interior axis)
    assert _fails(tg.test_P_equals_kronecker_of_np_interp, (8, 8, 8), (1, 1, 1), (5, 5, 5))


def test_mutation_laplacian_missing_spacing(monkeypatch):
    monkeypatch.setattr(OC, "laplacian", _laplacian_bad)
    monkeypatch.setattr(O, "laplacian", _laplacian_bad)
    assert _fails(tc.test_laplacian_equals_correlate1d_nearest, (2.0, 0.5, 1.5))
    # (a consistently wrong operator still passes the finite-difference pin of
    # S: that pin checks the gradient against S, the library pin checks A)


def _laplacian_bad_centre(u, hy):
    return _orig["laplacian"](u, hy) + 0.5 * u / (hy[0] * hy[0])


def test_mutation_laplacian_centre_weight(monkeypatch):
    monkeypatch.setattr(OC, "laplacian", _laplacian_bad_centre)
    monkeypatch.setattr(O, "laplacian", _laplacian_bad_centre)
    assert _fails(tc.test_curvature_quadratic_closed_form)
    assert _fails(tc.test_curvature_zero_on_shift_and_affine_interior)


def test_mutation_transposed_warp_derivative(monkeypatch):
    monkeypatch.setattr(ON, "warp", _warp_bad)
    monkeypatch.setattr(OO, "warp", _warp_bad)
    monkeypatch.setattr(O, "warp", _warp_bad)
    assert _fails(tn.test_warp_derivative_matches_finite_differences)
    assert _fails(to.test_gradient_matches_central_fd_everywhere, (8, 12, 6), (1.0, 0.5, 2.0))


def test_mutation_lbfgs_scaling(monkeypatch):
    monkeypatch.setattr(OL.LBFGS, "two_loop", _two_loop_bad_gamma)
    assert _fails(tl.test_two_loop_equals_dense_bfgs, 20, 3)


@pytest.mark.parametrize("name", sorted(_orig))
def test_originals_restored(name):
    # the planted mistakes are undone after each case
    mod = {"cdiff_adj": ON, "ngf_terms": ON, "index_map": OG, "omega_sets": OG, "laplacian": OC,
           "warp": ON, "two_loop": OL.LBFGS}[name]
    assert getattr(mod, name) is _orig[name]
