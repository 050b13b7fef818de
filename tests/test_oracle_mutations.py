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


def _curvature_double_weight(u, hy):
    S, g = _orig["curvature"](u, hy)
    return 2.0 * S, 2.0 * g


def _curvature_hbar_image(u, hy):
    # the image-cell volume (h^y / 2 per axis at ratio 2) in place of the node volume
    S, g = _orig["curvature"](u, hy)
    return S / 8.0, g / 8.0


def _curvature_no_half_grad_doubled(u, hy):
    S, g = _orig["curvature"](u, hy)
    return 2.0 * S, 2.0 * g


def _descent_no_reset(self, g):
    d = self.direction(g)
    gtd = float(np.vdot(g, d))
    if not gtd < 0.0:
        d = self.first_direction(g)
        gtd = float(np.vdot(g, d))
    return d, gtd


def _descent_no_fallback(self, g):
    d = self.direction(g)
    return d, float(np.vdot(g, d))


def _keep_every_pair(s, tv):
    return True


def _keep_positive_pair(s, tv):
    return float(np.vdot(s, tv)) > 0.0


def _early_stop_on_new(J_old, J_new, tol):
    return (J_old - J_new) <= tol * (1.0 + abs(J_new))


_orig_keep_pair_func = OL.LBFGS.__dict__["keep_pair"].__func__

_orig = {
    "cdiff_adj": ON.cdiff_adj,
    "ngf_terms": ON.ngf_terms,
    "index_map": OG.index_map,
    "omega_sets": OG.omega_sets,
    "laplacian": OC.laplacian,
    "warp": ON.warp,
    "two_loop": OL.LBFGS.two_loop,
    "curvature": OC.curvature,
    "descent_direction": OL.LBFGS.descent_direction,
    "keep_pair": OL.LBFGS.keep_pair,
    "early_stop_met": OL.early_stop_met,
    "store_pair": OL.LBFGS.store_pair,
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


@pytest.mark.parametrize("bad", [_curvature_double_weight, _curvature_hbar_image,
                                 _curvature_no_half_grad_doubled])
def test_mutation_curvature_weight(monkeypatch, bad):
    # a consistent slip of the quadrature weight in both S and grad S passes
    # every relative pin (FD of S, <grad S, u> = 2 S); the continuum limit
    # fixes it
    monkeypatch.setattr(OC, "curvature", bad)
    monkeypatch.setattr(O, "curvature", bad)
    tc.test_curvature_gradient_homogeneity_and_fd()
    assert _fails(tc.test_curvature_absolute_weight_converges_to_continuous_functional)


def test_mutation_no_memory_drop(monkeypatch):
    monkeypatch.setattr(OL.LBFGS, "descent_direction", _descent_no_reset)
    assert _fails(tl.test_lbfgs_non_descent_direction_drops_memory)


def test_mutation_no_descent_fallback(monkeypatch):
    monkeypatch.setattr(OL.LBFGS, "descent_direction", _descent_no_fallback)
    assert _fails(tl.test_lbfgs_non_descent_direction_drops_memory)


@pytest.mark.parametrize("bad", [_keep_every_pair, _keep_positive_pair])
def test_mutation_pair_test(monkeypatch, bad):
    monkeypatch.setattr(OL.LBFGS, "keep_pair", staticmethod(bad))
    assert _fails(tl.test_lbfgs_pair_curvature_test, 0.5e-10, False)


def _store_drop_newest(self, s, tv):
    # when full, the new pair replaces the newest instead of evicting the oldest
    if len(self.S) >= self.mem:
        self.S[-1], self.Tp[-1] = s, tv
    else:
        self.S.append(s)
        self.Tp.append(tv)


def test_mutation_memory_order(monkeypatch):
    monkeypatch.setattr(OL.LBFGS, "store_pair", _store_drop_newest)
    assert _fails(tl.test_lbfgs_memory_keeps_newest_pairs)


def test_mutation_early_stop_on_new_value(monkeypatch):
    monkeypatch.setattr(OL, "early_stop_met", _early_stop_on_new)
    monkeypatch.setattr(O, "early_stop_met", _early_stop_on_new)
    assert _fails(tl.test_early_stop_rule_on_hand_made_sequence)


@pytest.mark.parametrize("name", sorted(_orig))
def test_originals_restored(name):
    # the planted mistakes are undone after each case
    mod = {"cdiff_adj": ON, "ngf_terms": ON, "index_map": OG, "omega_sets": OG, "laplacian": OC,
           "warp": ON, "two_loop": OL.LBFGS, "curvature": OC,
           "descent_direction": OL.LBFGS, "keep_pair": OL.LBFGS,
           "early_stop_met": OL, "store_pair": OL.LBFGS}[name]
    got = getattr(mod, name)
    if name == "keep_pair":
        assert OL.LBFGS.__dict__["keep_pair"].__func__ is _orig_keep_pair_func
    else:
        assert got is _orig[name]
