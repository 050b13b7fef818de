"""Failure paths on the GPU, each forced from the host (every kernel still
runs to its normal end):

* a line search that never succeeds (Sec. 2.1, L-BFGS with Armijo
  backtracking): every trial is rejected by the injected fault, so each level
  ends after one iteration's 11 trial evaluations with LINESEARCH_FAIL and y
  left where it started; the objective reported is then the oracle's J at
  that (identity) deformation;
* NaN in the deformation: the evaluation and the start of L-BFGS report
  NGF_E_NONFINITE;
* a device allocation failure: NGF_E_OOM, and the context works again once
  the fault is cleared (its results then match the oracle).
"""

import sys

import numpy as np
import pytest

import oracle as O
from paper_1812_06765_amd import synth

pytestmark = pytest.mark.gpu

J_RTOL = 1e-5


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("driver", ["device", "host"])
def test_forced_linesearch_failure(gpu_lib, driver):
    ngf = gpu_lib
    _say(f"[fail] forced line-search failure, driver={driver}")
    pr = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    ctx = ngf.Context(alpha=0.1, tau=0.1, rho=0.1, levels=2, max_iter=5, lbfgs_mem=5)
    ctx.set_driver(driver)
    R, T = _t(pr.R), _t(pr.T)
    ctx.set_faults(ngf.Context.FAULT_REJECT_STEPS)
    y, rep = ctx.register(R, T)
    for r in rep:
        assert r["info"] == ngf.INFO_LINESEARCH_FAIL, rep
        assert r["iters"] == 0 and r["evals"] == 12, rep
    # y never moved: the identity of level 0 (the prolongated coarse identity)
    assert bool((y == ctx.identity(0)).all())
    # the J reported per level is J at the identity, as the oracle has it
    Rs, Ts = O.pyramid(pr.R, pr.T, 2)
    for r in rep:
        lev = r["level"]
        li = ctx.level_info(lev)
        prob = O.Problem(Rs[lev], Ts[lev], li.h, li.my, 0.1, 0.1, 0.1)
        Jo = O.eval_J_grad(prob, prob.identity().astype(np.float32).astype(np.float64))[0]
        assert abs(r["J"] - Jo) <= J_RTOL * abs(Jo), (lev, r["J"], Jo)
    # cleared: the same context registers normally again
    ctx.set_faults(0)
    y2, rep2 = ctx.register(R, T)
    assert all(r["info"] != ngf.INFO_LINESEARCH_FAIL and r["iters"] > 0 for r in rep2), rep2
    assert rep2[0]["J"] < rep[0]["J"]


def test_nan_in_y_is_reported(gpu_lib):
    ngf = gpu_lib
    _say("[fail] NaN in y")
    pr = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    ctx = ngf.Context(alpha=0.1, tau=0.1, rho=0.1, levels=1)
    ctx.build_pyramid(_t(pr.R), _t(pr.T))
    y = ctx.identity(0)
    y[1, 8, 8, 8] = float("nan")
    with pytest.raises(ngf.NgfError) as e:
        ctx.eval_J_grad(0, y)
    assert e.value.status == ngf.E_NONFINITE
    with pytest.raises(ngf.NgfError) as e:
        ctx.lbfgs_reset(0, y)
    assert e.value.status == ngf.E_NONFINITE
    # a NaN only in the gradient path still ends L-BFGS as non-finite: alpha
    # = 0 keeps S out of J, but 0 * NaN is NaN, so J reports it too
    ctx.set_params(alpha=0.0)
    with pytest.raises(ngf.NgfError) as e:
        ctx.eval_J_grad(0, y)
    assert e.value.status == ngf.E_NONFINITE
    # a finite y afterwards evaluates normally
    ctx.set_params(alpha=0.1)
    J, g, _ = ctx.eval_J_grad(0, ctx.identity(0))
    assert np.isfinite(J) and bool(g.isfinite().all())


def test_forced_allocation_failure(gpu_lib):
    ngf = gpu_lib
    _say("[fail] forced allocation failure")
    pr = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    R, T = _t(pr.R), _t(pr.T)
    ctx = ngf.Context(alpha=0.1, tau=0.1, rho=0.1, levels=1)
    ctx.set_faults(ngf.Context.FAULT_ALLOC)
    with pytest.raises(ngf.NgfError) as e:
        ctx.build_pyramid(R, T)
    assert e.value.status == ngf.E_OOM
    ctx.set_faults(0)
    ctx.build_pyramid(R, T)
    prob = O.Problem(pr.R, pr.T, (1.0, 1.0, 1.0), (17, 17, 17), 0.1, 0.1, 0.1)
    y = prob.identity().astype(np.float32)
    J, _, _ = ctx.eval_J_grad(0, _t(y))
    Jo = O.eval_J_grad(prob, y.astype(np.float64))[0]
    assert abs(J - Jo) <= J_RTOL * abs(Jo)
    # the float64 evaluation allocates its scratch on first use
    ctx.set_faults(ngf.Context.FAULT_ALLOC)
    import torch
    with pytest.raises(ngf.NgfError) as e:
        ctx.eval_J_grad_f64(0, torch.from_numpy(y.astype(np.float64)).cuda())
    assert e.value.status == ngf.E_OOM
    ctx.set_faults(0)
    J64, _, _ = ctx.eval_J_grad_f64(0, torch.from_numpy(y.astype(np.float64)).cuda())
    assert abs(J64 - Jo) <= 1e-9 * abs(Jo)
