"""Differentiation form on the GPU: the autograd Function around the library's
scatter backward, at 128^3 image / 65^3 deformation grid.

Checks: central finite differences (step 1e-3 in y, 1e-3 of the intensity
scale in T) of the library's own J on 256 random y entries and 64 random
template voxels inside the body (y entries
whose stencil moves a warp coordinate across a cell boundary are excluded:
the trilinear warp has a kink there); the FP64 oracle's gradients with
respect to y and T; and the plain (gather) form's gradient.  Random smooth
deformations of 0 to 3 voxels.
"""

import sys

import numpy as np
import pytest

import oracle as O
from oracle.objective import crossing_mask
from paper_1812_06765_amd import synth

pytestmark = pytest.mark.gpu

M = (128, 128, 128)
MY = (65, 65, 65)
H = (1.0, 1.0, 1.0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup(gpu_lib):
    ngf = gpu_lib
    pr = synth.ct_phantom_pair(M, seed_R=3, seed_u=4)
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    prob = O.Problem(pr.R, pr.T, H, MY, 0.1, 10.0, 10.0)
    return ngf, ctx, pr, prob


def _y(prob, amp, seed):
    d = synth.smooth_node_perturbation(prob.my, 8.0, amp, seed) if amp > 0 else 0.0
    return (prob.identity() + d).astype(np.float32)


@pytest.mark.parametrize("amp", [0.0, 0.75, 1.5, 2.25, 3.0])
def test_autograd_against_oracle_and_plain(setup, amp):
    import torch
    from paper_1812_06765_amd.autograd import ngf_objective
    ngf, ctx, pr, prob = setup
    y32 = _y(prob, amp, 70 + int(4 * amp))
    R, T = _t(pr.R), _t(pr.T)
    y = _t(y32).requires_grad_(True)
    Tg = T.clone().requires_grad_(True)
    J = ngf_objective(y, Tg, R, H, ctx)
    J.backward()
    Jo, go, gTo, _ = O.eval_J_grad_T(prob, y32.astype(np.float64))
    _say(f"[autograd] amp={amp} J={float(J.detach())} oracle={Jo}")
    assert abs(float(J.detach()) - Jo) <= 1e-5 * abs(Jo)
    gy = y.grad.cpu().numpy().astype(np.float64)
    gT = Tg.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gy - go) <= 1e-4 * np.linalg.norm(go)
    assert np.linalg.norm(gT - gTo) <= 1e-4 * np.linalg.norm(gTo)
    # the plain form (gather P^T, no atomics) on the same pair
    ctx.build_pyramid(R, T)
    Jp, gp, _ = ctx.eval_J_grad(0, _t(y32))
    assert abs(Jp - float(J)) <= 1e-9 * abs(Jp)
    gp = gp.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gy - gp) <= 1e-5 * np.linalg.norm(gp)


def test_autograd_upstream_scale_and_partial_inputs(setup):
    import torch
    from paper_1812_06765_amd.autograd import ngf_objective
    ngf, ctx, pr, prob = setup
    y32 = _y(prob, 1.5, 81)
    R, T = _t(pr.R), _t(pr.T)
    y = _t(y32).requires_grad_(True)
    J = ngf_objective(y, T, R, H, ctx)  # T constant
    (2.5 * J).backward()
    g1 = y.grad.clone()
    y.grad = None
    ngf_objective(y, T, R, H, ctx).backward()
    g2 = y.grad
    assert torch.allclose(g1, 2.5 * g2, rtol=1e-5, atol=1e-6 * float(g2.abs().max()))


def test_autograd_finite_differences(setup):
    import torch
    ngf, ctx, pr, prob = setup
    rng = np.random.default_rng(12)
    y32 = _y(prob, 2.0, 90)
    R, T = _t(pr.R), _t(pr.T)
    _, gy, gT = ctx.eval_pair(R, T, _t(y32), H)
    gy = gy.cpu().numpy().astype(np.float64)
    gT = gT.cpu().numpy().astype(np.float64)
    step = 1e-3
    bad = crossing_mask(prob, y32.astype(np.float64), step)
    cand = np.argwhere(~bad)
    picks = cand[rng.choice(len(cand), size=256, replace=False)]
    fds, ans = [], []
    for idx in picks:
        idx = tuple(int(v) for v in idx)
        yp, ym = y32.copy(), y32.copy()
        yp[idx] += np.float32(step)
        ym[idx] -= np.float32(step)
        Jp = ctx.eval_pair(R, T, _t(yp), H, grad_y=False, grad_T=False)[0]
        Jm = ctx.eval_pair(R, T, _t(ym), H, grad_y=False, grad_T=False)[0]
        fds.append((Jp - Jm) / (float(yp[idx]) - float(ym[idx])))
        ans.append(gy[idx])
    _check_fd("y", np.array(fds), np.array(ans), np.abs(gy).max(), int(bad.sum()), bad.size)
    # the template is in Hounsfield units (|T| up to ~1000): a step of 1e-3
    # of that scale; 1e-3 HU itself would be ~16 float32 ulps of T and the
    # difference quotient would measure rounding, not the derivative
    stepT = 1e-3 * float(np.abs(pr.T).max())
    body = np.argwhere(pr.R > -500.0)
    picks = body[rng.choice(len(body), size=64, replace=False)]
    fds, ans = [], []
    for idx in picks:
        idx = tuple(int(v) for v in idx)
        Tp, Tm = pr.T.copy(), pr.T.copy()
        Tp[idx] += np.float32(stepT)
        Tm[idx] -= np.float32(stepT)
        Jp = ctx.eval_pair(R, _t(Tp), _t(y32), H, grad_y=False, grad_T=False)[0]
        Jm = ctx.eval_pair(R, _t(Tm), _t(y32), H, grad_y=False, grad_T=False)[0]
        fds.append((Jp - Jm) / (float(Tp[idx]) - float(Tm[idx])))
        ans.append(gT[idx])
    _check_fd("T", np.array(fds), np.array(ans), np.abs(gT).max(), 0, 64)


def _check_fd(name, fd, an, gmax, excluded, total):
    """J is evaluated in float32 bulk arithmetic: the template values (about
    1000 HU) round at ~6e-5 HU, about 1e-3 of what a 1e-3 step changes, and a
    node's gradient is a cancelling sum of ~150 voxel terms, so single
    central differences carry noise of a few per cent of the entry.  The
    test therefore bounds the relative L2 error over all sampled entries
    (a wrong sign, a dropped term or a swapped axis gives O(1)) and each
    entry loosely."""
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    worst = np.max(np.abs(fd - an) / (0.1 * np.abs(an) + 5e-3 * gmax))
    _say(f"[fd] {name}: rel-L2 {rel:.2e} over {len(an)} entries, worst normalised {worst:.2f} "
         f"({excluded} of {total} entries excluded as kink crossings)")
    assert rel <= 2e-2, rel
    assert worst <= 1.0, worst


def test_pair_form_on_a_grid_of_a_million_nodes(gpu_lib):
    """The differentiation form on a 256 x 256 x 128 image (129 x 129 x 65 =
    1.08 M nodes, where the node pass runs in its marching form): J and the
    gradients with respect to y and T against the oracle."""
    ngf = gpu_lib
    m = (256, 256, 128)
    my = (129, 129, 65)
    pr = synth.ct_phantom_pair(m, seed_R=13, seed_u=14)
    prob = O.Problem(pr.R, pr.T, H, my, 0.1, 10.0, 10.0)
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    j = [np.arange(n, dtype=np.float64) / (n - 1) for n in my]
    w = (np.sin(2 * np.pi * j[0])[:, None, None] * np.sin(np.pi * j[1])[None, :, None]
         * np.cos(np.pi * j[2])[None, None, :])
    y32 = (prob.identity() + 2.0 * np.stack([w, -w, 0.5 * w])).astype(np.float32)
    J, gy, gT = ctx.eval_pair(_t(pr.R), _t(pr.T), _t(y32), H)
    Jo, go, gTo, _ = O.eval_J_grad_T(prob, y32.astype(np.float64))
    gy = gy.cpu().numpy().astype(np.float64)
    gT = gT.cpu().numpy().astype(np.float64)
    ey = np.linalg.norm(gy - go) / np.linalg.norm(go)
    eT = np.linalg.norm(gT - gTo) / np.linalg.norm(gTo)
    _say(f"[pair 1M] J {J} oracle {Jo}; grad y rel-L2 {ey:.2e}, grad T rel-L2 {eT:.2e}")
    assert abs(J - Jo) <= 1e-5 * abs(Jo)
    assert ey <= 1e-4 and eT <= 1e-4


def test_level_form_matches_pair_form_and_oracle(gpu_lib):
    """ngf_eval_J_grad_T on a pyramid level (buffers from the pyramid, no
    allocation) against the pair form on the same level's images, and both
    against the oracle's dJ/dy and dJ/dT."""
    ngf = gpu_lib
    m = (128, 128, 128)
    pr = synth.ct_phantom_pair(m, seed_R=3, seed_u=4)
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=2)
    ctx.build_pyramid(_t(pr.R), _t(pr.T))
    Rs, Ts = O.pyramid(pr.R, pr.T, 2)
    for lev in (1, 0):
        li = ctx.level_info(lev)
        prob = O.Problem(Rs[lev], Ts[lev], li.h, li.my, 0.1, 10.0, 10.0)
        d = synth.smooth_node_perturbation(li.my, 8.0, 1.5 * li.h[0], 17 + lev)
        y32 = (prob.identity() + d).astype(np.float32)
        J, gy, gT = ctx.eval_J_grad_T(lev, _t(y32))
        Rl, Tl = ctx.level_images(lev)
        Jp, gyp, gTp = ctx.eval_pair(Rl, Tl, _t(y32), li.h)
        Jo, go, gTo, _ = O.eval_J_grad_T(prob, y32.astype(np.float64))
        gy = gy.cpu().numpy().astype(np.float64)
        gT = gT.cpu().numpy().astype(np.float64)
        ey = np.linalg.norm(gy - go) / np.linalg.norm(go)
        eT = np.linalg.norm(gT - gTo) / np.linalg.norm(gTo)
        _say(f"[level form] level {lev}: J {J} pair {Jp} oracle {Jo}; grad y {ey:.2e}, "
             f"grad T {eT:.2e}")
        assert J == Jp
        assert abs(J - Jo) <= 1e-5 * abs(Jo)
        assert ey <= 1e-4 and eT <= 1e-4
        assert float((gyp.double() - torch_from(gy)).norm() / torch_from(gy).norm()) <= 1e-6
    # a general grid has no scatter form
    ctx2 = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    ctx2.set_node_grid((37, 37, 37))
    ctx2.build_pyramid(_t(pr.R), _t(pr.T))
    with pytest.raises(ngf.NgfError) as e:
        ctx2.eval_J_grad_T(0, ctx2.identity(0))
    assert e.value.status == ngf.E_SHAPE


def torch_from(a):
    import torch
    return torch.from_numpy(a).cuda()


@pytest.mark.parametrize("ratio,m,h", [
    (2, (36, 42, 50), (1.0, 1.25, 0.8)),
    (4, (36, 44, 52), (0.9, 1.0, 1.1)),
])
def test_pair_form_on_ragged_anisotropic_grids(gpu_lib, ratio, m, h):
    """The scatter form's 3D tiles (4 x 8 x 32 voxels) end partly outside these
    grids on two axes, and the spacing differs per axis: J and the gradients
    with respect to y and T still match the oracle (the blob pair, a smooth
    deformation of up to one voxel)."""
    ngf = gpu_lib
    my = tuple(v // ratio + 1 for v in m)
    pr = synth.blob_phantom_pair(m, h=h, seed_R=21, seed_u=22, max_disp=1.5)
    prob = O.Problem(pr.R, pr.T, h, my, 0.1, 0.1, 0.1)
    ctx = ngf.Context(alpha=0.1, tau=0.1, rho=0.1, levels=1, ratio=ratio)
    d = synth.smooth_node_perturbation(my, 4.0, 1.0, 23)
    y32 = (prob.identity() + d).astype(np.float32)
    J, gy, gT = ctx.eval_pair(_t(pr.R), _t(pr.T), _t(y32), h)
    Jo, go, gTo, _ = O.eval_J_grad_T(prob, y32.astype(np.float64))
    gy = gy.cpu().numpy().astype(np.float64)
    gT = gT.cpu().numpy().astype(np.float64)
    ey = np.linalg.norm(gy - go) / np.linalg.norm(go)
    eT = np.linalg.norm(gT - gTo) / np.linalg.norm(gTo)
    _say(f"[ragged r{ratio}] J {J} oracle {Jo}; grad y rel-L2 {ey:.2e}, grad T rel-L2 {eT:.2e}")
    assert abs(J - Jo) <= 1e-5 * abs(Jo)
    assert ey <= 1e-4 and eT <= 1e-4
    ctx.close()
