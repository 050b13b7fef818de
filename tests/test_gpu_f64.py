"""The float64 GPU evaluation against the float64 oracle, and the precision
study of the float32 evaluation (Sec. 3 of the paper compares its float32
GPU results with float64 CPU results).

Both float64 sides compute the same definitions; they differ only in the
order of rounding (summation order, fused multiply-adds).  Bound used here:
every value of the chain is a short fixed-length expression (<= 64 terms per
sum) except the sums over all voxels and nodes, whose rounding error is at
most n eps |sum of |terms||; for D the terms 1 - r^2 are non-negative and
for S the terms (A u)^2 are, so |J_gpu - J_oracle| <= ~1e-16 * n * J
(n <= 2^21 here) plus per-voxel errors of a few ulps: 1e-9 relative is a
safe bar and the observed differences are near 1e-15.  The gradient entries
are sums of at most 64 x 3 products with cancellation; relative L2 over the
vector 1e-9 is again far above the few-ulp differences observed.
"""

import sys
import time

import numpy as np
import pytest

import oracle as O
from paper_1812_06765_amd import synth

pytestmark = pytest.mark.gpu

J64_RTOL = 1e-9
G64_RTOL = 1e-9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check64(ctx, level, prob, y64, tag):
    import torch
    Jo, go, (Do, So) = O.eval_J_grad(prob, y64)
    J, g, (D, S) = ctx.eval_J_grad_f64(level, _dev(y64, torch.float64))
    g = g.cpu().numpy()
    eJ, eg = abs(J - Jo) / abs(Jo), _rel(g, go)
    _say(f"[f64] {tag}: J rel {eJ:.2e}, D rel {abs(D - Do) / abs(Do):.2e}, "
         f"S {S:.6e}/{So:.6e}, grad rel L2 {eg:.2e}")
    assert eJ <= J64_RTOL, (tag, J, Jo)
    assert abs(D - Do) <= J64_RTOL * abs(Do), (tag, D, Do)
    assert abs(S - So) <= J64_RTOL * abs(So) + 1e-12 * abs(Jo), (tag, S, So)
    assert eg <= G64_RTOL, (tag, eg)
    # value only: the same J; a second call: the same bits
    Jv, gv, _ = ctx.eval_J_grad_f64(level, _dev(y64, torch.float64), want_grad=False)
    assert gv is None and Jv == J
    J2, g2, _ = ctx.eval_J_grad_f64(level, _dev(y64, torch.float64))
    assert J2 == J and np.array_equal(g2.cpu().numpy(), g)
    return J, g


@pytest.mark.parametrize("m,h,ratio", [((32, 32, 32), (1.0, 1.0, 1.0), 2),
                                       ((44, 36, 40), (1.0, 1.5, 0.75), 2),
                                       ((36, 20, 132), (1.0, 1.0, 1.0), 2),
                                       ((64, 48, 32), (1.0, 1.0, 2.0), 4),
                                       ((28, 24, 68), (0.5, 2.0, 1.0), 4)])
def test_f64_eval_matches_oracle(gpu_lib, m, h, ratio):
    import torch
    ngf = gpu_lib
    pr = synth.ct_phantom_pair(m, h, seed_R=21, seed_u=22, max_disp=3.0, cp_spacing=8.0)
    ctx = ngf.Context(alpha=0.05, tau=10.0, rho=10.0, levels=1, ratio=ratio)
    ctx.build_pyramid(_dev(pr.R, torch.float32), _dev(pr.T, torch.float32), h)
    my = tuple(v // ratio + 1 for v in m)
    prob = O.Problem(pr.R, pr.T, h, my, 0.05, 10.0, 10.0)
    X = prob.identity()
    for amp, seed in ((0.0, 0), (1.5, 31), (4.0, 32)):
        y = X + (synth.smooth_node_perturbation(my, 4.0, amp, seed) if amp > 0 else 0.0)
        _check64(ctx, 0, prob, y, f"{m} h={h} r{ratio} amp={amp}")


def test_f64_pyramid_levels_and_errors(gpu_lib):
    import torch
    ngf = gpu_lib
    pr = synth.ct_phantom_pair((64, 64, 64), seed_R=3, seed_u=4)
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=2)
    ctx.build_pyramid(_dev(pr.R, torch.float32), _dev(pr.T, torch.float32))
    # coarse level first, then the finer one (the scratch grows), then coarse again
    for level in (1, 0, 1):
        li = ctx.level_info(level)
        R, T = (t.cpu().numpy() for t in ctx.level_images(level))
        prob = O.Problem(R, T, li.h, li.my, 0.1, 10.0, 10.0)
        y = prob.identity() + synth.smooth_node_perturbation(li.my, 4.0, 2.0 * li.h[0], 40)
        _check64(ctx, level, prob, y, f"pyramid level {level}")
    with pytest.raises(TypeError):
        ctx.eval_J_grad_f64(0, torch.zeros((3, 33, 33, 33), device="cuda"))
    with pytest.raises(ngf.NgfError):
        ctx.eval_J_grad_f64(2, torch.zeros((3, 9, 9, 9), dtype=torch.float64, device="cuda"))


def test_precision_study_128(gpu_lib):
    """The 128^3 CT pair at y = X + delta, delta a smooth field of peak norm
    0, 0.75, 1.5, 2.25, 3 voxels: the float32 evaluation (at y rounded to
    float32) and the float64 evaluation against the oracle.  Two float32
    errors are reported: against the oracle at the same float32 y (the
    arithmetic alone) and at the float64 y (arithmetic plus the rounding of
    y itself)."""
    import torch
    ngf = gpu_lib
    m = (128, 128, 128)
    pr = synth.ct_phantom_pair(m, seed_R=3, seed_u=4)
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    ctx.build_pyramid(_dev(pr.R, torch.float32), _dev(pr.T, torch.float32))
    my = (65, 65, 65)
    prob = O.Problem(pr.R, pr.T, (1.0, 1.0, 1.0), my, 0.1, 10.0, 10.0)
    X = prob.identity()
    for k, amp in enumerate((0.0, 0.75, 1.5, 2.25, 3.0)):
        y64 = X + (synth.smooth_node_perturbation(my, 8.0, amp, 7 + k) if amp > 0 else 0.0)
        y32 = y64.astype(np.float32)
        Jo, go, _ = O.eval_J_grad(prob, y64)
        Jo32, go32, _ = O.eval_J_grad(prob, y32.astype(np.float64))
        J32, g32, _ = ctx.eval_J_grad(0, _dev(y32, torch.float32))
        g32 = g32.cpu().numpy().astype(np.float64)
        J64, g64, _ = ctx.eval_J_grad_f64(0, _dev(y64, torch.float64))
        g64 = g64.cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.eval_J_grad_f64(0, _dev(y64, torch.float64))
        t64 = (time.perf_counter() - t0) / 5
        row = dict(amp=amp,
                   f32_J=abs(J32 - Jo32) / abs(Jo32), f32_g=_rel(g32, go32),
                   f32y_J=abs(J32 - Jo) / abs(Jo), f32y_g=_rel(g32, go),
                   f64_J=abs(J64 - Jo) / abs(Jo), f64_g=_rel(g64, go))
        _say("[precision128] " + " ".join(f"{a}={b:.3e}" for a, b in row.items())
             + f" f64_eval_ms={1e3 * t64:.2f}")
        assert row["f32_J"] <= 1e-5 and row["f32_g"] <= 1e-4
        assert row["f64_J"] <= J64_RTOL and row["f64_g"] <= G64_RTOL
