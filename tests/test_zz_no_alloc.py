"""The no-allocation entry point (ngf_eval_pair_static) against the entry
point it varies (ngf_eval_pair), through the C ABI: two calls in a row on
the static scratch, the second with a smaller grid, each compared with the
allocating form on the same inputs (J within the parity bar -- here equal,
the reductions are deterministic -- and both gradients, formed by atomic
scatter, within 1e-6 relative L2), plus a grid beyond the scratch's size,
which is refused before anything runs."""

import sys

import numpy as np
import pytest

from paper_1812_06765_amd import synth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float((a.double() - b.double()).norm() / b.double().norm())


def test_static_scratch_form_equals_allocating_form(gpu_lib):
    ngf = gpu_lib
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    for m, seed in (((128, 128, 96), 61), ((64, 48, 32), 62)):
        _say(f"[no-alloc] m={m}")
        pr = synth.ct_phantom_pair(m, seed_R=seed, seed_u=seed + 100, max_disp=3.0,
                                   cp_spacing=8.0)
        my = tuple(v // 2 + 1 for v in m)
        X = np.stack(np.meshgrid(*[np.arange(n) * 2.0 for n in my], indexing="ij"))
        y = X + synth.smooth_node_perturbation(my, 6.0, 2.0, seed)
        R, T, yt = _t(pr.R), _t(pr.T), _t(y)
        Js, gys, gTs = ctx.eval_pair(R, T, yt, static=True)
        Ja, gya, gTa = ctx.eval_pair(R, T, yt)
        ey, eT = _rel(gys, gya), _rel(gTs, gTa)
        _say(f"[no-alloc] J static {Js} allocating {Ja}; grad y {ey:.2e}, grad T {eT:.2e}")
        assert abs(Js - Ja) <= 1e-12 * abs(Ja)
        assert ey <= 1e-6 and eT <= 1e-6
        # value only
        Jv, _, _ = ctx.eval_pair(R, T, yt, grad_y=False, grad_T=False, static=True)
        assert abs(Jv - Ja) <= 1e-12 * abs(Ja)


def test_static_scratch_form_refuses_oversized_grid(gpu_lib):
    import torch
    ngf = gpu_lib
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    m = (1024, 1024, 1024)
    my = tuple(v // 2 + 1 for v in m)
    # the size check runs before anything touches the (never read) inputs
    R = torch.empty(1, dtype=torch.float32, device="cuda")
    y = torch.empty(1, dtype=torch.float32, device="cuda")
    import ctypes
    from paper_1812_06765_amd.ngf import Grid, _ptr
    g = Grid((ctypes.c_int32 * 3)(*m), (ctypes.c_double * 3)(1.0, 1.0, 1.0))
    myc = (ctypes.c_int32 * 3)(*my)
    st = ctx.lib.ngf_eval_pair_static(ctx.h, ctypes.byref(g), ctypes.byref(myc), _ptr(R),
                                      _ptr(R), _ptr(y), None, None, None, None, None)
    assert st == ngf.E_SHAPE
    assert "static scratch" in ctx.lib.ngf_last_error(ctx.h).decode()
