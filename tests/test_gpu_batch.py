"""Batched form on the GPU: registrations of many pairs of different shapes,
in graph mode (all pairs level by level, one batched launch sequence per
L-BFGS round, captured as a hipGraph and replayed) and in threads mode
(worker threads, each with its own context and stream).

Every pair's deformation and per-level report must equal, bit for bit, the
single-pair registration with the same image-pass variant (the single-pair
registration is itself checked against the FP64 oracle in the parity tests):
the batch changes where and when a pair runs, never what it computes.  Also
checked: independence from the number of workers, pairs whose shapes differ
only in axis order, the uneven-shape batch at its real sizes (a leading
subset of the 64 drawn shapes), and the error path.
"""

import sys

import numpy as np
import pytest

from paper_1812_06765_amd import synth

pytestmark = pytest.mark.gpu

PARAMS = dict(alpha=0.1, tau=10.0, rho=10.0, ratio=2, lbfgs_mem=5, tol_J=1e-6,
              early_stop=True)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pairs(shapes, seed0, max_disp=3.0):
    import torch
    out = []
    for i, m in enumerate(shapes):
        pr = synth.ct_phantom_pair(m, seed_R=seed0 + 2 * i, seed_u=seed0 + 2 * i + 1,
                                   max_disp=max_disp)
        out.append((torch.from_numpy(pr.R).cuda(), torch.from_numpy(pr.T).cuda()))
    return out


def _single(ngf, pairs, levels, max_iter, variant="by_size"):
    ctx = ngf.Context(levels=levels, max_iter=max_iter, **PARAMS)
    ctx.set_kernel(variant)
    ys, reps = [], []
    for R, T in pairs:
        y, rep = ctx.register(R, T)
        ys.append(y.clone())
        reps.append(rep)
    ctx.close()
    return ys, reps


def _same(a, b):
    import torch
    return a.shape == b.shape and bool(torch.equal(a, b))


def _strip(rep):
    return [{k: v for k, v in r.items() if k != "ms"} for r in rep]


SMALL = [(32, 48, 40), (64, 32, 48), (48, 48, 48), (40, 56, 32), (32, 32, 32),
         (56, 40, 64), (48, 32, 64), (64, 48, 32)]


def test_empty_batch_is_a_no_op(gpu_lib):
    ngf = gpu_lib
    for mode in ("graph", "threads"):
        b = ngf.Batch(levels=2, max_iter=5, workers=2, mode=mode, **PARAMS)
        ys, reps = b.register([], [])
        b.close()
        assert ys == [] and reps == [], mode


def test_batch_equals_single_pair_bitwise(gpu_lib):
    ngf = gpu_lib
    pairs = _pairs(SMALL, 100)
    _say(f"[batch] {len(pairs)} pairs, shapes {SMALL}")
    ys1, reps1 = _single(ngf, pairs, levels=2, max_iter=15)
    for mode, workers in (("graph", 1), ("threads", 1), ("threads", 3), ("threads", 8)):
        b = ngf.Batch(levels=2, max_iter=15, workers=workers, mode=mode, **PARAMS)
        b.set_kernel("by_size")
        ys, reps = b.register([p[0] for p in pairs], [p[1] for p in pairs])
        b.close()
        for i in range(len(pairs)):
            assert _same(ys[i], ys1[i]), (mode, workers, i)
            assert _strip(reps[i]) == _strip(reps1[i]), (mode, workers, i)
        _say(f"[batch] {mode} workers={workers}: all pairs bitwise equal to single-pair runs")
    # the registrations did something: J fell at the finest level
    for rep in reps1:
        assert rep[0]["iters"] >= 1 and np.isfinite(rep[0]["J"])


@pytest.mark.parametrize("MODE", ["graph", "threads"])
def test_batch_forced_variant_and_reuse(gpu_lib, MODE):
    """A forced variant applies to every worker; a second batch on the same
    object (storage kept from the first) gives the same results."""
    import torch
    ngf = gpu_lib
    pairs = _pairs(SMALL[:5], 200)
    ys1, _ = _single(ngf, pairs, levels=2, max_iter=8, variant="march32x8")
    b = ngf.Batch(levels=2, max_iter=8, workers=4, mode=MODE, **PARAMS)
    b.set_kernel("march32x8")
    for rnd in range(2):
        ys, _ = b.register([p[0] for p in pairs], [p[1] for p in pairs])
        for i in range(len(pairs)):
            assert _same(ys[i], ys1[i]), (rnd, i)
    # smaller pairs after larger ones, and an empty batch
    ys, _ = b.register([pairs[4][0]], [pairs[4][1]])
    assert _same(ys[0], ys1[4])
    ys, reps = b.register([], [])
    assert ys == [] and reps == []
    b.close()
    torch.cuda.synchronize()


def test_batch_uneven_shapes_at_full_size(gpu_lib):
    """The leading pairs of the 64-pair uneven batch (axes drawn from
    96..256, three levels) at their real sizes."""
    ngf = gpu_lib
    shapes = synth.batch_shapes(64)[:6]
    pairs = _pairs(shapes, 300, max_disp=6.0)
    _say(f"[batch] uneven shapes {shapes}")
    b = ngf.Batch(levels=3, max_iter=50, workers=4, **PARAMS)
    b.set_kernel("by_size")
    ys, reps = b.register([p[0] for p in pairs], [p[1] for p in pairs])
    pick = [0, 5]
    ys1, reps1 = _single(ngf, [pairs[i] for i in pick], levels=3, max_iter=50)
    for k, i in enumerate(pick):
        assert _same(ys[i], ys1[k]), i
        assert _strip(reps[i]) == _strip(reps1[k]), i
    import torch
    for i, (y, rep) in enumerate(zip(ys, reps)):
        assert bool(torch.isfinite(y).all()), i
        assert len(rep) == 3
        for r in rep:
            assert r["info"] in (ngf.INFO_CONVERGED, ngf.INFO_MAX_ITER), (i, r)
            assert r["evals"] >= r["iters"] + 1
    # the timed selection (the graph mode's default), shared by the pairs:
    # valid results and the same per-level outcome classes
    b.set_kernel("auto")
    ys2, reps2 = b.register([p[0] for p in pairs], [p[1] for p in pairs])
    b.close()
    for i, (y, rep) in enumerate(zip(ys2, reps2)):
        assert bool(torch.isfinite(y).all()), i
        for r, r0 in zip(rep, reps[i]):
            assert (r["iters"] == r0["iters"]
                    or ngf.INFO_CONVERGED in (r["info"], r0["info"])), (i, r, r0)
            assert abs(r["J"] - r0["J"]) <= 5e-2 * abs(r0["J"]), (i, r, r0)


@pytest.mark.parametrize("MODE", ["graph", "threads"])
def test_batch_error_names_the_pair(gpu_lib, MODE):
    ngf = gpu_lib
    import torch
    good = _pairs([(32, 32, 32)], 400)[0]
    bad = (torch.zeros((30, 32, 32), device="cuda"), torch.zeros((30, 32, 32), device="cuda"))
    b = ngf.Batch(levels=2, max_iter=3, workers=2, mode=MODE, **PARAMS)
    with pytest.raises(ngf.NgfError) as e:
        b.register([good[0], bad[0]], [good[1], bad[1]])
    assert e.value.status == ngf.E_SHAPE and "pair 1" in str(e.value)
    nan = good[1].clone()
    nan[3, 4, 5] = float("nan")
    with pytest.raises(ngf.NgfError) as e:
        b.register([good[0], good[0]], [good[1], nan])
    assert e.value.status == ngf.E_NONFINITE and "pair 1" in str(e.value)
    # the batch object stays usable after a failure
    ys, _ = b.register([good[0]], [good[1]])
    assert bool(torch.isfinite(ys[0]).all())
    b.close()


def test_batch_eval_equals_single_pair_eval_and_oracle(gpu_lib):
    """The batched evaluation (ngf_batch_build, then ngf_batch_eval: one
    image pass per variant in use, one node pass and one reduction over all
    pairs) on pairs of different shapes, at two pyramid levels: every J and
    gradient bit for bit the single-pair ngf_eval_J_grad's with the same
    variant, which the oracle pins (J within 1e-5, grad J within 1e-4
    relative L2), checked here again for one pair; the value-only form gives
    the same J."""
    import torch

    import oracle as O
    ngf = gpu_lib
    shapes = [(64, 48, 32), (32, 64, 48), (48, 48, 48)]
    pairs = _pairs(shapes, 71)
    b = ngf.Batch(levels=2, max_iter=5, **PARAMS)
    b.set_kernel("by_size")
    b.build([p[0] for p in pairs], [p[1] for p in pairs])
    single = ngf.Context(levels=2, max_iter=5, **PARAMS)
    single.set_kernel("by_size")
    for lev in (0, 1):
        ys = []
        for i, m in enumerate(shapes):
            my = b.node_shape(i, lev)
            X = O.identity(tuple(v >> lev for v in m), (2.0 ** lev,) * 3, my)
            d = synth.smooth_node_perturbation(my, 4.0, 1.5 * 2 ** lev, 80 + i)
            ys.append(torch.from_numpy((X + d).astype(np.float32)).cuda())
        Js, gs = b.eval(lev, ys)
        Jv, gv = b.eval(lev, ys, want_grad=False)
        assert gv is None and Jv == Js
        for i, (R, T) in enumerate(pairs):
            single.build_pyramid(R, T)
            J, g, _ = single.eval_J_grad(lev, ys[i])
            _say(f"[batch eval] level {lev} pair {shapes[i]}: J {Js[i]} single {J}")
            assert Js[i] == J and bool(torch.equal(gs[i], g))
        # the oracle on the last pair at this level
        Rl, Tl = single.level_images(lev)
        prob = O.Problem(Rl.cpu().numpy().astype(np.float64), Tl.cpu().numpy().astype(np.float64),
                         (2.0 ** lev,) * 3, b.node_shape(2, lev), 0.1, 10.0, 10.0)
        Jo, go, _ = O.eval_J_grad(prob, ys[2].cpu().numpy().astype(np.float64))
        err = float(np.linalg.norm(gs[2].cpu().numpy() - go) / np.linalg.norm(go))
        assert abs(Js[2] - Jo) <= 1e-5 * abs(Jo) and err <= 1e-4
    single.close()
    b.close()
