"""Benchmark: full NGF + curvature registration of a 256^3 CT-like pair on one
MI355X, through the HIP library's C ABI.

One step = one full registration from device-resident R and T: the pyramid
(4 levels, 32^3 ... 256^3), then multi-level L-BFGS (memory 5, up to 50
iterations per level, early stop at a relative decrease of 1e-6), with every
J + grad J evaluation (P, warp, NGF, adjoint, P^T gather, curvature, fused
reductions) in the library's kernels.

Printed (one JSON line):
* value       J + grad J evaluations per second at the 256^3 level (a loop of
              evaluations back to back at the registered deformation);
* ms_per_step the full-registration time (pyramid and all four levels);
  evals_per_s_registration the evaluations of the timed registrations (all
              levels, line-search trials included) per second;
* accuracy_voxels  distance of the registration to the true correspondence at
              sampled body and edge voxels, next to the identity's;
* image_mismatch_hu  mean |T(P y) - R| at sampled voxels for the registration,
              the identity and the true correspondence;
* roofline    the dominant kernel (the fused image-grid pass), timed with HIP
              events on the library's stream over the timed region;
* forms       the differentiation form (level form and autograd) and the
              batched form (64 uneven pairs) beside the plain one;
* cpu_baseline the FP64 oracle on the host, one 256^3 evaluation.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Vector ALU peak for this build: packed FP32 instructions are disabled, so
# FP32 and FP64 FMAs issue at one per lane per clock:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# algorithmic flops of the image-grid pass per voxel (P 63, warp coordinate 6,
# warped value 21, its derivative 22, central differences 12, NGF term and v
# 36, adjoint stencil and chain rule 11, tile-local P^T 21)
FLOPS_PER_VOXEL = 192
METRIC = "J+∇J evals/s and full-registration seconds at 256^3; HBM GB/s vs peak"


def _src_hash():
    h = hashlib.sha256()
    for f in ("k_eval.hip", "k_march.hip", "ngf_internal.h"):
        with open(os.path.join(ROOT, "paper_1812_06765_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel_hash, shape, variant):
    """HBM bytes per launch of the 256^3 image-pass kernel from the committed
    counter summary, only if it was taken from the current kernel source, on
    the same image shape and with the same image-pass variant."""
    path = os.path.join(ROOT, "profiles", "image_pass_256_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if (t.get("kernel_src_sha256_16") != kernel_hash
            or t.get("image_shape") != [int(v) for v in shape]
            or t.get("variant") != variant):
        return None
    return t.get("hbm_bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _nproc():
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def accuracy(ctx, y, pr, samples=20000, seed=5):
    """Mean distance (voxels) between the registration's correspondence P y and
    the true one at sampled voxels: inside the body (R > -500 HU) and on
    strong edges (|grad R| > 200 HU per voxel), next to the same distance for
    the identity.  The true correspondence of T(x) = R(x + u(x)) is z(x)
    with z + u(z) = x (fixed point).  P y is applied by the library."""
    import numpy as np
    import torch

    from paper_1812_06765_amd import synth
    R = pr.R
    rng = np.random.default_rng(seed)
    g = np.stack(np.gradient(R.astype(np.float32)))
    gn = np.sqrt((g.astype(np.float64) ** 2).sum(0))
    del g
    yh = ctx.apply_P(0, y)
    yid = ctx.apply_P(0, ctx.identity(0))
    out = {"samples_per_region": samples}
    for name, mask in (("body", R > -500.0), ("edges", gn > 200.0)):
        cand = np.flatnonzero(mask)
        pick = np.unravel_index(rng.choice(cand, size=min(samples, cand.size), replace=False),
                                R.shape)
        zstar = synth.invert_displacement(pr.field, np.stack(pick).astype(np.float64) + 0.5)
        idx = tuple(torch.from_numpy(p.astype(np.int64)).cuda() for p in pick)
        res = []
        for v in (yid, yh):
            at = v[:, idx[0], idx[1], idx[2]].double().cpu().numpy()
            res.append(float(np.sqrt(((at - zstar) ** 2).sum(0)).mean()))
        out[name] = {"identity": res[0], "registered": res[1]}
    return out


def _trilinear(V, p):
    """V (float64 array) at points p (3, n) in voxel units, voxel i's centre at
    i + 1/2; points outside are clamped to the edge voxels."""
    import numpy as np
    i0, f = [], []
    for d in range(3):
        xi = np.clip(p[d] - 0.5, 0.0, V.shape[d] - 1.0)
        i = np.minimum(np.floor(xi), V.shape[d] - 2).astype(np.int64)
        i0.append(i)
        f.append(xi - i)
    out = np.zeros(p.shape[1])
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                w = ((f[0] if a else 1.0 - f[0]) * (f[1] if b else 1.0 - f[1])
                     * (f[2] if c else 1.0 - f[2]))
                out += w * V[i0[0] + a, i0[1] + b, i0[2] + c]
    return out


def image_mismatch(ctx, y, pr, samples=200000, seed=7):
    """Mean |T(P y) - R| (HU) at uniformly sampled voxels, next to the same for
    the identity and for the true correspondence: the registration's image
    match, which the objective rewards, beside the correspondence error."""
    import numpy as np
    import torch

    from paper_1812_06765_amd import synth
    m = pr.R.shape
    rng = np.random.default_rng(seed)
    pick = np.unravel_index(rng.choice(m[0] * m[1] * m[2], size=samples, replace=False), m)
    pts = np.stack(pick).astype(np.float64) + 0.5
    idx = tuple(torch.from_numpy(p.astype(np.int64)).cuda() for p in pick)
    at = ctx.apply_P(0, y)[:, idx[0], idx[1], idx[2]].double().cpu().numpy()
    zstar = synth.invert_displacement(pr.field, pts)
    Rv = pr.R[pick].astype(np.float64)
    Tv = pr.T.astype(np.float64)
    out = {"samples": samples}
    for name, p in (("identity", pts), ("registered", at), ("truth", zstar)):
        out[name] = float(np.abs(_trilinear(Tv, p) - Rv).mean())
    return out


def cpu_baseline(R, T, evals=2):
    """J + grad J evaluations of the FP64 oracle at the 256^3 level."""
    import numpy as np

    import oracle as O
    m = R.shape
    my = tuple(v // 2 + 1 for v in m)
    prob = O.Problem(R, T, (1.0, 1.0, 1.0), my, 0.1, 10.0, 10.0)
    X = prob.identity()
    # a smooth displacement of up to 2 voxels per component (separable sines)
    j = [np.arange(n, dtype=np.float64) / (n - 1) for n in my]
    wave = (np.sin(2 * np.pi * j[0])[:, None, None] * np.sin(np.pi * j[1])[None, :, None]
            * np.cos(np.pi * j[2])[None, None, :])
    ys = [X, X + 2.0 * np.stack([wave, -wave, 0.5 * wave])]
    dt = 0.0
    for k in range(evals):
        y = ys[k % 2].astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        O.eval_J_grad(prob, y)
        dt += time.perf_counter() - t0
        print(f"[bench] oracle evaluation {k + 1}/{evals} done", file=sys.stderr, flush=True)
    return {"value": evals / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "seconds": dt, "cpu_model": _cpu_model(), "nproc": _nproc(),
            "sample": f"{evals} J+grad J evaluations of the float64 numpy oracle at the "
                      f"{m[0]}x{m[1]}x{m[2]} finest level ({my[0]}x{my[1]}x{my[2]} nodes; "
                      "identity and a smooth displacement of up to 2 voxels), "
                      "single-threaded numpy"}


def bench_pt(args, torch, ngf):
    """P and the three ways of applying P^T (Sec. 2.2, "Grid conversion") as
    standalone operators on the 256^3 image grid / 129^3 deformation grid:
    gather (Eq. 3), atomic scatter, red-black slices (the scatter schemes
    include zeroing their output).  Input: seeded normal values."""
    n = args.size
    ctx = ngf.Context(levels=1)
    R = torch.zeros((n, n, n), dtype=torch.float32, device="cuda")
    ctx.build_pyramid(R, R)
    gen = torch.Generator(device="cuda").manual_seed(9)
    li = ctx.level_info(0)
    z = torch.randn((3,) + li.m, generator=gen, device="cuda")
    y = torch.randn((3,) + li.my, generator=gen, device="cuda")
    out = {"mode": "P^T schemes", "grid": list(li.m), "nodes": list(li.my)}
    reps = 20

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 1e3 * e0.elapsed_time(e1) / reps

    N = li.m[0] * li.m[1] * li.m[2]
    Ny = li.my[0] * li.my[1] * li.my[2]
    us = timed(lambda: ctx.apply_P(0, y))
    out["P_us"] = us
    out["P_GBs"] = (12 * Ny + 12 * N) / (us * 1e-6) / 1e9
    for name in ("gather", "atomic", "redblack"):
        us = timed(lambda: ctx.apply_PT(0, z, name))
        out[f"PT_{name}_us"] = us
        out[f"PT_{name}_GBs"] = (12 * N + 12 * Ny) / (us * 1e-6) / 1e9
    ref = ctx.apply_PT(0, z, "gather").double()
    for name in ("atomic", "redblack"):
        d = (ctx.apply_PT(0, z, name).double() - ref).norm() / ref.norm()
        out[f"PT_{name}_rel_diff_vs_gather"] = float(d)
    print(json.dumps(out), flush=True)


def _batch_inputs(torch, synth, npairs):
    """The uneven batch: axes drawn from {96, 128, 160, 192, 256}, the CT
    phantom recipe per pair (seeds 1000 + 2 i and 1001 + 2 i), generated on
    host threads."""
    from concurrent.futures import ThreadPoolExecutor
    shapes = synth.batch_shapes(npairs)
    t_gen = time.perf_counter()

    def gen(i):
        return synth.ct_phantom_pair(shapes[i], seed_R=1000 + 2 * i, seed_u=1001 + 2 * i)

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        prs = list(ex.map(gen, range(npairs)))
    Rs = [torch.from_numpy(p.R).cuda() for p in prs]
    Ts = [torch.from_numpy(p.T).cuda() for p in prs]
    del prs
    print(f"[bench] {npairs} pairs generated in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    return shapes, Rs, Ts


def _batch_times(torch, ngf, Rs, Ts, max_iter, workers, steps, warmup):
    """Seconds and evaluations of `steps` registrations of the whole batch:
    the batched form in graph and in threads mode, and the pairs one after
    another in one context (3 levels, the workload's parameters)."""
    kw = dict(alpha=0.1, tau=10.0, rho=10.0, levels=3, ratio=2, max_iter=max_iter,
              lbfgs_mem=5, tol_J=1e-6, early_stop=True)

    def timed(run):
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        evals = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            reps = run()
            evals += sum(r["evals"] for rep in reps for r in rep)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, evals

    res = {}
    for mode in ("graph", "threads"):
        b = ngf.Batch(workers=workers, mode=mode, **kw)
        if mode == "threads":
            b.set_kernel("by_size")
        res[mode] = timed(lambda: b.register(Rs, Ts)[1])
        b.close()
        print(f"[bench] batch {mode}: {res[mode][0] / steps:.3f} s per batch", file=sys.stderr,
              flush=True)
    ctx = ngf.Context(**kw)
    res["sequential"] = timed(lambda: [ctx.register(R, T)[1] for R, T in zip(Rs, Ts)])
    ctx.close()
    print(f"[bench] sequential: {res['sequential'][0] / steps:.3f} s per batch",
          file=sys.stderr, flush=True)
    return res


def _batch_summary(res, npairs, steps):
    return {"batch_s": {k: v[0] / steps for k, v in res.items()},
            "evals_per_s": {k: v[1] / v[0] for k, v in res.items()},
            "pairs_per_s": {k: npairs * steps / v[0] for k, v in res.items()}}


def bench_batch(args, torch, ngf, synth):
    """Uneven batch of args.batch pairs, 3 levels.  Timed: the batched form in
    graph mode (the reported value), in threads mode, and the same pairs
    registered one after another by a single context."""
    shapes, Rs, Ts = _batch_inputs(torch, synth, args.batch)
    res = _batch_times(torch, ngf, Rs, Ts, args.max_iter, args.workers, args.steps, args.warmup)
    dt, evals = res["graph"]
    vox = sum(m[0] * m[1] * m[2] for m in shapes)
    out = {
        "metric": METRIC,
        "value": evals / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 coordinates and reductions)",
        "data": "synthetic: seeded CT-like phantom pairs, B-spline warps (max 6 voxels)",
        "config": {"workload": f"batch of {args.batch} pairs, axes drawn from 96..256, "
                               f"{vox / 1e6:.1f} M voxels at the finest levels, 3 levels, "
                               f"alpha=0.1, eps=10, L-BFGS m=5, <= {args.max_iter} it/level, "
                               "early stop 1e-6; batched form in graph mode",
                   "global_batch": args.batch, "seq_len": None, "parallelism": "single GPU"},
        **_batch_summary(res, args.batch, args.steps),
        "threads_workers": args.workers,
    }
    print(json.dumps(out), flush=True)


def bench_forms(args, torch, ngf, synth, reps=20):
    """The differentiation and batched forms beside the plain one, on this
    device.  Differentiation: one 128^3 CT pair (65^3 nodes, alpha 0.1,
    eps 10) at a smooth deformation of up to 2 voxels; per call, the plain
    J + grad J (gather), the level form J, grad_y and grad_T (scatter), and
    the autograd function's forward and backward (J, then both gradients);
    each the median of 5 runs of `reps` calls.
    Batched: the uneven batch of args.forms_batch pairs (1 warm-up, 1 timed
    registration of the whole batch per mode)."""
    from paper_1812_06765_amd.autograd import ngf_objective
    m = (128, 128, 128)
    pr = synth.ct_phantom_pair(m, seed_R=3, seed_u=4)
    R = torch.from_numpy(pr.R).cuda()
    T = torch.from_numpy(pr.T).cuda()
    ctx = ngf.Context(alpha=0.1, tau=10.0, rho=10.0, levels=1)
    ctx.build_pyramid(R, T)
    my = ctx.level_info(0).my
    d = torch.from_numpy(synth.smooth_node_perturbation(my, 8.0, 2.0, 7).astype("float32"))
    y = (ctx.identity(0) + d.cuda()).contiguous()
    g = torch.empty_like(y)
    yv = y.clone().requires_grad_(True)
    Tv = T.clone().requires_grad_(True)

    def autograd_call():
        J = ngf_objective(yv, Tv, R, (1.0, 1.0, 1.0), ctx)
        torch.autograd.grad(J, (yv, Tv))

    calls = {"plain": lambda: ctx.eval_J_grad_async(0, y, g),
             "level_form": lambda: ctx.eval_J_grad_T(0, y, sync=False),
             "autograd": autograd_call}
    us = {}
    for name, call in calls.items():
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        runs = []
        for _ in range(5):
            t0 = time.perf_counter()
            for _ in range(reps):
                call()
            torch.cuda.synchronize()
            runs.append(1e6 * (time.perf_counter() - t0) / reps)
        us[name] = sorted(runs)[2]  # median of 5 runs
    ctx.close()
    print(f"[bench] forms at 128^3: {us}", file=sys.stderr, flush=True)
    out = {"differentiation": {
        "workload": "128x128x128 CT pair, 65x65x65 nodes, alpha=0.1, eps=10, smooth y",
        "us_per_call": us,
        "vs_plain": {k: us[k] / us["plain"] for k in us}}}
    if args.forms_batch > 0:
        shapes, Rs, Ts = _batch_inputs(torch, synth, args.forms_batch)
        res = _batch_times(torch, ngf, Rs, Ts, args.max_iter, args.workers, 1, 1)
        vox = sum(s[0] * s[1] * s[2] for s in shapes)
        out["batched"] = {
            "workload": f"{args.forms_batch} pairs, axes drawn from 96..256, "
                        f"{vox / 1e6:.1f} M voxels at the finest levels, 3 levels",
            **_batch_summary(res, args.forms_batch, 1),
            "speedup_vs_sequential": {k: res["sequential"][0] / res[k][0]
                                      for k in ("graph", "threads")},
            "threads_workers": args.workers}
        del Rs, Ts
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--shape", type=int, nargs=3, default=None,
                    help="image shape (x y z) instead of size^3, e.g. 512 512 1536")
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--max-iter", type=int, default=50)
    ap.add_argument("--alpha", type=float, default=0.1, help="curvature weight")
    ap.add_argument("--ratio", type=int, default=2,
                    help="image cells per deformation-grid cell between levels (2 or 4)")
    ap.add_argument("--node-grid", type=int, nargs=3, default=None,
                    help="finest-level deformation-grid nodes per axis (default m/ratio + 1)")
    ap.add_argument("--eps", type=float, default=10.0,
                    help="NGF edge parameter of R and T (HU per unit length)")
    ap.add_argument("--noise", type=float, default=20.0,
                    help="std of the phantom's Gaussian noise in R and T (HU)")
    ap.add_argument("--finest-evals", type=int, default=100,
                    help="evaluations per run of the finest-level rate")
    ap.add_argument("--finest-runs", type=int, default=5,
                    help="runs of the finest-level rate (the median is reported)")
    ap.add_argument("--host-reps", type=int, default=3,
                    help="registrations from pinned host arrays (PCIe-inclusive timing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the distance of the registration to the true correspondence")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead: the uneven batch of this many pairs (axes drawn from "
                         "96..256, 3 levels) through the batched form")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--forms-batch", type=int, default=64,
                    help="pairs of the batched form timed beside the plain one in the default "
                         "line (0: none)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the differentiation and batched forms in the default line")
    ap.add_argument("--pt-ablation", action="store_true",
                    help="instead: time the three P^T schemes and P at the 256^3 grids")
    ap.add_argument("--kernel", default="auto",
                    help="image-pass selection: auto (the timed selection, default), by_size "
                         "(the size rule) or a variant name")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only copy 1 GiB device-to-device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the registration of one pair runs on one "
              "device and this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.pmc_probe:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": "copy", "bytes_read": x.numel() * 4,
                          "bytes_written": y.numel() * 4}), flush=True)
        return

    from paper_1812_06765_amd import ngf, synth

    if args.batch:
        return bench_batch(args, torch, ngf, synth)
    if args.pt_ablation:
        return bench_pt(args, torch, ngf)

    shape = tuple(args.shape) if args.shape else (args.size,) * 3
    sname = "x".join(str(v) for v in shape)
    t_gen = time.perf_counter()
    if shape[0] * shape[1] * shape[2] > (1 << 26):  # large volumes: in slabs
        def progress(done, total):
            if done % 128 == 0 or done == total:
                print(f"[bench] inputs: {done}/{total} planes", file=sys.stderr, flush=True)
        pr = synth.ct_phantom_pair_slabs(shape, seed_R=5, seed_u=6, noise=args.noise,
                                         progress=progress,
                                         workers=min(16, os.cpu_count() or 1))
    else:
        pr = synth.ct_phantom_pair(shape, seed_R=5, seed_u=6, noise=args.noise)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] inputs {sname} generated in {t_gen:.1f}s", file=sys.stderr, flush=True)
    R = torch.from_numpy(pr.R).cuda()
    T = torch.from_numpy(pr.T).cuda()
    ctx = ngf.Context(alpha=args.alpha, tau=args.eps, rho=args.eps, levels=args.levels,
                      ratio=args.ratio,
                      max_iter=args.max_iter, lbfgs_mem=5, tol_J=1e-6, early_stop=True)
    # image-pass variants: the timed selection times its candidates for every
    # level shape when the pyramid is first built, here, before the warm-up
    # and the timed region (later pyramids of the same shapes reuse them)
    ctx.set_kernel(args.kernel)
    if args.node_grid:
        ctx.set_node_grid(args.node_grid)
    ctx.build_pyramid(R, T)
    vname = {v: k for k, v in ngf.Context.VARIANTS.items()}
    variants = [vname[ctx.get_kernel(lev)] for lev in range(args.levels)]
    print(f"[bench] image-pass variants per level: {variants}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        ctx.register(R, T)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    ctx.set_profiling(True, level=0)  # events only where the roofline is taken
    evals = 0
    reports = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y, rep = ctx.register(R, T)
        evals += sum(r["evals"] for r in rep)
        reports.append(rep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the finest level's launches of the image pass, the dominant kernel
    launches, kms, vox, _ = ctx.kernel_time(level=0)
    ctx.set_profiling(False)
    print(f"[bench] timed {args.steps} registrations in {dt:.3f}s", file=sys.stderr, flush=True)

    # finest level alone, at the registered y: 10 warm-up evaluations, then
    # the median of 5 runs of back-to-back evaluations (warm: R, T and y stay
    # in the 256 MB last-level cache); then single evaluations, each after a
    # 1 GiB device buffer has been overwritten (cold: the cache holds that
    # buffer, not the level's data), timed with events on the same stream
    li = ctx.level_info(0)
    g = torch.empty_like(y)
    for _ in range(10):
        ctx.eval_J_grad_async(0, y, g)
    torch.cuda.synchronize()
    runs = []
    for _ in range(args.finest_runs):
        t0f = time.perf_counter()
        for _ in range(args.finest_evals):
            ctx.eval_J_grad_async(0, y, g)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0f) / max(args.finest_evals, 1))
    tf = sorted(runs)[len(runs) // 2] * args.finest_evals  # median run
    flush = torch.empty(1 << 28, dtype=torch.float32, device=y.device)
    cold = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(20):
        flush.fill_(1.0)
        ev0.record()
        ctx.eval_J_grad_async(0, y, g)
        ev1.record()
        ev1.synchronize()
        cold.append(1e3 * ev0.elapsed_time(ev1))
    del flush
    cold_us = sorted(cold)[len(cold) // 2]
    N = li.m[0] * li.m[1] * li.m[2]
    Ny = li.my[0] * li.my[1] * li.my[2]
    finest_bytes = 8 * N + 24 * Ny

    # the paper's convention: registration from host arrays (pinned), with the
    # copies of R and T to the device, the pyramid and the copy of y back
    Rh, Th = R.cpu().pin_memory(), T.cpu().pin_memory()
    ctx.register(Rh, Th)
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(args.host_reps):
        ctx.register(Rh, Th)
    torch.cuda.synchronize()
    th = (time.perf_counter() - th) / max(args.host_reps, 1)
    del Rh, Th
    print(f"[bench] registration from host arrays: {th * 1e3:.1f} ms", file=sys.stderr,
          flush=True)

    # roofline of the dominant kernel (the image pass at the finest level)
    # over the timed region: it is bound by vector-ALU issue, not by HBM
    # (its traffic is a few hundred MB per launch at well under 1 TB/s)
    avg_s = kms * 1e-3 / max(launches, 1)
    flops_launch = FLOPS_PER_VOXEL * vox / max(launches, 1)
    achieved = flops_launch / avg_s / 1e12 if kms > 0 else 0.0
    khash = _src_hash()
    kname = {v: k for k, v in ngf.Context.VARIANTS.items()}[ctx.get_kernel(0)]
    traffic = _traffic(khash, shape, kname)
    out = {
        "metric": METRIC,
        "value": args.finest_evals / tf,
        "unit": "evals/s",
        "value_note": f"J + grad J evaluations per second at the {sname} finest level "
                      f"(median of {args.finest_runs} runs of {args.finest_evals} back to back "
                      "at the registered y, after 10 warm-up evaluations); "
                      "ms_per_step is one full registration (pyramid + all levels)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 coordinates and reductions)",
        "data": "synthetic: seeded CT-like phantom pair, B-spline warp (max 6 voxels)",
        "config": {"workload": f"single pair {sname} CT phantom, {args.levels}-level pyramid, "
                               f"deformation grid {'x'.join(str(v) for v in li.my)} at the "
                               f"finest level, noise {args.noise:g} HU, "
                               f"alpha={args.alpha:g}, eps={args.eps:g}, L-BFGS m=5, "
                               f"<= {args.max_iter} it/level, "
                               "early stop 1e-6",
                   "global_batch": 1, "seq_len": None, "parallelism": "single GPU"},
        "registration_s": dt / args.steps,
        "image_pass_variants": {"selection": args.kernel, "per_level": variants},
        "evals_per_registration": evals / args.steps,
        "evals_per_s_registration": evals / dt,
        "levels": reports[-1],
        "from_host": {"registration_s": th, "reps": args.host_reps,
                      "note": "pinned host R and T in, y out: includes both copies over PCIe "
                              "and the pyramid (not the metric's value)"},
        "finest": {"evals_per_s": args.finest_evals / tf,
                   "eval_us": 1e6 * tf / args.finest_evals,
                   "compulsory_bytes": finest_bytes,
                   "effective_GBs": finest_bytes * args.finest_evals / tf / 1e9,
                   "runs_us": [1e6 * r for r in runs],
                   "cold_eval_us": cold_us,
                   "cold_effective_GBs": finest_bytes / cold_us / 1e3,
                   "cold_note": "median of 20 single evaluations, each after overwriting a "
                                "1 GiB device buffer (last-level cache flushed of R, T, y)"},
        "roofline": {
            "kernel": f"image pass at the finest level (variant {kname})",
            "bound": "alu",
            "achieved": achieved,
            "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / ALU_PEAK_TFLOPS,
            "traffic": traffic,
            "launches": launches,
            "avg_launch_us": 1e6 * avg_s,
            "flops_per_launch": flops_launch,
            "flops_per_voxel": FLOPS_PER_VOXEL,
            "hbm_GBs": (traffic / avg_s / 1e9) if traffic else None,
            "hbm_frac": (traffic / avg_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
            "kernel_src": khash,
        },
    }
    if not args.no_accuracy and shape[0] * shape[1] * shape[2] <= (1 << 26):
        out["accuracy_voxels"] = accuracy(ctx, y, pr)
        out["image_mismatch_hu"] = image_mismatch(ctx, y, pr)
        print("[bench] accuracy sampled", file=sys.stderr, flush=True)
    if not args.no_forms:
        ctx.close()  # the 256^3 context's buffers are not needed any more
        del R, T
        out["forms"] = bench_forms(args, torch, ngf, synth)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, 256^3 eval)...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pr.R, pr.T)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
