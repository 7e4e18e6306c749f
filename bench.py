"""Benchmark: AB-/BA-GKB on the 512x512 fan-beam workload (720 views over
360 degrees, 1024 equiangular bins, source at twice the image width), FP32
projectors and Krylov vectors with FP64 reductions and projected solve,
150 iterations per solve.

One step = one BA-GKB solve of 150 iterations followed by one AB-GKB solve of
150 iterations on the same synthetic sinogram (random-ellipse phantom,
0.5 % Gaussian noise), with the discrepancy test evaluated every iteration.
value = GKB iterations per second over the timed steps.

Also reported: per-projector device time (HIP events on the library's
stream), the dominant kernel's roofline position, the projector
throughput in GB/s against the HBM peak, and the CPU oracle timed on a
bounded sample of the same workload.

Batched workload (the "s/slice to discrepancy" part of the metric): 64
parallel-beam slices, n = 128 + 32 U{0..12}, 180 + 30 U{0..18} views,
ceil(n sqrt 2) bins, 0.5-5 % noise, BA-GKB with the discrepancy stop
(tau = 1, k_max = 150) per slice; timed once solved one slice after another
and once as one batched call, after an untimed pass of each that builds the
geometry tables.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch]
                  [--only-headline | --only-batch | --cone | --learned]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

K_ITERS = 150
HBM_PEAK_GBS = 8000.0
# FP32 vector FMA rate without packed math: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# flops per algorithmic unit: ray-driven kernels 2 FMA per dominant-line
# crossing; pixel-driven kernels 3 FMA per (pixel, view) pair
FLOPS_PER_UNIT = {"fwd": 4.0, "back_adj": 4.0, "back": 6.0, "fwd_adj": 6.0}
OPERAND_BYTES_PER_UNIT = 8.0  # two FP32 taps
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (each
# scaled by the plain-copy calibration), profiles/fan512_gkb_hbm_traffic.txt.
# An entry must be removed when its kernel changes.
MEASURED_TRAFFIC = {"fwd": (14860.2 * 1.9855 + 8785.3) * 1024.0, "back": (8322.4 * 1.9855 + 2952.5) * 1024.0,
                    "fwd_adj": (22211.3 * 1.9855 + 2062.2) * 1024.0, "back_adj": (21661.7 * 1.9855 + 5938.4) * 1024.0}


def joseph_crossings(geom) -> int:
    """Number of (ray, dominant line) pairs with a tap inside the image: the
    terms of Joseph's sum for this geometry (fan or parallel, 2D)."""
    from paper_2606_31153_amd import synth
    nx, ny, nu = geom.nx, geom.ny, geom.n_det_u
    off = (nu - 1) / 2.0
    k = np.arange(nu) - off
    total = 0
    for ang in geom.view_angles():
        if geom.kind == synth.KIND_FAN2D:
            g = k * geom.det_pitch_u
            dx, dy = -np.cos(ang + g), -np.sin(ang + g)
            sx = np.full(nu, geom.src_dist * math.cos(ang))
            sy = np.full(nu, geom.src_dist * math.sin(ang))
        else:
            dx = np.full(nu, -math.sin(ang))
            dy = np.full(nu, math.cos(ang))
            s = k * geom.det_pitch_u
            sx, sy = s * math.cos(ang), s * math.sin(ang)
        rowdom = np.abs(dy) >= np.abs(dx)
        # crossings with rows (row-dominant rays) or columns
        lines_r = np.arange(ny) - (ny - 1) / 2.0
        lines_c = np.arange(nx) - (nx - 1) / 2.0
        with np.errstate(divide="ignore", invalid="ignore"):
            xr = (sx[:, None] + (lines_r[None, :] - sy[:, None]) * (dx / dy)[:, None]) + (nx - 1) / 2.0
            yc = (sy[:, None] + (lines_c[None, :] - sx[:, None]) * (dy / dx)[:, None]) + (ny - 1) / 2.0
        inr = ((xr > -1.0) & (xr < nx)).sum(axis=1)
        inc = ((yc > -1.0) & (yc < ny)).sum(axis=1)
        total += int(np.where(rowdom, inr, inc).sum())
    return total


def make_problem(geom, seed: int, nu: float):
    """Phantom and noisy sinogram on the GPU (forward projector of the
    library), noise scaled to nu*||b_true||."""
    import torch

    import paper_2606_31153_amd as gk
    from paper_2606_31153_amd import synth
    dev = torch.device("cuda:0")
    ctx = gk.Context(0)
    x_true = torch.tensor(synth.ellipse_phantom(geom.nx, seed), dtype=torch.float32, device=dev).reshape(-1)
    b_true = torch.empty(geom.m, dtype=torch.float32, device=dev)
    gk.gkb_forward(ctx, geom, x_true, b_true)
    torch.cuda.synchronize()
    bt = b_true.double().cpu().numpy()
    b, enorm = synth.add_noise(bt, synth.noise_direction(geom.m, seed), nu)
    ctx.close()
    return x_true, torch.tensor(b, dtype=torch.float32, device=dev), enorm


def batch_problems(count: int = 64):
    """The 64-slice workload: per-slice geometry, device b (FP32) and ||e||."""
    import torch

    import paper_2606_31153_amd as gk
    from paper_2606_31153_amd import synth
    dev = torch.device("cuda:0")
    ctx = gk.Context(0)
    geoms, bs, ens = [], [], []
    for (n, v, nu, seed) in synth.batch_slices(3000, count):
        g = synth.par2d(n, v)
        x = torch.tensor(synth.ellipse_phantom(n, seed).reshape(-1), dtype=torch.float32, device=dev)
        y = torch.empty(g.m, dtype=torch.float32, device=dev)
        gk.gkb_forward(ctx, g, x, y)
        torch.cuda.synchronize()
        b, en = synth.add_noise(y.double().cpu().numpy(), synth.noise_direction(g.m, seed), nu)
        geoms.append(g)
        bs.append(torch.tensor(b, dtype=torch.float32, device=dev))
        ens.append(en)
    ctx.close()
    return geoms, bs, ens


def batch_bench(ctx):
    import torch

    import paper_2606_31153_amd as gk
    geoms, bs, ens = batch_problems()
    xs = [torch.zeros(g.n, dtype=torch.float32, device=b.device) for g, b in zip(geoms, bs)]
    opts = [dict(k_max=150, use_dp=True, tau=1.0, noise_norm=e) for e in ens]

    def sequential():
        return [gk.gkb_ba_solve(ctx, g, b, x, **o) for g, b, x, o in zip(geoms, bs, xs, opts)]

    def batched(mode=gk.GKB_BATCH_LAUNCHES):
        ctx.set_batch_mode(mode)
        try:
            return gk.gkb_batch_solve(ctx, gk.GKB_METHOD_BA, geoms, bs, xs, opts)
        finally:
            ctx.set_batch_mode(gk.GKB_BATCH_LAUNCHES)

    def timed(f, *a):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f(*a)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # launch shapes with the library's defaults, then autotuned per slice
    # geometry (the tuning itself is not timed)
    for g in geoms:
        gk.gkb_set_tuning(ctx, g, 1, 4)
    batched()
    _, t_untuned = timed(batched)
    t0 = time.perf_counter()
    tunes = [gk.gkb_autotune(ctx, g) for g in geoms]
    t_tune = time.perf_counter() - t0
    sequential()
    batched()
    batched(gk.GKB_BATCH_GRAPH)
    rs, t_seq = timed(sequential)
    rb, t_bat = timed(batched)
    rg, t_graph = timed(batched, gk.GKB_BATCH_GRAPH)
    ks = [r.k_stop for r in rb]
    assert ks == [r.k_stop for r in rs] == [r.k_stop for r in rg]
    ns = len(geoms)
    return {"workload": "64 parallel-beam slices, n 128..512, 180..720 views, 0.5-5% noise, BA-GKB, DP tau=1",
            "slices": ns, "s_per_slice_batched": t_bat / ns, "s_per_slice_sequential": t_seq / ns,
            "s_per_slice_batched_graph": t_graph / ns,
            "s_per_slice_batched_one_view_per_step": t_untuned / ns,
            "autotune": {"seconds": t_tune,
                         "at_views_per_step": [t.at_views_per_step for t in tunes],
                         "b_views_per_step": [t.b_views_per_step for t in tunes]},
            "batched_speedup": t_seq / t_bat, "iterations_mean": float(np.mean(ks)),
            "iterations_min": int(min(ks)), "iterations_max": int(max(ks)),
            "stopped_by_dp": sum(1 for r in rb if r.reason == gk.STOP_DP),
            "pixels_total": int(sum(g.n for g in geoms)), "bins_total": int(sum(g.m for g in geoms))}


def cone_units(geom) -> int:
    """Joseph-3D samples of A (= nonzero bilinear stencils of A and A^T): the
    (ray, plane) pairs whose crossing lies inside the volume.  Per ray the
    planes with the in-plane crossing inside and those with the height inside
    are two intervals; the count is the length of their intersection."""
    nx, ny, nz, nu, nw = geom.nx, geom.ny, geom.nz, geom.n_det_u, geom.n_det_v
    D, SDD, du, dw = geom.src_dist, geom.src_det_dist, geom.det_pitch_u, geom.det_pitch_v
    uu = (np.arange(nu) - (nu - 1) / 2.0) * du
    vv = (np.arange(nw) - (nw - 1) / 2.0) * dw
    total = 0

    def interval(c0, c1, lo, hi):
        # integers t with lo < c0 + c1 t < hi
        with np.errstate(divide="ignore", invalid="ignore"):
            ta, tb = (lo - c0) / c1, (hi - c0) / c1
        a, b = np.minimum(ta, tb), np.maximum(ta, tb)
        flat = c1 == 0
        inside = (c0 > lo) & (c0 < hi)
        a = np.where(flat, np.where(inside, -np.inf, np.inf), a)
        b = np.where(flat, np.where(inside, np.inf, -np.inf), b)
        return np.floor(a) + 1, np.ceil(b) - 1

    for b in geom.view_angles():
        cb, sb = math.cos(b), math.sin(b)
        Sx, Sy = D * cb, D * sb
        dx = -SDD * cb - uu * sb
        dy = -SDD * sb + uu * cb
        ydom = np.abs(dy) > np.abs(dx)
        dax = np.where(ydom, dy, dx)
        dob = np.where(ydom, dx, dy)
        nax = np.where(ydom, ny, nx)
        n1 = np.where(ydom, nx, ny)
        lam0 = (-(nax - 1) / 2.0 - np.where(ydom, Sy, Sx)) / dax  # lambda at plane 0
        p10 = np.where(ydom, Sx, Sy) + lam0 * dob + (n1 - 1) / 2.0
        p1s = dob / dax
        lo1, hi1 = interval(p10, p1s, -1.0, n1)
        lo1 = np.maximum(lo1, 0)
        hi1 = np.minimum(hi1, nax - 1)
        lo2, hi2 = interval(lam0[:, None] * vv[None, :] + (nz - 1) / 2.0, (1.0 / dax)[:, None] * vv[None, :],
                            -1.0, nz)
        lo = np.maximum(lo1[:, None], lo2)
        hi = np.minimum(hi1[:, None], hi2)
        total += int(np.clip(hi - lo + 1, 0, None).sum())
    return total


def cone_main(args):
    """512^3 cone beam (720 views, 1024 x 768 flat detector, D = 1024,
    SDD = 2048): the four projectors and BA-GKB iterations."""
    import torch

    import paper_2606_31153_amd as gk
    from paper_2606_31153_amd import synth
    dev = torch.device("cuda:0")
    geom = synth.cone3d(512, 720, 1024, 768)
    print("bench: cone phantom", file=sys.stderr, flush=True)
    xt = torch.from_numpy(synth.rasterize_ellipsoids(synth.ellipsoid_params(5000), 512).reshape(-1)).to(dev)
    ctx = gk.Context(0)
    bt = torch.empty(geom.m, dtype=torch.float32, device=dev)
    gk.gkb_forward(ctx, geom, xt, bt)
    torch.cuda.synchronize()
    print("bench: cone noise", file=sys.stderr, flush=True)
    b, enorm = synth.add_noise(bt.double().cpu().numpy(), synth.noise_direction(geom.m, 5000), 0.01)
    bd = torch.from_numpy(b.astype(np.float32)).to(dev)
    del b
    x = torch.empty(geom.n, dtype=torch.float32, device=dev)
    y = torch.empty(geom.m, dtype=torch.float32, device=dev)
    calls = {"fwd": lambda: gk.gkb_forward(ctx, geom, xt, y), "back": lambda: gk.gkb_back(ctx, geom, bd, x),
             "fwd_adj": lambda: gk.gkb_forward_adjoint(ctx, geom, bd, x),
             "back_adj": lambda: gk.gkb_back_adjoint(ctx, geom, xt, y)}
    for f in calls.values():
        f()
    torch.cuda.synchronize()
    ctx.trace_enable(True)
    ctx.trace_reset()
    for _ in range(args.steps):
        for f in calls.values():
            f()
    torch.cuda.synchronize()
    kernels = {}
    for name in calls:
        cnt, ms = ctx.trace_get(name)
        kernels[name] = {"launches": cnt, "avg_ms": ms / cnt}
    ctx.trace_enable(False)
    print("bench: cone BA-GKB", file=sys.stderr, flush=True)
    iters = args.cone_iters
    t0 = time.perf_counter()
    r = gk.gkb_ba_solve(ctx, geom, bd, x, iters, use_dp=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # BA-GKB with a sinogram filter inside B applied per detector row (M = B F A,
    # F the Ram-Lak filter carried exactly by the learned-filter network and its
    # kernels): the cost per iteration of the per-row F at this size
    print("bench: cone BA-GKB with a per-row filter", file=sys.stderr, flush=True)
    from paper_2606_31153_amd import learned
    net = gk.Net(ctx)
    net.set_weights(learned.linear_pair_weights(learned.ramlak()))
    fiters = max(1, min(iters, args.cone_filter_iters))
    t0 = time.perf_counter()
    rf = gk.gkb_ba_solve(ctx, geom, bd, x, fiters, use_dp=False, precond=net)
    torch.cuda.synchronize()
    elf = time.perf_counter() - t0
    net.close()
    print("bench: cone units", file=sys.stderr, flush=True)
    units = cone_units(geom)
    pv = geom.n * geom.n_views
    u = {"fwd": units, "fwd_adj": units, "back": pv, "back_adj": pv}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    ach = u[dom] * 8.0 / (kernels[dom]["avg_ms"] / 1e3) / 1e12
    out = {"metric": "cone 512^3: BA-GKB iters/s; projector time per call", "value": r.k_stop / el,
           "unit": "GKB iters/s", "n_gpus": 1, "iterations": r.k_stop, "seconds": el,
           "higher_is_better": True, "dtype": "f32 vectors/projectors, f64 reductions and projected solve",
           "data": "synthetic: seeded 8-ellipsoid phantom, 1% Gaussian noise",
           "config": {"workload": "cone beam 512^3, 720 views over 360 deg, 1024x768 flat detector, D=1024, "
                                  "SDD=2048; BA-GKB %d iterations" % iters},
           "kernels": kernels, "units": {"joseph_samples": units, "voxel_views": pv},
           "per_row_filter": {"filter": "Ram-Lak (9 taps) through the learned-filter network, per detector row "
                                        "(720 x 768 rows of 1024 bins), inside B", "iterations": rf.k_stop,
                              "iters_per_s": rf.k_stop / elf, "plain_iters_per_s": r.k_stop / el},
           "roofline": {"bound": "alu", "kernel": dom, "achieved": ach, "peak": VALU_FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / VALU_FP32_PEAK_TFLOPS,
                        "work_per_launch": "%d units x 8 flop (bilinear: 3 lerps + accumulate)" % u[dom]}}
    ctx.close()
    print(json.dumps(out))


def learned_main(args):
    """Learned filter: train on 256^2 / 360-view parallel-beam samples (1-5 %
    noise), evaluate on 16 held-out 512^2 / 720-view slices against plain
    BA-GKB at the same discrepancy stop."""
    import torch

    import paper_2606_31153_amd as gk
    from paper_2606_31153_amd import learned, synth

    def log(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    ctx = gk.Context(0)
    tg, eg = synth.par2d(256, 360), synth.par2d(512, 720)
    t0 = time.perf_counter()
    log("training set (%d samples)" % args.train_samples)
    bd, xd, tn = learned.make_set(ctx, tg, range(4_000_000, 4_000_000 + args.train_samples), 0.01, 0.05, 4_000_000)
    if args.targets == "gkb":
        log("targets: plain BA-GKB discrepancy solutions")
        xd = learned.gkb_targets(ctx, tg, bd, tn)
    if args.textures > 0:
        log("texture samples (%d)" % args.textures)
        bt, xt = learned.make_textures(ctx, tg, args.textures, 4_200_000, 0.01, 0.05)
        bd, xd = torch.cat([bd, bt]), torch.cat([xd, xt])
        del bt, xt
    t_data = time.perf_counter() - t0
    net = gk.Net(ctx, seed=4_000_000)
    net.set_weights(learned.init_weights(4_000_000, noise=args.init_noise,
                                         first=learned.ramlak() if args.init == "ramlak" else None))
    learned.rescale_output(ctx, net, tg, bd, xd)
    t0 = time.perf_counter()
    objective = gk.GKB_NET_FROZEN if args.objective == "frozen" else gk.GKB_NET_FBP
    losses = learned.train(ctx, net, tg, bd, xd, args.epochs, args.batch, args.lr, seed=4_000_000, log=log,
                           objective=objective)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = args.epochs * (args.train_samples // args.batch)
    del bd, xd
    log("evaluation set")
    eb, ex, en = learned.make_set(ctx, eg, range(4_100_000, 4_100_016), 0.01, 0.05, 4_100_000)
    ev = learned.evaluate(ctx, net, eg, eb, ex, en)
    if args.save_filter:
        net.save(args.save_filter)
    # control: the same kernels with the network set to the analytic Ram-Lak
    # filter (a linear filter, exactly, whatever the masks)
    log("Ram-Lak control")
    ctl = gk.Net(ctx, seed=0)
    ctl.set_weights(learned.linear_pair_weights(learned.ramlak()))
    evc = learned.evaluate(ctx, ctl, eg, eb, ex, en)
    ctl.close()
    out = {"metric": "learned vs plain BA-GKB: s/slice to discrepancy at 512^2, 720 views",
           "value": ev["speedup_s_per_slice"], "unit": "x (plain s/slice / learned s/slice)",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f32 vectors, bf16-MFMA filter (3-term split)",
           "data": "synthetic: seeded ellipse phantoms, 1-5% Gaussian noise",
           "config": {"workload": "train 256^2/360 views/363 bins, %d samples, %d epochs, batch %d, lr %g; "
                                  "evaluate 16 slices 512^2/720 views/725 bins, DP tau=1, k_max 150; "
                                  "%d random-texture samples; init %s + %g He noise; objective %s; targets %s"
                                  % (args.train_samples, args.epochs, args.batch, args.lr, args.textures, args.init,
                                     args.init_noise, args.objective, args.targets)},
           "training": {"seconds_data": t_data, "seconds_train": t_train, "steps": steps,
                        "ms_per_step": 1e3 * t_train / max(steps, 1), "loss_per_epoch": losses},
           "plain": ev["plain"], "learned": ev["learned"],
           "learned_over_plain_s_per_slice": ev["learned"]["s_per_slice"] / ev["plain"]["s_per_slice"],
           "ramlak_control": {"filter": evc["learned"], "speedup_s_per_slice": evc["speedup_s_per_slice"],
                              "plain": evc["plain"]},
           "learned_min_residual_over_e": [r["learned_free"]["min_res_over_e"] for r in ev["slices"]],
           "target_over_e_mean": ev["target_over_e_mean"],
           "per_slice": [{k: ({kk: v[kk] for kk in ("k", "seconds", "rre", "res_over_e")}
                              if isinstance(v, dict) and "k" in v else v) for k, v in r.items()}
                         for r in ev["slices"]]}
    net.close()
    ctx.close()
    print(json.dumps(out))


def cpu_baseline(geom, b_host: np.ndarray, enorm: float, iters: int, runs: int):
    import oracle
    op = oracle.Operator(geom)
    rates = []
    for _ in range(runs):
        t0 = time.perf_counter()
        res = oracle.gkb(op, oracle.MODE_BA, b_host, iters)
        rates.append(res.k_stop / (time.perf_counter() - t0))
    cores = oracle.num_threads()
    # the same problem on one thread: 2 iterations
    oracle.set_threads(1)
    t0 = time.perf_counter()
    res1 = oracle.gkb(op, oracle.MODE_BA, b_host, 2)
    one = res1.k_stop / (time.perf_counter() - t0)
    oracle.set_threads(cores)
    return {"value": float(np.mean(rates)), "unit": "GKB iters/s", "cores": cores, "kind": "oracle",
            "median": float(np.median(rates)), "runs": runs,
            "single_thread": {"value": one, "iterations": 2},
            "sample": "FP64 CPU oracle (OpenMP, all host threads), BA-GKB, %d runs of %d iterations of the same "
                      "fan-beam 512^2/720/1024 problem, each iteration with its residual ||A x_k - b|| evaluated "
                      "literally (one more A and a Q u product); value = mean and median over the runs of "
                      "iterations/s; a 150-iteration run takes minutes, so the sample is short" % (runs, iters)}


def par512_point(ctx, iters: int):
    """AB- and BA-GKB iterations/s on the 512x512 parallel-beam workload
    (720 views over 180 degrees, 725 bins), the second image size of the
    timing experiments (context beside the fan-beam headline)."""
    import torch

    import paper_2606_31153_amd as gk
    from paper_2606_31153_amd import synth
    geom = synth.workload_par512()
    _, b, enorm = make_problem(geom, 2000, 0.005)
    x = torch.zeros(geom.n, dtype=torch.float32, device=b.device)
    gk.gkb_autotune(ctx, geom)
    out = {"workload": "parallel beam 512x512, 720 views over 180 deg, 725 bins; %d iterations" % iters}
    for name, fn in (("ba", gk.gkb_ba_solve), ("ab", gk.gkb_ab_solve)):
        fn(ctx, geom, b, x, iters)
        torch.cuda.synchronize()
        r = fn(ctx, geom, b, x, iters)
        torch.cuda.synchronize()
        out["%s_iters_per_s" % name] = iters / r.seconds
    return out


def gmres_point(ctx, geom, b, iters: int):
    """The paper's comparison methods on the benchmark workload (context)."""
    import torch

    import paper_2606_31153_amd as gk
    x = torch.zeros(geom.n, dtype=torch.float32, device=b.device)
    out = {"workload": "fan-beam 512x512 as above; %d iterations" % iters}
    for name, fn in (("ba_gmres", gk.gkb_ba_gmres_solve), ("ab_gmres", gk.gkb_ab_gmres_solve)):
        fn(ctx, geom, b, x, iters)
        torch.cuda.synchronize()
        r = fn(ctx, geom, b, x, iters)
        torch.cuda.synchronize()
        out["%s_iters_per_s" % name] = iters / r.seconds
    return out


def hybrid_point(ctx, geom, b, iters: int):
    """Hybrid BA-GKB (lambda_k on C_k by the projected discrepancy rule or GCV)
    and the enlarged-subspace TSVD on the benchmark workload: iterations/s
    beside plain BA-GKB, the same number of iterations."""
    import torch

    import paper_2606_31153_amd as gk
    x = torch.zeros(geom.n, dtype=torch.float32, device=b.device)
    out = {"workload": "fan-beam 512x512 as above; BA-GKB, %d iterations" % iters}
    for name, kw in (("plain", None), ("hybrid_dp", dict(rule=gk.GKB_LAMBDA_DP, eta_proj=1.0)),
                     ("hybrid_gcv", dict(rule=gk.GKB_LAMBDA_GCV)), ("tsvd_rank100", dict(tsvd_rank=100))):
        fn = gk.gkb_ba_solve if kw is None else gk.gkb_ba_hybrid_solve
        kw = kw or {}
        fn(ctx, geom, b, x, iters, **kw)
        torch.cuda.synchronize()
        r = fn(ctx, geom, b, x, iters, **kw)
        torch.cuda.synchronize()
        out["%s_iters_per_s" % name] = iters / r.seconds
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=K_ITERS)
    ap.add_argument("--cpu-iters", type=int, default=4)
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="the timed fan-beam steps and kernel table only (for profiling its kernels)")
    ap.add_argument("--only-batch", action="store_true", help="the 64-slice batched workload only (profiling)")
    ap.add_argument("--cone", action="store_true", help="measure the 512^3 cone-beam workload instead")
    ap.add_argument("--cone-iters", type=int, default=60)
    ap.add_argument("--cone-filter-iters", type=int, default=10,
                    help="iterations of the cone solve with the per-row filter")
    ap.add_argument("--learned", action="store_true", help="train and evaluate the learned filter instead")
    ap.add_argument("--train-samples", type=int, default=20000)
    ap.add_argument("--save-filter", default="", help="with --learned: write the trained network's weights to this file")
    ap.add_argument("--textures", type=int, default=0, help="extra random-texture training samples")
    ap.add_argument("--init", choices=("identity", "ramlak"), default="identity")
    ap.add_argument("--objective", choices=("fbp", "frozen"), default="frozen")
    ap.add_argument("--init-noise", type=float, default=0.1)
    ap.add_argument("--epochs", type=int, default=5)
    ap.add_argument("--targets", choices=("truth", "gkb"), default="truth",
                    help="training targets: the phantoms, or plain BA-GKB discrepancy solutions")
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-4)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.cone:
        cone_main(args)
        return
    if args.learned:
        learned_main(args)
        return
    if args.only_batch:  # the batched workload alone (profiling)
        import paper_2606_31153_amd as gk
        ctx = gk.Context(0)
        res = batch_bench(ctx)
        ctx.close()
        print(json.dumps({"metric": "s/slice to discrepancy, 64-slice batched workload",
                          "value": res["s_per_slice_batched"], "unit": "s/slice", "higher_is_better": False,
                          "n_gpus": 1, "s_per_slice_to_discrepancy": res}))
        return

    import torch

    import paper_2606_31153_amd as gk
    from paper_2606_31153_amd import synth

    geom = synth.workload_fan512()
    dev = torch.device("cuda:0")
    print("bench: building problem", file=sys.stderr, flush=True)
    x_true, b, enorm = make_problem(geom, 2000, 0.005)
    x = torch.zeros(geom.n, dtype=torch.float32, device=dev)
    ctx = gk.Context(0)
    kw = dict(use_dp=False, tau=1.0, noise_norm=enorm)

    def step():
        r1 = gk.gkb_ba_solve(ctx, geom, b, x, args.iters, **kw)
        r2 = gk.gkb_ab_solve(ctx, geom, b, x, args.iters, **kw)
        return r1, r2

    for i in range(args.warmup):
        step()
        print("bench: warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # per-kernel breakdown from one untimed step with every kernel bracketed by
    # HIP events (each pair costs the stream a few microseconds between
    # launches, so the timed steps below record the dominant kernel only)
    ctx.trace_enable(True)
    ctx.trace_reset()
    step()
    torch.cuda.synchronize()
    ctx.trace_enable(False)
    kernels = {}
    for name in ("fwd", "back", "fwd_adj", "back_adj", "reorth", "small_solve", "residual"):
        cnt, ms = ctx.trace_get(name)
        if cnt:
            kernels[name] = {"launches": cnt, "avg_ms": ms / cnt, "total_ms": ms}
    # algorithmic units per launch
    cross = joseph_crossings(geom)
    pv = geom.n * geom.n_views
    units = {"fwd": cross, "back_adj": cross, "back": pv, "fwd_adj": pv}
    proj = {k: v for k, v in kernels.items() if k in units}
    dom = max(proj, key=lambda k: proj[k]["total_ms"])
    print("bench: breakdown step done, dominant kernel %s" % dom, file=sys.stderr, flush=True)

    # timed region: HIP events around the dominant kernel's launches only
    ctx.trace_only(dom)
    ctx.trace_enable(True)
    ctx.trace_reset()
    t0 = time.perf_counter()
    ba_s = ab_s = 0.0
    for i in range(args.steps):
        r1, r2 = step()
        ba_s += r1.seconds
        ab_s += r2.seconds
        print("bench: step %d done (BA %.3f s, AB %.3f s)" % (i, r1.seconds, r2.seconds), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.trace_enable(False)
    ctx.trace_only(None)
    cnt, ms = ctx.trace_get(dom)
    t_dom = ms / cnt / 1e3
    ach = units[dom] * FLOPS_PER_UNIT[dom] / t_dom / 1e12
    gbps = {}
    for k, v in proj.items():
        t = v["avg_ms"] / 1e3
        comp = 4.0 * (geom.n + geom.m) / t / 1e9
        oper = units[k] * OPERAND_BYTES_PER_UNIT / t / 1e9
        gbps[k] = {"avg_us": v["avg_ms"] * 1e3, "units": units[k], "compulsory_GBs": comp,
                   "compulsory_pct_hbm": 100 * comp / HBM_PEAK_GBS,
                   # two FP32 taps per unit, served from L1/LDS/L2: a cache-bandwidth figure, not HBM
                   "operand_cache_GBs": oper}
        if k in MEASURED_TRAFFIC:
            hb = MEASURED_TRAFFIC[k] / t / 1e9
            gbps[k]["measured_hbm_GBs"] = hb
            gbps[k]["measured_hbm_pct"] = 100 * hb / HBM_PEAK_GBS

    iters = 2 * args.iters * args.steps
    out = {
        "metric": "GKB iters/s and projector GB/s (% HBM roofline) at 512^2; s/slice to discrepancy",
        "value": iters / elapsed,
        "unit": "GKB iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 vectors/projectors, f64 reductions and projected solve",
        "data": "synthetic: seeded random-ellipse phantom, 0.5% Gaussian noise",
        "config": {"workload": "fan-beam 512x512, 720 views over 360 deg, 1024 equiangular bins, D=1024; "
                               "BA-GKB then AB-GKB, %d iterations each" % args.iters,
                   "iterations_per_step": 2 * args.iters},
        "ba_iters_per_s": args.iters * args.steps / ba_s,
        "ab_iters_per_s": args.iters * args.steps / ab_s,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": ach, "peak": VALU_FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / VALU_FP32_PEAK_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get(dom),
                     "work_per_launch": "%d units x %g flop" % (units[dom], FLOPS_PER_UNIT[dom]),
                     "avg_us_timed_region": t_dom * 1e6, "launches_timed_region": cnt},
        "projector_gbps": gbps,
        "kernels": kernels,
        "kernels_source": "one untimed step with every kernel bracketed by HIP events",
    }
    if args.only_headline:  # profiling the headline kernels alone
        ctx.close()
        print(json.dumps(out))
        return
    print("bench: parallel-beam 512 point", file=sys.stderr, flush=True)
    out["par512"] = par512_point(ctx, args.iters)
    print("bench: GMRES on the benchmark workload", file=sys.stderr, flush=True)
    out["gmres"] = gmres_point(ctx, geom, b, args.iters)
    print("bench: hybrid regularisation and TSVD on the benchmark workload", file=sys.stderr, flush=True)
    out["hybrid"] = hybrid_point(ctx, geom, b, args.iters)
    if not args.no_batch:
        print("bench: 64-slice batched workload", file=sys.stderr, flush=True)
        out["s_per_slice_to_discrepancy"] = batch_bench(ctx)
    if not args.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(geom, b.double().cpu().numpy(), enorm, args.cpu_iters, args.cpu_runs)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
