"""Training and evaluation of the learned sinogram filter inside B (BA-GKB).

Training set: seeded random-ellipse phantoms x_i (parallel beam, n x n
pixels, V views, ceil(n sqrt 2) bins), b_i = A x_i + e_i with the library's
own forward projector and Gaussian noise at a level nu_i ~ U[nu_lo, nu_hi]
(relative to ||A x_i||).  Loss: ||B N(b_i) - x_i||^2 / ||x_i||^2, Adam,
mini-batches drawn by a seeded permutation per epoch.

Evaluation: held-out phantoms at the evaluation geometry; plain BA-GKB and
BA-GKB with the trained filter, both stopped by the discrepancy principle
(tau = 1, the same ||e||), so both end at the same residual level; the
comparison is iterations, wall-clock seconds per slice and the relative
reconstruction error ||x - x_true|| / ||x_true||.
"""
from __future__ import annotations

import multiprocessing as mp
import time

import numpy as np

from . import synth


def _phantom(args):
    n, seed = args
    return synth.ellipse_phantom(n, seed).astype(np.float32)


def _texture(args):
    n, seed = args
    return synth.gaussian_texture(n, seed).astype(np.float32)


def _noisy(ctx, geom, xd, seeds, nus):
    """b_i = A x_i + e_i for the device images xd [N, n]: A x_i by the
    library's forward projector, then, on the host in float64, the noise of
    sample seeds[i] (synth.noise_direction) at level nus[i] relative to
    ||A x_i|| (synth.add_noise).  Returns device b [N, m] (FP32) and ||e_i||."""
    import torch

    import paper_2606_31153_amd as gk
    N, m = xd.shape[0], geom.m
    bd = torch.empty(N, m, dtype=torch.float32, device=xd.device)
    enorm = np.zeros(N)
    chunk = max(1, (1 << 27) // m)
    tmp = torch.empty(min(N, chunk), m, dtype=torch.float32, device=xd.device)
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        for i in range(c0, c1):
            gk.gkb_forward(ctx, geom, xd[i], tmp[i - c0])
        torch.cuda.synchronize()
        bt = tmp[:c1 - c0].cpu().numpy()
        out = np.empty_like(bt)
        for i in range(c0, c1):
            b, enorm[i] = synth.add_noise(bt[i - c0], synth.noise_direction(m, int(seeds[i])), float(nus[i]))
            out[i - c0] = b
        bd[c0:c1].copy_(torch.from_numpy(out))
    torch.cuda.synchronize()
    return bd, enorm


def phantoms(n: int, seeds, workers: int = 16) -> np.ndarray:
    """[len(seeds), n*n] float32 phantoms, generated in a pool of processes
    (spawned, so that no child inherits a GPU context)."""
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 64:
        return np.stack([_phantom((n, s)).reshape(-1) for s in seeds])
    with mp.get_context("spawn").Pool(workers) as pool:
        out = pool.map(_phantom, [(n, s) for s in seeds], chunksize=max(1, len(seeds) // (4 * workers)))
    return np.stack([o.reshape(-1) for o in out])


def make_set(ctx, geom, seeds, nu_lo: float, nu_hi: float, key: int, workers: int = 16):
    """Device tensors b [N, m], x [N, n] (FP32) and the noise norms ||e_i||.
    Noise levels from the Philox stream keyed (key, batch); each sample's
    noise direction from its own seed (synth.noise_direction)."""
    import torch

    dev = torch.device("cuda:0")
    seeds = list(seeds)
    X = phantoms(geom.nx, seeds, workers)
    xd = torch.from_numpy(X).to(dev)
    nus = synth.rng(key, synth.PURPOSE_BATCH).uniform(nu_lo, nu_hi, len(seeds))
    bd, enorm = _noisy(ctx, geom, xd, seeds, nus)
    return bd, xd, enorm


def gkb_targets(ctx, geom, bd, enorms, k_max: int = 150):
    """Training targets from plain BA-GKB: the discrepancy-principle solution
    (tau = 1, the sample's own ||e_i||) of every sample, [N, n] FP32 on the
    device (the smallest-residual iterate where the level is not reached)."""
    import torch

    import paper_2606_31153_amd as gk
    N = bd.shape[0]
    out = torch.empty(N, geom.n, dtype=torch.float32, device=bd.device)
    for i in range(N):
        r = gk.gkb_ba_solve(ctx, geom, bd[i], out[i], k_max, use_dp=True, tau=1.0, noise_norm=float(enorms[i]))
        if r.reason != gk.STOP_DP and r.rho.size:
            kb = int(np.argmin(r.rho)) + 1
            gk.gkb_ba_solve(ctx, geom, bd[i], out[i], kb)
    torch.cuda.synchronize()
    return out


def ramlak(K: int = 9) -> np.ndarray:
    """The Ram-Lak (ramp) filter of filtered back projection for unit bin
    pitch, truncated to K taps: h(0) = 1/4, h(k) = -1/(pi k)^2 for odd k,
    0 for even k != 0."""
    h = np.zeros(K)
    for k in range(-(K // 2), K // 2 + 1):
        h[k + K // 2] = 0.25 if k == 0 else (-1.0 / (np.pi * k) ** 2 if k % 2 else 0.0)
    return h


def init_weights(seed: int, noise: float = 0.1, first=None) -> np.ndarray:
    """A linear filter path plus scaled He noise: channel 0 carries f * y
    and channel 1 carries -f * y through the ReLUs (relu(z) - relu(-z) = z),
    the middle layers pass the pair on, the last layer takes their
    difference, so the network starts as the linear filter f (the identity
    by default, or e.g. the Ram-Lak filter); the other weights are
    N(0, 2 / fan_in) times `noise`."""
    C, K, h = 32, 9, 4
    g = synth.rng(seed, synth.PURPOSE_PHANTOM)
    shapes = [(C, 1, K), (C, C, K), (C, C, K), (1, C, K)]
    Ws = [g.standard_normal(s) * noise * np.sqrt(2.0 / (s[1] * s[2])) for s in shapes]
    f = np.eye(1, K, h)[0] if first is None else np.asarray(first, dtype=np.float64)
    Ws[0][0, 0, :] += f
    Ws[0][1, 0, :] -= f
    for l in (1, 2):
        Ws[l][0, 0, h] += 1.0
        Ws[l][1, 1, h] += 1.0
    Ws[3][0, 0, h] += 1.0
    Ws[3][0, 1, h] -= 1.0
    return np.concatenate([W.reshape(-1) for W in Ws]).astype(np.float32)


def rescale_output(ctx, net, geom, bd, xd, count: int = 16):
    """Scale the weights so that ||B N(b)|| matches ||x|| on the first
    samples.  N is positively homogeneous of degree one in the weights of
    every layer, so the gain s is spread as s^(1/4) over the four layers
    (keeping their magnitudes, which Adam's step sizes are relative to,
    balanced)."""
    import torch

    import paper_2606_31153_amd as gk
    y = torch.empty(geom.m, dtype=torch.float32, device=bd.device)
    xb = torch.empty(geom.n, dtype=torch.float32, device=bd.device)
    num = den = 0.0
    for i in range(min(count, bd.shape[0])):
        gk.gkb_net_apply(ctx, net, geom, bd[i], y)
        gk.gkb_back(ctx, geom, y, xb)
        torch.cuda.synchronize()
        num += float(np.linalg.norm(xd[i].cpu().numpy().astype(np.float64)))
        den += float(np.linalg.norm(xb.cpu().numpy().astype(np.float64)))
    w = net.get_weights()
    net.set_weights(w * np.float32((num / den) ** 0.25))


def make_textures(ctx, geom, count: int, key: int, nu_lo: float, nu_hi: float, workers: int = 16):
    """Random-texture training samples: Gaussian random fields with a random
    correlation length (synth.gaussian_texture, seeds key + i), b = A z +
    noise as in make_set.  Returns device b [count, m], z [count, n]."""
    import torch

    dev = torch.device("cuda:0")
    seeds = [key + i for i in range(count)]
    args = [(geom.nx, s) for s in seeds]
    if workers <= 1 or count < 64:
        Z = np.stack([_texture(a).reshape(-1) for a in args])
    else:
        with mp.get_context("spawn").Pool(workers) as pool:
            Z = np.stack([z.reshape(-1) for z in pool.map(_texture, args, chunksize=max(1, count // (4 * workers)))])
    zs = torch.from_numpy(Z).to(dev)
    nus = synth.rng(key, synth.PURPOSE_BATCH).uniform(nu_lo, nu_hi, count)
    bd, _ = _noisy(ctx, geom, zs, seeds, nus)
    return bd, zs


def train(ctx, net, geom, bd, xd, epochs: int, batch: int, lr: float, seed: int = 0, log=None, objective: int = 0):
    """Adam over mini-batches; returns the mean loss of every epoch."""
    import torch

    import paper_2606_31153_amd as gk
    N = bd.shape[0]
    losses = []
    for ep in range(epochs):
        perm = np.random.default_rng(seed + ep).permutation(N)
        tot, cnt = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            idx = torch.from_numpy(perm[s:s + batch]).to(bd.device)
            tot += gk.gkb_net_train_step(ctx, net, geom, bd[idx].contiguous(), xd[idx].contiguous(), lr, objective)
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log("epoch %d: loss %.5f" % (ep, losses[-1]))
    return losses


def evaluate(ctx, net, geom, bd, xd, enorms, k_max: int = 150):
    """Plain and learned BA-GKB to the same residual level on every slice:
    the discrepancy level ||e|| (tau = 1) when plain BA-GKB reaches it within
    k_max iterations, otherwise the smallest residual plain BA-GKB reaches
    (with the unmatched pair BA-GKB minimises ||B (A x - b)||, and ||A x - b||
    can level off above ||e||)."""
    import torch

    import paper_2606_31153_amd as gk
    rows = []
    x = torch.zeros(geom.n, dtype=torch.float32, device=bd.device)
    for pc in (None, net):  # untimed: geometry tables, workspaces
        gk.gkb_ba_solve(ctx, geom, bd[0], x, k_max, use_dp=True, tau=1.0, noise_norm=float(enorms[0]), precond=pc)
    for i in range(bd.shape[0]):
        probe = gk.gkb_ba_solve(ctx, geom, bd[i], x, k_max, use_dp=True, tau=1.0, noise_norm=float(enorms[i]))
        target = float(enorms[i]) if probe.reason == gk.STOP_DP else float(np.min(probe.rho)) * (1.0 + 1e-6)
        res = {"target_over_e": target / float(enorms[i])}
        for name, pc in (("plain", None), ("learned", net)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = gk.gkb_ba_solve(ctx, geom, bd[i], x, k_max, use_dp=True, tau=1.0, noise_norm=target, precond=pc)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            xh, th = x.cpu().numpy().astype(np.float64), xd[i].cpu().numpy().astype(np.float64)
            rre = float(np.linalg.norm(xh - th) / np.linalg.norm(th))
            res[name] = {"k": r.k_stop, "reason": r.reason, "seconds": dt, "residual": r.residual, "rre": rre,
                         "res_over_e": r.residual / float(enorms[i])}
        # the learned recurrence without a stop: smallest residual and where
        free = gk.gkb_ba_solve(ctx, geom, bd[i], x, k_max, precond=net)
        res["learned_free"] = {"min_res_over_e": float(np.min(free.rho)) / float(enorms[i]),
                               "argmin_k": int(np.argmin(free.rho)) + 1,
                               "res_over_e_k": [float(v) / float(enorms[i]) for v in free.rho[:12]]}
        rows.append(res)
    out = {"target_over_e_mean": float(np.mean([r["target_over_e"] for r in rows]))}
    for name in ("plain", "learned"):
        ks = [r[name]["k"] for r in rows]
        out[name] = {"iterations_mean": float(np.mean(ks)), "s_per_slice": float(np.mean([r[name]["seconds"]
                                                                                           for r in rows])),
                     "rre_mean": float(np.mean([r[name]["rre"] for r in rows])),
                     "fallbacks": sum(1 for r in rows if r[name]["reason"] == gk.STOP_FALLBACK),
                     "dp_reached": sum(1 for r in rows if r[name]["reason"] in (gk.STOP_DP,))}
    out["speedup_s_per_slice"] = out["plain"]["s_per_slice"] / out["learned"]["s_per_slice"]
    out["slices"] = rows
    return out


def linear_pair_weights(f) -> np.ndarray:
    """Weights that make the network the linear filter f exactly, for any
    frozen masks: f and -f on channels 0 and 1, the middle layers pass the
    pair on, the last layer takes the difference; all other weights zero."""
    return init_weights(0, noise=0.0, first=f)
