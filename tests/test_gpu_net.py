"""The learned sinogram filter on the GPU (through the C ABI) against the
FP64 oracle of oracle/net.py.

* N(y), F y and F^T z: relative L2 error <= 1e-5 (FP32 accumulation; the
  matrix-core layers take each activation as three bfloat16 terms).
* <F y, z> = <y, F^T z> to 1e-5 and F b = N(b) bit for bit on the GPU.
* Identity network: N(y) = y exactly, and BA-GKB with it equals plain
  BA-GKB bit for bit.
* Training gradient (bfloat16 operands in the matrix-core layers) against
  the oracle's gradient with the same rounding points: relative L2 <= 1e-4
  per layer; one Adam step against the oracle's update; the loss decreases
  over a few steps.
* A network whose filter is zero makes the learned solve fall back to plain
  BA-GKB (reason FALLBACK, the plain result bit for bit).
* Weights: save/load round trip; invalid arguments."""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import dense
from oracle import net as onet
from paper_2606_31153_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2606_31153_amd as gk  # noqa: E402

DEV = torch.device("cuda:0")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gk.Context(0)
    yield c
    c.close()


def dev32(a):
    return torch.tensor(np.asarray(a, dtype=np.float32).reshape(-1), device=DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


GEOMS = {"par": synth.par2d(40, 30, 57), "fan": synth.fan2d(48, 40, 300)}


def sino(geom, seed):
    x = synth.rasterize_ellipses(synth.ellipse_params(seed), geom.nx, geom.ny)
    b = oracle.Operator(geom).A(x).reshape(geom.n_views, geom.n_det_u)
    r = np.random.default_rng(seed)
    return b + 0.01 * np.abs(b).max() * r.standard_normal(b.shape)


def rows(a, geom):
    return np.asarray(a, dtype=np.float64).reshape(geom.n_views, geom.n_det_u)


@pytest.mark.parametrize("gname", list(GEOMS))
def test_filter_matches_oracle(ctx, gname):
    geom = GEOMS[gname]
    net = gk.Net(ctx, seed=11)
    Ws = onet.split_weights(net.get_weights().astype(np.float64))
    b = sino(geom, 900).astype(np.float32).astype(np.float64)
    r = np.random.default_rng(901)
    y = r.standard_normal(b.shape).astype(np.float32).astype(np.float64)
    z = r.standard_normal(b.shape).astype(np.float32).astype(np.float64)
    note("filter %s: N(b)" % gname)
    out = torch.empty(geom.m, dtype=torch.float32, device=DEV)
    gk.gkb_net_apply(ctx, net, geom, dev32(b), out)
    torch.cuda.synchronize()
    Nb_ref, _, _ = onet.forward(Ws, b)
    Nb = out.cpu().numpy().astype(np.float64)
    assert rel(Nb, Nb_ref.reshape(-1)) <= 1e-5
    masks = onet.masks_of(Ws, b)
    note("filter %s: F y, F^T z" % gname)
    Fy = torch.empty(geom.m, dtype=torch.float32, device=DEV)
    Ftz = torch.empty(geom.m, dtype=torch.float32, device=DEV)
    gk.gkb_net_frozen_apply(ctx, net, geom, dev32(b), dev32(y), Fy)
    gk.gkb_net_frozen_apply(ctx, net, geom, dev32(b), dev32(z), Ftz, transpose=True)
    Fb = torch.empty(geom.m, dtype=torch.float32, device=DEV)
    gk.gkb_net_frozen_apply(ctx, net, geom, dev32(b), dev32(b), Fb)
    torch.cuda.synchronize()
    Fy, Ftz = Fy.cpu().numpy().astype(np.float64), Ftz.cpu().numpy().astype(np.float64)
    assert rel(Fy, onet.apply_F(Ws, masks, y).reshape(-1)) <= 1e-5
    assert rel(Ftz, onet.apply_Ft(Ws, masks, z).reshape(-1)) <= 1e-5
    # L1: adjointness on the GPU and F b = N(b)
    lhs, rhs = float(Fy @ z.reshape(-1)), float(y.reshape(-1) @ Ftz)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Fy) * np.linalg.norm(z)
    assert np.array_equal(Fb.cpu().numpy().astype(np.float64), Nb)
    net.close()


def test_identity_network_gives_plain_ba_gkb(ctx):
    geom = synth.par2d(48, 61)
    net = gk.Net(ctx, seed=0)
    net.set_weights(onet.flatten(onet.identity_weights()).astype(np.float32))
    op = oracle.Operator(geom)
    x = synth.rasterize_ellipses(synth.ellipse_params(930), geom.nx, geom.ny)
    b, en = synth.add_noise(op.A(x).reshape(-1), synth.noise_direction(geom.m, 930), 0.02)
    assert np.all(b != 0)
    note("identity network: N(y) = y")
    y = torch.tensor(np.random.default_rng(1).standard_normal(geom.m), dtype=torch.float32, device=DEV)
    out = torch.empty_like(y)
    gk.gkb_net_apply(ctx, net, geom, y, out)
    torch.cuda.synchronize()
    assert torch.equal(out, y)
    note("identity network: learned vs plain BA-GKB")
    bd = dev32(b)
    x1 = torch.full((geom.n,), float("nan"), dtype=torch.float32, device=DEV)
    x2 = torch.full((geom.n,), float("nan"), dtype=torch.float32, device=DEV)
    kw = dict(use_dp=True, tau=1.0, noise_norm=en)
    r1 = gk.gkb_ba_solve(ctx, geom, bd, x1, 40, **kw)
    r2 = gk.gkb_ba_solve(ctx, geom, bd, x2, 40, precond=net, **kw)
    torch.cuda.synchronize()
    assert r1.k_stop == r2.k_stop and r1.reason == r2.reason == gk.STOP_DP
    assert torch.equal(x1, x2)
    assert np.array_equal(r1.rho, r2.rho)
    net.close()


def test_training_gradient_matches_oracle(ctx):
    geom = synth.par2d(24, 15, 35)
    net = gk.Net(ctx, seed=5)
    Ws = onet.split_weights(net.get_weights().astype(np.float64))
    op = oracle.Operator(geom)
    S = 2
    xs, bs = [], []
    for i in range(S):
        x = synth.rasterize_ellipses(synth.ellipse_params(940 + i), geom.nx, geom.ny).reshape(-1)
        b, _ = synth.add_noise(op.A(x).reshape(-1), synth.noise_direction(geom.m, 940 + i), 0.02)
        xs.append(x.astype(np.float32).astype(np.float64))
        bs.append(b.astype(np.float32).astype(np.float64))
    note("training gradient")
    loss, grad = gk.gkb_net_grad(ctx, net, geom, dev32(np.stack(bs)).reshape(S, -1), dev32(np.stack(xs)).reshape(S, -1))
    ref_loss, ref_grads = onet.loss_and_grad(
        Ws, lambda v: op.B(v).reshape(-1), lambda v: op.Bt(v).reshape(-1),
        [b.reshape(geom.n_views, geom.n_det_u) for b in bs], xs, train=True)
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    g = onet.split_weights(grad.astype(np.float64))
    note("training gradient rel per layer: " + " ".join("%.2e" % rel(g[l], ref_grads[l]) for l in range(4)))
    for l in range(4):
        assert rel(g[l], ref_grads[l]) <= 1e-4, l
    # the operator objective: the filter frozen at b applied to A x
    note("training gradient, frozen objective")
    loss_f, grad_f = gk.gkb_net_grad(ctx, net, geom, dev32(np.stack(bs)).reshape(S, -1),
                                     dev32(np.stack(xs)).reshape(S, -1), objective=gk.GKB_NET_FROZEN)
    ref_lf, ref_gf = onet.frozen_loss_and_grad(
        Ws, lambda v: op.A(v.astype(np.float32).astype(np.float64)).reshape(-1),
        lambda v: op.B(v).reshape(-1), lambda v: op.Bt(v).reshape(-1),
        [b.reshape(geom.n_views, geom.n_det_u) for b in bs], xs, train=True)
    assert loss_f == pytest.approx(ref_lf, rel=1e-4)
    gf = onet.split_weights(grad_f.astype(np.float64))
    note("frozen-objective gradient rel per layer: " + " ".join("%.2e" % rel(gf[l], ref_gf[l]) for l in range(4)))
    for l in range(4):
        assert rel(gf[l], ref_gf[l]) <= 1e-4, l
    # one Adam step from the GPU's own gradient
    w0 = net.get_weights().astype(np.float64)
    gk.gkb_net_train_step(ctx, net, geom, dev32(np.stack(bs)).reshape(S, -1), dev32(np.stack(xs)).reshape(S, -1),
                          1e-3)
    w1_ref, _, _ = onet.adam(w0, grad.astype(np.float64), np.zeros_like(w0), np.zeros_like(w0), 1, 1e-3)
    assert np.max(np.abs(net.get_weights() - w1_ref)) <= 1e-6
    net.close()


def test_training_reduces_the_loss(ctx):
    geom = synth.par2d(32, 24, 47)
    net = gk.Net(ctx, seed=9)
    op = oracle.Operator(geom)
    S = 4
    xs, bs = [], []
    for i in range(S):
        x = synth.rasterize_ellipses(synth.ellipse_params(950 + i), geom.nx, geom.ny).reshape(-1)
        b, _ = synth.add_noise(op.A(x).reshape(-1), synth.noise_direction(geom.m, 950 + i), 0.02)
        xs.append(x)
        bs.append(b)
    bd, xd = dev32(np.stack(bs)).reshape(S, -1), dev32(np.stack(xs)).reshape(S, -1)
    note("training steps")
    losses = [gk.gkb_net_train_step(ctx, net, geom, bd, xd, 3e-3) for _ in range(40)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
    net.close()


def test_zero_filter_falls_back_to_plain(ctx):
    geom = synth.par2d(32, 40)
    net = gk.Net(ctx, seed=1)
    net.set_weights(np.zeros(gk.NET_PARAMS, dtype=np.float32))
    op = oracle.Operator(geom)
    x = synth.rasterize_ellipses(synth.ellipse_params(960), geom.nx, geom.ny)
    b, en = synth.add_noise(op.A(x).reshape(-1), synth.noise_direction(geom.m, 960), 0.02)
    bd = dev32(b)
    x1 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    x2 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    note("fallback")
    r1 = gk.gkb_ba_solve(ctx, geom, bd, x1, 30, use_dp=True, noise_norm=en)
    r2 = gk.gkb_ba_solve(ctx, geom, bd, x2, 30, use_dp=True, noise_norm=en, precond=net)
    torch.cuda.synchronize()
    assert r2.reason == gk.STOP_FALLBACK and r2.k_stop == r1.k_stop
    assert torch.equal(x1, x2)
    net.close()


def test_learned_stop_above_the_discrepancy_level_falls_back(ctx):
    # With the discrepancy principle on, a learned attempt that the residual
    # stagnation rule ends above tau ||e|| must not be returned: the plain
    # BA-GKB result comes back with reason FALLBACK.  tau = 0.5 lies below the
    # smallest residual this overdetermined problem can reach (about
    # sqrt((m - n) / m) ||e||), and rns_eps = 0.9 ends the attempt at k = 2.
    geom = synth.par2d(32, 40)
    net = gk.Net(ctx, seed=5)  # He-initialised random network
    op = oracle.Operator(geom)
    x = synth.rasterize_ellipses(synth.ellipse_params(961), geom.nx, geom.ny)
    b, en = synth.add_noise(op.A(x).reshape(-1), synth.noise_direction(geom.m, 961), 0.02)
    bd = dev32(b)
    x1 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    x2 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    note("learned RNS stop above the DP level")
    kw = dict(use_dp=True, tau=0.5, noise_norm=en, rns_eps=0.9)
    r1 = gk.gkb_ba_solve(ctx, geom, bd, x1, 30, **kw)
    r2 = gk.gkb_ba_solve(ctx, geom, bd, x2, 30, precond=net, **kw)
    torch.cuda.synchronize()
    assert r1.residual > 0.5 * en
    assert r2.reason == gk.STOP_FALLBACK and r2.k_stop == r1.k_stop
    assert torch.equal(x1, x2)
    net.close()


def test_failing_learned_attempt_ends_at_stagnation(ctx):
    # With the discrepancy principle on, a learned attempt whose residual
    # levels off above the level ends at the first k > 5 at which the mean
    # decrease of the last five iterations, continued to k_max, would leave
    # it above tau ||e||, instead of running to k_max; the plain result is
    # returned (reason FALLBACK).  tau = 0.5 is out of reach (the residual of
    # this overdetermined problem stays above about sqrt((m - n) / m) ||e||).
    geom = synth.par2d(48, 60)
    net = gk.Net(ctx, seed=7)  # He-initialised random network
    op = oracle.Operator(geom)
    x = synth.rasterize_ellipses(synth.ellipse_params(962), geom.nx, geom.ny)
    b, en = synth.add_noise(op.A(x).reshape(-1), synth.noise_direction(geom.m, 962), 0.02)
    bd = dev32(b)
    K = 150
    x1 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    x2 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    free = gk.gkb_ba_solve(ctx, geom, bd, x2, K, precond=net)
    rho, level, W = free.rho, 0.5 * en, 5
    k_stall = next(k for k in range(W + 1, K + 1)
                   if not (rho[k - 1 - W] - rho[k - 1]) / W * (K - k) + level >= rho[k - 1])
    kw = dict(use_dp=True, tau=0.5, noise_norm=en)
    r1 = gk.gkb_ba_solve(ctx, geom, bd, x1, K, **kw)
    ctx.trace_reset()
    ctx.trace_enable(True)
    r2 = gk.gkb_ba_solve(ctx, geom, bd, x2, K, precond=net, **kw)
    torch.cuda.synchronize()
    ctx.trace_enable(False)
    n_ft, _ = ctx.trace_get("filter_t")
    note("learned stall: k_stall %d of %d, F^T launches %d" % (k_stall, K, n_ft))
    assert k_stall < K // 2
    # one F^T per iteration and one at start-up; up to four iterations are
    # queued before the host sees the stop
    assert k_stall + 1 <= n_ft <= k_stall + 5
    assert r2.reason == gk.STOP_FALLBACK and r2.k_stop == r1.k_stop
    assert torch.equal(x1, x2)
    net.close()


LEARNED_GEOMS = {
    "par": synth.par2d(20, 16, 29),
    "fan": synth.fan2d(20, 18, 40),
    # cone beam: the filter runs along every detector row of every view
    "cone": synth.cone3d(6, 5, 13, 7),
}


def dense_filter(Ws, masks, rows, L):
    """F_b as a dense m x m matrix from the oracle's frozen-mask filter
    applied to unit vectors (one position of every row at a time: the rows
    are independent)."""
    m = rows * L
    F = np.zeros((m, m))
    for l in range(L):
        E = np.zeros((rows, L))
        E[:, l] = 1.0
        out = onet.apply_F(Ws, masks, E)
        for r in range(rows):
            F[r * L:(r + 1) * L, r * L + l] = out[r]
    return F


def dp_tau_with_margin(rho, en, k_min=4):
    """tau whose first discrepancy crossing (eq. DP) falls at an iteration
    whose residual lies at least 2 % below every earlier one, halfway
    between them; None if there is none."""
    for k in range(k_min, len(rho)):
        prev = np.min(rho[:k])
        if rho[k] < 0.98 * prev:
            return 0.5 * (rho[k] + prev) / en, k + 1
    return None, None


@pytest.mark.parametrize("gname", list(LEARNED_GEOMS))
def test_learned_ba_gkb_matches_oracle(ctx, gname):
    # BA-GKB with M = B F_b A (Alg. "BA-GKB" with the learned filter inside B)
    # against the oracle's BA-GKB on the dense pair (A, B F_b), F_b built from
    # the oracle's network with the masks of b frozen, for a random
    # He-initialised network: the fixed-iteration run and a discrepancy-
    # principle run, FP32 GPU against FP64 oracle
    geom = LEARNED_GEOMS[gname]
    cone = geom.kind == synth.KIND_CONE3D
    net = gk.Net(ctx, seed=21)
    Ws = onet.split_weights(net.get_weights().astype(np.float64))
    op = oracle.Operator(geom)
    if cone:
        x_true = synth.rasterize_ellipsoids(synth.ellipsoid_params(990), geom.nx)
    else:
        x_true = synth.rasterize_ellipses(synth.ellipse_params(990), geom.nx, geom.ny)
    b, en = synth.add_noise(op.A(x_true).reshape(-1), synth.noise_direction(geom.m, 990), 0.02)
    b32 = b.astype(np.float32).astype(np.float64)
    L = geom.n_det_u
    rows = geom.m // L
    masks = onet.masks_of(Ws, b32.reshape(rows, L))
    F = dense_filter(Ws, masks, rows, L)
    # the GPU's frozen filter, column block by column block (its masks come
    # from its own FP32 evaluation of N at b)
    note("learned %s: F columns" % gname)
    for l in range(0, L, max(1, L // 5)):
        E = np.zeros((rows, L))
        E[:, l] = 1.0
        out = torch.empty(geom.m, dtype=torch.float32, device=DEV)
        gk.gkb_net_frozen_apply(ctx, net, geom, dev32(b32), dev32(E), out)
        torch.cuda.synchronize()
        ref = np.stack([F[r * L:(r + 1) * L, r * L + l] for r in range(rows)]).reshape(-1)
        assert rel(out.cpu().numpy().astype(np.float64), ref) <= 1e-5, l
    if cone:
        Ad, Bd = dense.dense_A_cone(geom), dense.dense_B_cone(geom)
    else:
        Ad, Bd = dense.dense_A(geom), dense.dense_B(geom)
    opF = oracle.Operator(A=Ad, B=Bd @ F)
    K = 12
    ref = oracle.gkb(opF, oracle.MODE_BA, b32, K)
    note("learned %s: %d iterations" % (gname, K))
    bd = dev32(b32)
    xd = torch.full((geom.n,), float("nan"), dtype=torch.float32, device=DEV)
    res = gk.gkb_ba_solve(ctx, geom, bd, xd, K, precond=net)
    torch.cuda.synchronize()
    x = xd.cpu().numpy().astype(np.float64)
    note("learned %s: x rel %.2e" % (gname, rel(x, ref.x.reshape(-1))))
    assert (res.k_stop, res.reason) == (ref.k_stop, ref.reason) == (K, gk.STOP_KMAX)
    assert rel(x, ref.x.reshape(-1)) <= 1e-4
    assert np.allclose(res.alpha[:K], ref.alpha[:K], rtol=1e-4)
    assert np.allclose(res.t, ref.t[:K + 1], rtol=1e-4)
    assert np.allclose(res.rho, ref.rho, rtol=1e-4)
    tau, k_dp = dp_tau_with_margin(ref.rho, en)
    if tau is not None:
        refd = oracle.gkb(opF, oracle.MODE_BA, b32, K, use_dp=True, tau=tau, noise_norm=en)
        assert (refd.k_stop, refd.reason) == (k_dp, oracle.STOP_DP)
        note("learned %s: DP at k=%d (tau %.4f)" % (gname, k_dp, tau))
        res = gk.gkb_ba_solve(ctx, geom, bd, xd, K, use_dp=True, tau=tau, noise_norm=en, precond=net)
        torch.cuda.synchronize()
        assert (res.k_stop, res.reason) == (refd.k_stop, gk.STOP_DP)
        assert rel(xd.cpu().numpy().astype(np.float64), refd.x.reshape(-1)) <= 1e-4
    net.close()


def test_weights_roundtrip_and_errors(ctx, tmp_path):
    net = gk.Net(ctx, seed=3)
    w = net.get_weights()
    # He initialisation: std sqrt(2 / fan_in) per layer
    Ws = onet.split_weights(w.astype(np.float64))
    assert abs(Ws[1].std() / np.sqrt(2.0 / (32 * 9)) - 1.0) < 0.05
    path = str(tmp_path / "net.bin")
    net.save(path)
    net2 = gk.Net(ctx, seed=4)
    assert not np.array_equal(net2.get_weights(), w)
    net2.load(path)
    assert np.array_equal(net2.get_weights(), w)
    with open(path, "r+b") as f:
        f.write(b"XXXX")
    with pytest.raises(gk.GkbError):
        net2.load(path)
    with pytest.raises(gk.GkbError) as e:
        gk.Net(ctx, channels=16)
    assert e.value.status == gk.GKB_EUNSUPPORTED
    geom = synth.par2d(16, 10)
    bd = torch.ones(geom.m, dtype=torch.float32, device=DEV)
    xd = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_ab_solve(ctx, geom, bd, xd, 5, precond=net)
    assert e.value.status == gk.GKB_EUNSUPPORTED
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_ba_solve(ctx, geom, bd.double(), xd.double(), 5, precond=net)
    assert e.value.status == gk.GKB_EUNSUPPORTED
    net.close()
    net2.close()


def test_linear_filter_through_the_network_path_preconditions_ba_gkb(ctx):
    # the filter path with the network set to the Ram-Lak filter (an exactly
    # linear F for any masks) reaches the discrepancy level in fewer
    # iterations than plain BA-GKB, with the residual at the same level
    from paper_2606_31153_amd import learned
    geom = synth.par2d(96, 120)
    net = gk.Net(ctx, seed=0)
    net.set_weights(learned.linear_pair_weights(learned.ramlak()))
    op = oracle.Operator(geom)
    x_true = synth.rasterize_ellipses(synth.ellipse_params(970), geom.nx, geom.ny)
    b, en = synth.add_noise(op.A(x_true).reshape(-1), synth.noise_direction(geom.m, 970), 0.03)
    bd = dev32(b)
    x1 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    x2 = torch.zeros(geom.n, dtype=torch.float32, device=DEV)
    note("Ram-Lak filter vs plain")
    r1 = gk.gkb_ba_solve(ctx, geom, bd, x1, 100, use_dp=True, noise_norm=en)
    r2 = gk.gkb_ba_solve(ctx, geom, bd, x2, 100, use_dp=True, noise_norm=en, precond=net)
    torch.cuda.synchronize()
    note("plain k %d, filtered k %d" % (r1.k_stop, r2.k_stop))
    assert r1.reason == gk.STOP_DP and r2.reason == gk.STOP_DP
    assert r2.residual <= en and r1.residual <= en
    assert r2.k_stop < r1.k_stop
    net.close()
