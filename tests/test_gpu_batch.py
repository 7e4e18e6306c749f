"""Batched multi-slice solves (gkb_batch_solve, through the C ABI).

* Batched = single-slice, bit for bit: every slice of a batch runs the same
  kernel bodies on the same workgroup partition as gkb_ab_solve /
  gkb_ba_solve, so x, the stopping iteration and reason, and the residual
  and alpha/t histories must be identical (also with reorthogonalisation
  switched off for some slices).
* Batched = oracle: FP64 on geometries without rotation symmetry, x within
  1e-10 relative and identical stopping iterations.
* The 64-slice workload (parallel beam, n = 128..512, 180..720 views,
  0.5-5 % noise, discrepancy stop): every slice stops at the first
  iteration whose residual is at most tau*||e||, its reported residual is
  ||A x - b|| of the returned x (oracle's A, FP64), and sampled slices equal
  their single-slice solves bit for bit.
* Error paths: mixed geometry kinds, NaN in one slice, bad counts."""
import sys

import numpy as np
import pytest

import oracle
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


def problem(geom, seed, nu):
    op = oracle.Operator(geom)
    x_true = synth.rasterize_ellipses(synth.ellipse_params(seed), geom.nx, geom.ny)
    b_true = op.A(x_true).reshape(-1)
    b, en = synth.add_noise(b_true, synth.noise_direction(b_true.size, seed), nu)
    return b, en


def dev(a, dtype):
    return torch.tensor(np.asarray(a, dtype=np.float64), dtype=dtype, device=DEV)


SOLVE = {gk.GKB_METHOD_AB: ("gkb_ab_solve", oracle.MODE_AB), gk.GKB_METHOD_BA: ("gkb_ba_solve", oracle.MODE_BA)}

# ragged mix: square and non-square images, odd and even view counts, a
# non-unit detector pitch (more B^T candidates than the others)
MIX = [
    (synth.par2d(37, 23, 55, ny=29), dict(k_max=25, use_dp=True, tau=1.0), 0.02),
    (synth.par2d(48, 61), dict(k_max=30, use_dp=True, tau=1.02), 0.01),
    (synth.par2d(40, 31, 40, det_pitch=1.7), dict(k_max=12), 0.01),
    (synth.par2d(64, 89, 91), dict(k_max=40, use_dp=True, tau=1.0, lam=0.05), 0.01),
    (synth.par2d(24, 9, 35), dict(k_max=6), 0.05),
]
FAN_MIX = [
    (synth.fan2d(45, 33, 70), dict(k_max=20, use_dp=True, tau=1.0), 0.02),
    (synth.fan2d(32, 41, 50, src_dist=70.0), dict(k_max=15), 0.01),
    (synth.fan2d(57, 40, 81), dict(k_max=25, use_dp=True, tau=1.0), 0.01),
]


def build(mix, seed0):
    geoms, bs, opts = [], [], []
    for i, (g, o, nu) in enumerate(mix):
        b, en = problem(g, seed0 + i, nu)
        o = dict(o)
        if o.get("use_dp"):
            o["noise_norm"] = en
        geoms.append(g)
        bs.append(b)
        opts.append(o)
    return geoms, bs, opts


def run_batch(ctx, method, geoms, bs, opts, dtype):
    bd = [dev(b, dtype) for b in bs]
    xd = [torch.full((g.n,), float("nan"), dtype=dtype, device=DEV) for g in geoms]
    res = gk.gkb_batch_solve(ctx, method, geoms, bd, xd, opts)
    torch.cuda.synchronize()
    return res, [x.cpu().numpy() for x in xd]


def run_single(ctx, method, g, b, o, dtype):
    bd = dev(b, dtype)
    xd = torch.full((g.n,), float("nan"), dtype=dtype, device=DEV)
    r = getattr(gk, SOLVE[method][0])(ctx, g, bd, xd, **o)
    torch.cuda.synchronize()
    return r, xd.cpu().numpy()


def assert_same(rb, xb, rs, xs):
    assert rb.k_stop == rs.k_stop and rb.reason == rs.reason
    assert np.array_equal(xb, xs)
    assert rb.residual == rs.residual and rb.proj_residual == rs.proj_residual
    assert rb.t1 == rs.t1 and rb.alpha1 == rs.alpha1
    assert np.array_equal(rb.rho, rs.rho)
    assert np.array_equal(rb.alpha, rs.alpha) and np.array_equal(rb.t, rs.t)


@pytest.mark.parametrize("method", [gk.GKB_METHOD_BA, gk.GKB_METHOD_AB])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", ["par", "fan"])
def test_batch_equals_single_bitwise(ctx, method, dtype, kind):
    geoms, bs, opts = build(MIX if kind == "par" else FAN_MIX, 700)
    # a zero right-hand side: breakdown at start, x = 0
    geoms.append(geoms[0])
    bs.append(np.zeros(geoms[0].m))
    opts.append(dict(k_max=5))
    note("batch vs single %s %s %s" % (kind, method, dtype))
    rb, xb = run_batch(ctx, method, geoms, bs, opts, dtype)
    for s in range(len(geoms)):
        rs, xs = run_single(ctx, method, geoms[s], bs[s], opts[s], dtype)
        assert_same(rb[s], xb[s], rs, xs)
    assert rb[-1].reason == gk.STOP_BREAKDOWN and rb[-1].k_stop == 0 and not xb[-1].any()
    assert any(r.reason in (gk.STOP_DP, gk.STOP_DP_NOT_REACHED) for r in rb)
    assert any(r.reason == gk.STOP_KMAX for r in rb)


@pytest.mark.parametrize("method", [gk.GKB_METHOD_BA, gk.GKB_METHOD_AB])
@pytest.mark.parametrize("kind", ["par", "fan"])
def test_batch_graph_mode_equals_launch_mode(ctx, method, kind):
    # the hipGraph-captured iteration replays the same launches: every slice
    # bit for bit as in the launch-per-step mode, over a batch whose slices
    # stop at different iterations (the graph is captured again each time the
    # active set shrinks); the graph-mode batch is run twice, with eager work
    # and synchronisations in between, and both runs compared
    geoms, bs, opts = build(MIX if kind == "par" else FAN_MIX, 720)
    opts = [dict(o, k_max=max(o["k_max"], 36)) if not o.get("use_dp") else o for o in opts]
    note("batch graph vs launches %s %s" % (kind, method))
    ref, xref = run_batch(ctx, method, geoms, bs, opts, torch.float32)
    try:
        ctx.set_batch_mode(gk.GKB_BATCH_GRAPH)
        for rep in range(2):
            rb, xb = run_batch(ctx, method, geoms, bs, opts, torch.float32)
            for s in range(len(geoms)):
                assert_same(rb[s], xb[s], ref[s], xref[s])
            # eager work between the replays
            r1, x1 = run_single(ctx, method, geoms[0], bs[0], opts[0], torch.float32)
            assert_same(r1, x1, ref[0], xref[0])
    finally:
        ctx.set_batch_mode(gk.GKB_BATCH_LAUNCHES)
    ks = sorted({r.k_stop for r in ref})
    assert len(ks) >= 3 and ks[-1] > 33


def test_batch_without_reorthogonalisation(ctx):
    geoms, bs, opts = build(MIX[:3], 710)
    opts = [dict(o, reorth=(i != 1)) for i, o in enumerate(opts)]
    note("batch no-reorth slice")
    rb, xb = run_batch(ctx, gk.GKB_METHOD_BA, geoms, bs, opts, torch.float64)
    for s in range(3):
        rs, xs = run_single(ctx, gk.GKB_METHOD_BA, geoms[s], bs[s], opts[s], torch.float64)
        assert_same(rb[s], xb[s], rs, xs)


@pytest.mark.parametrize("method", [gk.GKB_METHOD_BA, gk.GKB_METHOD_AB])
def test_batch_with_stagnation_stops(ctx, method):
    # per-slice residual norm stagnation tolerances (eq. RNS), one slice
    # without, one with the discrepancy principle as well
    geoms, bs, opts = build(MIX[:4], 740)
    for o, eps in zip(opts, (0.05, 0.0, 0.01, 0.002)):
        o["rns_eps"] = eps
        o["k_max"] = 40
    note("batch rns %s" % method)
    rb, xb = run_batch(ctx, method, geoms, bs, opts, torch.float64)
    for s in range(4):
        rs, xs = run_single(ctx, method, geoms[s], bs[s], opts[s], torch.float64)
        assert_same(rb[s], xb[s], rs, xs)
    assert any(r.reason == gk.STOP_RNS for r in rb)


@pytest.mark.parametrize("method", [gk.GKB_METHOD_BA, gk.GKB_METHOD_AB])
def test_batch_mixes_k_max(ctx, method):
    # FP64 slices with k_max 113, 114 and 20 in one batch (Gram matrices and
    # inner-product partials of three sizes), each bit for bit as alone
    geoms, bs, opts = build(MIX[:3], 730)
    opts = [dict(o, k_max=k) for o, k in zip(opts, (113, 114, 20))]
    note("batch mixed k_max %s" % method)
    rb, xb = run_batch(ctx, method, geoms, bs, opts, torch.float64)
    for s in range(3):
        rs, xs = run_single(ctx, method, geoms[s], bs[s], opts[s], torch.float64)
        assert_same(rb[s], xb[s], rs, xs)
    assert rb[2].k_stop == 20


@pytest.mark.parametrize("method", [gk.GKB_METHOD_BA, gk.GKB_METHOD_AB])
def test_batch_matches_oracle_fp64(ctx, method):
    mix = [MIX[0], MIX[1], MIX[3]]
    geoms, bs, opts = build(mix, 720)
    note("batch vs oracle %s" % method)
    rb, xb = run_batch(ctx, method, geoms, bs, opts, torch.float64)
    for s, g in enumerate(geoms):
        o = opts[s]
        ref = oracle.gkb(oracle.Operator(g), SOLVE[method][1], bs[s], o["k_max"], lam=o.get("lam", 0.0),
                         use_dp=o.get("use_dp", False), tau=o.get("tau", 1.0), noise_norm=o.get("noise_norm", 0.0))
        assert rb[s].k_stop == ref.k_stop and rb[s].reason == ref.reason
        xr = ref.x.reshape(-1)
        assert np.linalg.norm(xb[s] - xr) <= 1e-10 * np.linalg.norm(xr)
        assert np.allclose(rb[s].rho, ref.rho, rtol=1e-10, atol=0)


def d3_problems(count=64):
    geoms, bs, opts, ens = [], [], [], []
    ctxp = gk.Context(0)
    for (n, v, nu, seed) in synth.batch_slices(3000, count):
        g = synth.par2d(n, v)
        x = torch.tensor(synth.ellipse_phantom(n, seed).reshape(-1), dtype=torch.float32, device=DEV)
        y = torch.empty(g.m, dtype=torch.float32, device=DEV)
        gk.gkb_forward(ctxp, g, x, y)
        torch.cuda.synchronize()
        b, en = synth.add_noise(y.double().cpu().numpy(), synth.noise_direction(g.m, seed), nu)
        geoms.append(g)
        bs.append(b)
        ens.append(en)
        opts.append(dict(k_max=150, use_dp=True, tau=1.0, noise_norm=en))
    ctxp.close()
    return geoms, bs, opts, ens


def test_batch_64_slice_workload(ctx):
    note("64-slice workload: building problems")
    geoms, bs, opts, ens = d3_problems()
    note("64-slice workload: batched BA-GKB")
    rb, xb = run_batch(ctx, gk.GKB_METHOD_BA, geoms, bs, opts, torch.float32)
    for s, r in enumerate(rb):
        assert r.reason in (gk.STOP_DP, gk.STOP_DP_NOT_REACHED, gk.STOP_BREAKDOWN), (s, r.reason)
        if r.reason == gk.STOP_DP:
            assert r.residual <= ens[s] and r.rho[-1] == r.residual
            assert np.all(r.rho[:-1] > ens[s])  # first crossing
    # the reported residual is ||A x - b|| of the returned x (FP32 x, FP64 oracle A)
    for s in (0, 17, 40):
        ax = oracle.Operator(geoms[s]).A(xb[s].astype(np.float64)).reshape(-1)
        lit = np.linalg.norm(ax - np.asarray(bs[s], dtype=np.float32).astype(np.float64))
        assert abs(lit - rb[s].residual) <= 1e-4 * lit
    # sampled slices equal their single-slice solves bit for bit
    for s in (3, 29, 63):
        note("64-slice workload: single-slice check %d" % s)
        rs, xs = run_single(ctx, gk.GKB_METHOD_BA, geoms[s], bs[s], opts[s], torch.float32)
        assert_same(rb[s], xb[s], rs, xs)


def test_batch_errors(ctx):
    g1, g2 = synth.par2d(16, 10), synth.fan2d(16, 10, 30)
    b1 = torch.ones(g1.m, dtype=torch.float32, device=DEV)
    b2 = torch.ones(g2.m, dtype=torch.float32, device=DEV)
    x1 = torch.zeros(g1.n, dtype=torch.float32, device=DEV)
    x2 = torch.zeros(g2.n, dtype=torch.float32, device=DEV)
    o = dict(k_max=3)
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_batch_solve(ctx, gk.GKB_METHOD_BA, [g1, g2], [b1, b2], [x1, x2], [o, o])
    assert e.value.status == gk.GKB_EINVAL
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_batch_solve(ctx, gk.GKB_METHOD_BA, [], [], [], [])
    assert e.value.status == gk.GKB_EINVAL
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_batch_solve(ctx, 7, [g1], [b1], [x1], [o])
    assert e.value.status == gk.GKB_EINVAL
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_batch_solve(ctx, gk.GKB_METHOD_BA, [g1], [b1], [x1], [dict(k_max=0)])
    assert e.value.status == gk.GKB_EINVAL and "slice 0" in str(e.value)
    # NaN in one slice: nothing written to any x
    bn = b1.clone()
    bn[5] = float("nan")
    xa = torch.full((g1.n,), 7.0, dtype=torch.float32, device=DEV)
    xb = torch.full((g1.n,), 7.0, dtype=torch.float32, device=DEV)
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_batch_solve(ctx, gk.GKB_METHOD_BA, [g1, g1], [b1, bn], [xa, xb], [o, o])
    assert e.value.status == gk.GKB_ENONFINITE
    torch.cuda.synchronize()
    assert bool((xa == 7.0).all()) and bool((xb == 7.0).all())
