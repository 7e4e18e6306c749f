"""GPU parity of AB-/BA-/matched GKB (through the C ABI) against the FP64 CPU
oracle on the same seeded inputs.

FP64 path: identical stopping iteration and reason; on geometries without
rotation symmetry, reconstructions within 1e-10 relative and alpha/t
histories within 1e-11 (the 64x64 / 90-view workload itself is checked to
the limit its repeated singular values allow, see below).  FP32/FP64 split:
identical discrepancy-principle iteration and reconstructions within 1e-4
relative."""
import sys

import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2606_31153_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2606_31153_amd as gk  # noqa: E402

MODES = {"ab": (oracle.MODE_AB, "gkb_ab_solve"), "ba": (oracle.MODE_BA, "gkb_ba_solve"),
         "gkb": (oracle.MODE_GKB, "gkb_gkb_solve")}


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
    return op, x_true, b, en


def gpu_solve(ctx, geom, mode, b, dtype, k_max, **kw):
    dev = torch.device("cuda:0")
    bd = torch.tensor(np.asarray(b, dtype=np.float64), dtype=dtype, device=dev)
    xd = torch.full((geom.n,), float("nan"), dtype=dtype, device=dev)
    res = getattr(gk, MODES[mode][1])(ctx, geom, bd, xd, k_max, **kw)
    torch.cuda.synchronize()
    return res, xd.cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def stable_prefix(op, mode, b, k_max, **kw):
    """Number of leading iterations whose alpha_i and t_i the oracle itself
    reproduces to 1e-12 under a 1e-15 relative perturbation of b, and the
    resulting spread of x."""
    r1 = oracle.gkb(op, MODES[mode][0], b, k_max, **kw)
    bp = b * (1.0 + 1e-15 * np.random.default_rng(0).standard_normal(b.size))
    r2 = oracle.gkb(op, MODES[mode][0], bp, k_max, **kw)
    k = min(r1.k_stop, r2.k_stop)
    d = np.maximum(np.abs(r1.alpha[:k] / r2.alpha[:k] - 1.0), np.abs(r1.t[:k] / r2.t[:k] - 1.0))
    kp = int(np.argmax(d > 1e-12)) if (d > 1e-12).any() else k
    return kp, rel(r2.x.reshape(-1), r1.x.reshape(-1))


# Config 1 exactly as specified: 64x64 image, 90 views over [0, pi), 91 bins.
# The geometry maps onto itself under 90-degree rotations, so M has exactly
# repeated singular values and the Krylov recurrence becomes ill-determined
# once the leading copy of such a pair has converged: two FP64
# implementations (or one with b perturbed by 1e-15) then differ far above
# rounding level.  Iteration counts must still agree; alpha/t are compared
# over the prefix the oracle itself reproduces, x to the 1e-4 reconstruction
# bar (or rounding level when the stop comes inside the stable prefix).
@pytest.mark.parametrize("mode", ["ab", "ba", "gkb"])
@pytest.mark.parametrize("seed", [1000, 1003, 1007])
@pytest.mark.parametrize("lam_rel", [0.0, 1e-3, 1e-1])
def test_fp64_config1_matches_oracle(ctx, mode, seed, lam_rel):
    geom = synth.workload_par64()
    op, xt, b, en = problem(geom, seed, 0.01)
    a1 = oracle.gkb(op, MODES[mode][0], b, 1).alpha1
    lam = lam_rel * a1
    kw = dict(lam=lam, use_dp=True, tau=1.0, noise_norm=en)
    ref = oracle.gkb(op, MODES[mode][0], b, 30, **kw)
    kp, spread = stable_prefix(op, mode, b, 30, **kw)
    note("fp64 config1 %s seed=%d lam=%g (stable prefix %d, spread %.1e)" % (mode, seed, lam_rel, kp, spread))
    res, x = gpu_solve(ctx, geom, mode, b, torch.float64, 30, **kw)
    assert (res.k_stop, res.reason) == (ref.k_stop, ref.reason)
    k = ref.k_stop
    tol = 1e-10 if k <= kp else 1e-4
    assert rel(x, ref.x.reshape(-1)) <= tol
    assert np.allclose(res.alpha[:kp], ref.alpha[:kp], rtol=1e-9)
    assert np.allclose(res.t[:kp], ref.t[:kp], rtol=1e-9)
    assert np.allclose(res.rho[:kp], ref.rho[:kp], rtol=1e-9)


# The same workload with the rotation symmetry broken (89 views, or a 64x57
# image): the oracle is reproducible to rounding level over all iterations,
# and so must the GPU FP64 path be.
@pytest.mark.parametrize("mode", ["ab", "ba", "gkb"])
@pytest.mark.parametrize("gname", ["par64_v89", "par64x57"])
@pytest.mark.parametrize("lam_rel", [0.0, 1e-1])
def test_fp64_strict_parity(ctx, mode, gname, lam_rel):
    geom = synth.par2d(64, 89, 91) if gname == "par64_v89" else synth.par2d(64, 90, 91, ny=57)
    op, xt, b, en = problem(geom, 1000, 0.01)
    a1 = oracle.gkb(op, MODES[mode][0], b, 1).alpha1
    kw = dict(lam=lam_rel * a1, use_dp=True, tau=1.0, noise_norm=en)
    ref = oracle.gkb(op, MODES[mode][0], b, 30, **kw)
    note("fp64 strict %s %s lam=%g" % (gname, mode, lam_rel))
    res, x = gpu_solve(ctx, geom, mode, b, torch.float64, 30, **kw)
    assert (res.k_stop, res.reason) == (ref.k_stop, ref.reason)
    k = ref.k_stop
    assert rel(x, ref.x.reshape(-1)) <= 1e-10
    assert np.allclose(res.alpha[:k], ref.alpha[:k], rtol=1e-11)
    assert np.allclose(res.t[:k + 1], ref.t[:k + 1], rtol=1e-11)
    assert np.allclose(res.rho, ref.rho, rtol=1e-9)
    assert res.residual == pytest.approx(ref.residual, rel=1e-9)
    assert res.proj_residual == pytest.approx(oracle.proj_solve(ref.alpha, ref.t, k, kw["lam"])[1], rel=1e-8)


@pytest.mark.parametrize("mode", ["ab", "ba"])
def test_fp64_fixed_30_iterations(ctx, mode):
    geom = synth.par2d(64, 89, 91)
    op, xt, b, en = problem(geom, 1001, 0.01)
    ref = oracle.gkb(op, MODES[mode][0], b, 30)
    note("fp64 30 its %s" % mode)
    res, x = gpu_solve(ctx, geom, mode, b, torch.float64, 30)
    assert (res.k_stop, res.reason) == (30, gk.STOP_KMAX) == (ref.k_stop, ref.reason)
    assert rel(x, ref.x.reshape(-1)) <= 1e-9
    assert np.allclose(res.rho, ref.rho, rtol=1e-8)


def rns_eps_with_margin(rho, k_min=4):
    """A stagnation tolerance whose first crossing (eq. RNS) falls at some k
    >= k_min with a factor of at least 1.1 to spare on both sides (FP32
    rounding moves these ratios by about 1e-4 relative), so that rounding
    cannot move the stop; returns (eps, k)."""
    ratio = np.abs(np.diff(rho)) / rho[:-1]  # ratio[j] belongs to k = j + 2
    for j in range(k_min - 2, ratio.size):
        lo = ratio[j]
        hi = ratio[:j].min() if j > 0 else np.inf
        if hi > 1.21 * lo:
            return float(np.sqrt(lo * min(hi, 4 * lo))), j + 2
    raise AssertionError("no well-separated stagnation point")


# Residual norm stagnation (eq. RNS) against the oracle: same stopping
# iteration and reason, x to the FP64 / FP32 bars.
@pytest.mark.parametrize("mode", ["ab", "ba"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rns_stop_matches_oracle(ctx, mode, dtype):
    geom = synth.par2d(64, 89, 91)
    op, xt, b, en = problem(geom, 1004, 0.01)
    if dtype == torch.float32:
        b = np.float32(b).astype(np.float64)
    plain = oracle.gkb(op, MODES[mode][0], b, 40)
    eps, k_exp = rns_eps_with_margin(plain.rho, k_min=12)
    ref = oracle.gkb(op, MODES[mode][0], b, 40, rns_eps=eps)
    assert (ref.k_stop, ref.reason) == (k_exp, oracle.STOP_RNS)
    note("rns %s %s eps=%.3g k=%d" % (mode, dtype, eps, k_exp))
    res, x = gpu_solve(ctx, geom, mode, b, dtype, 40, rns_eps=eps)
    assert (res.k_stop, res.reason) == (k_exp, gk.STOP_RNS)
    assert rel(x, ref.x.reshape(-1)) <= (1e-10 if dtype == torch.float64 else 1e-4)
    assert np.allclose(res.rho, ref.rho, rtol=1e-9 if dtype == torch.float64 else 1e-3)


# RRE(x_k) per iteration (eq. RE) against the oracle's history; recording it
# leaves the solve itself bit for bit unchanged.
@pytest.mark.parametrize("mode", ["ab", "ba", "gkb"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rre_history_matches_oracle(ctx, mode, dtype):
    geom = synth.par2d(64, 89, 91)
    op, xt, b, en = problem(geom, 1005, 0.01)
    xt = xt.reshape(-1)
    if dtype == torch.float32:
        b = np.float32(b).astype(np.float64)
        xt = np.float32(xt).astype(np.float64)
    ref = oracle.gkb(op, MODES[mode][0], b, 25, x_true=xt)
    note("rre %s %s" % (mode, dtype))
    xtd = torch.tensor(xt, dtype=dtype, device=torch.device("cuda:0"))
    res, x = gpu_solve(ctx, geom, mode, b, dtype, 25, x_true=xtd)
    plain, x0 = gpu_solve(ctx, geom, mode, b, dtype, 25)
    assert res.k_stop == ref.k_stop == 25
    assert np.allclose(res.rre, ref.rre, rtol=1e-9 if dtype == torch.float64 else 1e-4, atol=0)
    assert np.array_equal(x, x0) and np.array_equal(res.rho, plain.rho)


def test_rns_invalid_tolerance_rejected(ctx):
    geom = synth.par2d(16, 10)
    b = np.ones(geom.m)
    for bad in (-1e-3, float("nan"), float("inf")):
        with pytest.raises(RuntimeError):
            gpu_solve(ctx, geom, "ba", b, torch.float32, 5, rns_eps=bad)


# The second reorthogonalisation round takes its coefficients from the Gram
# matrix of the stored basis (c1 - G c1, no second read of Q; the oracle
# takes two classical rounds).  Long discrepancy-stopped solves against the
# oracle, with the Gram matrix and the inner-product partials sized by k_max.
@pytest.mark.parametrize("mode", ["ab", "ba"])
@pytest.mark.parametrize("k_max", [113, 114])
def test_fp64_long_solves_match_oracle(ctx, mode, k_max):
    geom = synth.par2d(64, 89, 91)
    op, xt, b, en = problem(geom, 1002, 0.01)
    kw = dict(use_dp=True, tau=1.0, noise_norm=en)
    ref = oracle.gkb(op, MODES[mode][0], b, k_max, **kw)
    note("fp64 long solve %s k_max=%d" % (mode, k_max))
    res, x = gpu_solve(ctx, geom, mode, b, torch.float64, k_max, **kw)
    assert (res.k_stop, res.reason) == (ref.k_stop, ref.reason)
    k = ref.k_stop
    assert rel(x, ref.x.reshape(-1)) <= 1e-10
    assert np.allclose(res.alpha[:k], ref.alpha[:k], rtol=1e-11)
    assert np.allclose(res.t[:k + 1], ref.t[:k + 1], rtol=1e-11)


@pytest.mark.parametrize("k_max", [227, 228])
def test_fp32_long_solves_match_oracle(ctx, k_max):
    geom = synth.fan2d(96, 143, 160)
    op, xt, b, en = problem(geom, 2002, 0.01)
    b32 = np.float32(b).astype(np.float64)
    ref = oracle.gkb(op, oracle.MODE_BA, b32, k_max, use_dp=True, tau=1.0, noise_norm=en)
    note("fp32 long solve k_max=%d" % k_max)
    res, x = gpu_solve(ctx, geom, "ba", b32, torch.float32, k_max, use_dp=True, tau=1.0, noise_norm=en)
    assert ref.reason == oracle.STOP_DP
    assert (res.k_stop, res.reason) == (ref.k_stop, ref.reason)
    assert rel(x, ref.x.reshape(-1)) <= 1e-4


# Long FP32 runs (150 iterations, no stopping rule) with k_max 150 and 228:
# the iterates do not depend on k_max (the workspace layouts do: partial
# strides, Gram matrix), bit for bit; x at k = 150 matches the oracle.
@pytest.mark.parametrize("mode", ["ab", "ba"])
def test_fp32_long_run_does_not_depend_on_k_max(ctx, mode):
    geom = synth.fan2d(96, 143, 160)
    op, xt, b, en = problem(geom, 2003, 0.01)
    b32 = np.float32(b).astype(np.float64)
    note("fp32 long run %s" % mode)
    r1, x1 = gpu_solve(ctx, geom, mode, b32, torch.float32, 150)
    r2, x2 = gpu_solve(ctx, geom, mode, b32, torch.float32, 228)
    assert r1.k_stop == 150 and r2.k_stop == 228
    assert np.array_equal(r1.alpha[:150], r2.alpha[:150])
    assert np.array_equal(r1.t[:151], r2.t[:151])
    ref = oracle.gkb(op, MODES[mode][0], b32, 150)
    assert rel(x1, ref.x.reshape(-1)) <= 1e-4


# Past 512 columns the reorthogonalisation's coefficient kernel gives each
# thread a row, and past 1024 it takes the rows in several rounds.  On a
# 33x33 image with 61 views (M of full rank n = 1089, no rotation symmetry)
# n iterations fill the whole space, so x_n is the full-space solution,
# computed here from the oracle's dense A and B: BA, (BA)^-1 B b; AB, B z with
# z the least-norm minimiser of ||A B z - b||.  BA-GKB must also break down
# at k = n: t_{n+1} is then what rounding leaves of a vector orthogonalised
# against a complete orthonormal basis (6e-12 against the 4e-11 threshold,
# and 5e-5 one step earlier); a basis that lost orthogonality runs on.  (AB's
# last step, from n to n + 1, divides by an alpha_{n+1} of about 1e-9 and is
# left out: its x moves by 1e-6.)
@pytest.mark.parametrize("mode", ["ba", "ab"])
def test_fp64_fills_the_space_past_1024_columns(ctx, mode):
    geom = synth.par2d(33, 61)
    op, xt, b, en = problem(geom, 1006, 0.01)
    A, B = dense.dense_A(geom), dense.dense_B(geom)
    if mode == "ba":
        xs = np.linalg.solve(B @ A, B @ b)
    else:
        xs = B @ np.linalg.lstsq(A @ B, b, rcond=None)[0]
    note("fp64 full space %s, n=%d" % (mode, geom.n))
    res, x = gpu_solve(ctx, geom, mode, b, torch.float64, 1200 if mode == "ba" else geom.n)
    note("  k_stop %d reason %d, x rel %.2e" % (res.k_stop, res.reason, rel(x, xs)))
    assert res.k_stop == geom.n
    assert res.reason == (gk.STOP_BREAKDOWN if mode == "ba" else gk.STOP_KMAX)
    assert rel(x, xs) <= 1e-8


# FP32 projectors and vectors, FP64 reductions and projected solve, against
# the FP64 oracle on the same (float32-rounded) data.
@pytest.mark.parametrize("mode", ["ab", "ba"])
@pytest.mark.parametrize("gname", ["par128_v179", "fan96_v143"])
def test_fp32_split_matches_oracle(ctx, mode, gname):
    geom = synth.par2d(128, 179) if gname == "par128_v179" else synth.fan2d(96, 143, 160)
    op, xt, b, en = problem(geom, 2001, 0.01)
    b32 = np.float32(b).astype(np.float64)
    ref = oracle.gkb(op, MODES[mode][0], b32, 60, use_dp=True, tau=1.0, noise_norm=en)
    note("fp32 %s %s" % (gname, mode))
    res, x = gpu_solve(ctx, geom, mode, b32, torch.float32, 60, use_dp=True, tau=1.0, noise_norm=en)
    assert ref.reason == oracle.STOP_DP
    assert (res.k_stop, res.reason) == (ref.k_stop, ref.reason)
    assert rel(x, ref.x.reshape(-1)) <= 1e-4
    # near-repeated singular values amplify float rounding transiently in the
    # residual history; the stopping decision and x are what must agree
    assert np.allclose(res.rho, ref.rho, rtol=1e-3)


def test_fp32_full_size_fan512_properties(ctx):
    # full-size workload: the residual the solver reports equals ||A x - b||
    # evaluated by the oracle on the returned x, and AB residuals decrease
    geom = synth.workload_fan512()
    op, xt, b, en = problem(geom, 2000, 0.005)
    for mode in ("ba", "ab"):
        note("fp32 fan512 %s 12 its" % mode)
        res, x = gpu_solve(ctx, geom, mode, np.float32(b), torch.float32, 12)
        assert res.k_stop == 12
        r_or = np.linalg.norm(op.A(x).reshape(-1) - np.float32(b).astype(np.float64))
        assert res.residual == pytest.approx(r_or, rel=2e-4)
        if mode == "ab":
            assert np.all(np.diff(res.rho) <= 1e-4 * res.rho[0])


def test_fp32_full_size_fan512_first_iterations_match_oracle(ctx):
    geom = synth.workload_fan512()
    op, xt, b, en = problem(geom, 2001, 0.005)
    b32 = np.float32(b)
    ref = oracle.gkb(op, oracle.MODE_BA, b32.astype(np.float64), 3)
    note("fp32 fan512 ba 3 its vs oracle")
    res, x = gpu_solve(ctx, geom, "ba", b32, torch.float32, 3)
    assert rel(x, ref.x.reshape(-1)) <= 1e-4
    assert np.allclose(res.alpha[:3], ref.alpha[:3], rtol=1e-5)


def test_solve_is_deterministic(ctx):
    geom = synth.par2d(96, 120)
    op, xt, b, en = problem(geom, 5, 0.02)
    note("determinism solve")
    r1, x1 = gpu_solve(ctx, geom, "ba", np.float32(b), torch.float32, 25)
    r2, x2 = gpu_solve(ctx, geom, "ba", np.float32(b), torch.float32, 25)
    assert np.array_equal(x1, x2) and np.array_equal(r1.rho, r2.rho)


def test_zero_rhs_is_breakdown_with_zero_solution(ctx):
    geom = synth.par2d(32, 20)
    note("zero rhs")
    res, x = gpu_solve(ctx, geom, "ba", np.zeros(geom.m), torch.float32, 10)
    assert res.k_stop == 0 and res.reason == gk.STOP_BREAKDOWN
    assert not x.any()
    assert res.alpha1 == 0.0 and res.t1 == 0.0
    assert np.array_equal(res.alpha, [0.0]) and np.array_equal(res.t, [0.0])


def test_nonfinite_rhs_rejected(ctx):
    geom = synth.par2d(32, 20)
    b = np.ones(geom.m)
    b[7] = np.nan
    note("nan rhs")
    dev = torch.device("cuda:0")
    xd = torch.full((geom.n,), 3.0, dtype=torch.float32, device=dev)
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_ab_solve(ctx, geom, torch.tensor(b, dtype=torch.float32, device=dev), xd, 5)
    assert e.value.status == gk.GKB_ENONFINITE
    assert torch.all(xd == 3.0)


def test_invalid_options_rejected(ctx):
    geom = synth.par2d(16, 10)
    dev = torch.device("cuda:0")
    b = torch.ones(geom.m, dtype=torch.float32, device=dev)
    x = torch.zeros(geom.n, dtype=torch.float32, device=dev)
    for k_max in (0, 4097):  # k_max in [1, 4096]
        with pytest.raises(gk.GkbError) as e:
            gk.gkb_ba_solve(ctx, geom, b, x, k_max)
        assert e.value.status == gk.GKB_EINVAL
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_ba_solve(ctx, geom, b, x, 5, use_dp=True, tau=0.0, noise_norm=1.0)
    assert e.value.status == gk.GKB_EINVAL
    # the largest k_max allocates its basis and Gram matrix ((k_max + 1)^2
    # doubles) and launches the reorthogonalisation with grids for all its columns; a
    # discrepancy level above ||b|| stops the solve at k = 1
    res = gk.gkb_ba_solve(ctx, geom, b, x, 4096, use_dp=True, tau=1.0, noise_norm=1e30)
    torch.cuda.synchronize()
    assert (res.k_stop, res.reason) == (1, gk.STOP_DP) and torch.isfinite(x).all()


def test_dp_not_reached(ctx):
    geom = synth.par2d(32, 40)
    op, xt, b, en = problem(geom, 9, 0.02)
    note("dp not reached")
    res, x = gpu_solve(ctx, geom, "ba", b, torch.float64, 4, use_dp=True, tau=1e-6, noise_norm=en)
    ref = oracle.gkb(op, oracle.MODE_BA, b, 4, use_dp=True, tau=1e-6, noise_norm=en)
    assert res.reason == gk.STOP_DP_NOT_REACHED == ref.reason and res.k_stop == 4
    assert rel(x, ref.x.reshape(-1)) <= 1e-10


def test_no_reorth_matches_oracle_without_reorth(ctx):
    geom = synth.par2d(32, 39)
    op, xt, b, en = problem(geom, 10, 0.02)
    ref = oracle.gkb(op, oracle.MODE_BA, b, 8, reorth=0)
    note("no reorth")
    res, x = gpu_solve(ctx, geom, "ba", b, torch.float64, 8, reorth=False)
    # without reorthogonalisation the bases drift apart from rounding alone
    assert rel(x, ref.x.reshape(-1)) <= 1e-6
