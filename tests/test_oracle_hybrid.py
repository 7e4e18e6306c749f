"""Pins of the oracle's hybrid regularisation and enlarged-subspace TSVD
(oracle/hybrid.py; readings of Sec. 1, Sec. 3.1 and Sec. 6 stated there).
None re-runs the oracle's SVD formulas:

* the projected Tikhonov solution against a least-squares solve of the
  stacked system [C; lambda I] u = [beta e_1; 0];
* the discrepancy rule: the residual of that independent solution at the
  chosen lambda equals tau * eta, and lambda = 0 exactly when the
  unregularised projected residual already reaches tau * eta;
* GCV: the function evaluated from the dense influence matrix
  C (C^T C + lambda^2 I)^-1 C^T is no smaller anywhere on a fine grid;
* the full Krylov space: the hybrid solution is the full Tikhonov solution
  of the preconditioned problem at the chosen lambda, and the discrepancy
  rule's lambda is the full problem's discrepancy lambda (brentq on the dense
  matrices); the TSVD solution is the dense TSVD solution of B A;
* the TSVD at full rank is the plain GKB iterate (the C oracle's Jacobi path),
  and the discrepancy rule with eta = 0 reduces to plain GKB;
* the stopping rules act on the literal residuals.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from oracle import dense
from oracle import hybrid as hy
from paper_2606_31153_amd import synth


def random_C(k, seed):
    rng = np.random.default_rng(seed)
    # singular values spread over decades, as in an ill-posed problem
    alpha = np.exp(-0.4 * np.arange(k)) * rng.uniform(0.5, 1.5, k)
    t = np.concatenate([[1.0], np.exp(-0.4 * np.arange(k)) * rng.uniform(0.2, 1.0, k)])
    C = hy.bidiag(alpha, t, k)
    return C, float(rng.uniform(0.5, 2.0))


def stacked_u(C, beta, lam):
    k = C.shape[1]
    M = np.vstack([C, lam * np.eye(k)])
    rhs = np.zeros(M.shape[0])
    rhs[0] = beta
    return np.linalg.lstsq(M, rhs, rcond=None)[0]


def proj_res(C, beta, u):
    r = C @ u
    r[0] -= beta
    return np.linalg.norm(r)


@pytest.mark.parametrize("seed", range(4))
def test_tikhonov_solution_matches_stacked_least_squares(seed):
    C, beta = random_C(9, seed)
    P = hy.Projected(C, beta)
    for lam in (0.0, 1e-4, 1e-2, 0.3, 3.0):
        u = stacked_u(C, beta, lam)
        assert np.allclose(P.u(lam), u, rtol=1e-9, atol=1e-12 * np.abs(u).max())
        assert P.residual(lam) == pytest.approx(proj_res(C, beta, u), rel=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_discrepancy_rule_meets_the_target(seed):
    C, beta = random_C(10, seed)
    P = hy.Projected(C, beta)
    r0 = proj_res(C, beta, np.linalg.lstsq(C, np.eye(11)[0] * beta, rcond=None)[0])
    for frac in (0.2, 0.5, 0.9):
        target = r0 + frac * (beta - r0)
        lam = hy.lambda_dp(P, target)
        assert lam > 0
        assert proj_res(C, beta, stacked_u(C, beta, lam)) == pytest.approx(target, rel=1e-9)
    # below the unregularised residual the subspace cannot reach the target: lambda = 0
    assert hy.lambda_dp(P, 0.9 * r0) == 0.0
    assert hy.lambda_dp(P, 0.0) == 0.0


def dense_gcv(C, beta, lam):
    k = C.shape[1]
    H = C @ np.linalg.solve(C.T @ C + lam * lam * np.eye(k), C.T)
    e1 = np.zeros(k + 1)
    e1[0] = beta
    r = e1 - H @ e1
    return (r @ r) / np.trace(np.eye(k + 1) - H) ** 2


@pytest.mark.parametrize("seed", range(4))
def test_gcv_rule_minimises_the_dense_gcv_function(seed):
    C, beta = random_C(8, seed)
    # a noisy right-hand side direction: rotate beta e_1 by a random residual part
    P = hy.Projected(C, beta)
    lam = hy.lambda_gcv(P)
    s = P.scale
    grid = np.exp(np.linspace(np.log(hy.LAM_LO * s), np.log(hy.LAM_HI * s), 3000))
    g = np.array([dense_gcv(C, beta, z) for z in grid])
    assert dense_gcv(C, beta, lam) <= g.min() * (1.0 + 1e-7)
    assert P.gcv(lam) == pytest.approx(dense_gcv(C, beta, lam), rel=1e-8)


def tiny_problem(seed=5, noise=0.05):
    g = synth.par2d(3, 5, 5)  # n = 9, m = 25: BA is 9 x 9 and nonsingular
    A, B = dense.dense_A(g), dense.dense_B(g)
    op = oracle.Operator(A=A, B=B)
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0, 1, g.n)
    e = rng.standard_normal(g.m)
    e *= noise * np.linalg.norm(A @ xt) / np.linalg.norm(e)
    return g, A, B, op, A @ xt + e, e


def test_full_space_ba_hybrid_is_full_tikhonov():
    g, A, B, op, b, e = tiny_problem()
    M, rhs = B @ A, B @ b
    eta = np.linalg.norm(B @ e)
    res = hy.hybrid(op, oracle.MODE_BA, b, g.n, hy.RULE_DP, 1.0, eta)
    assert res.k_stop == g.n
    lam = res.lam[-1]
    assert lam > 0

    def full(l):
        return np.linalg.solve(M.T @ M + l * l * np.eye(g.n), M.T @ rhs)

    x = full(lam)
    assert np.linalg.norm(res.x.reshape(-1) - x) <= 1e-8 * np.linalg.norm(x)
    lam_ref = brentq(lambda l: np.linalg.norm(M @ full(l) - rhs) - eta, 1e-8, 1e3, xtol=1e-14, rtol=1e-13)
    assert lam == pytest.approx(lam_ref, rel=1e-7)


def test_full_space_ab_hybrid_is_full_tikhonov():
    g, A, B, op, b, e = tiny_problem(6)
    M = A @ B  # 25 x 25, rank 9: the Krylov space of A B breaks down at rank 9
    res = hy.hybrid(op, oracle.MODE_AB, b, g.m, hy.RULE_GCV)
    k = res.k_stop
    assert res.reason == oracle.STOP_BREAKDOWN and k == np.linalg.matrix_rank(M)
    lam = res.lam[-1]
    # min ||A B y - b||^2 + lam^2 ||y||^2 over the Krylov space = over range(M^T) = over R^m (the
    # Tikhonov solution lies in range(M^T)); x = B y
    y = np.linalg.solve(M.T @ M + lam * lam * np.eye(g.m), M.T @ b)
    x = B @ y
    assert np.linalg.norm(res.x.reshape(-1) - x) <= 1e-7 * np.linalg.norm(x)


def test_full_space_tsvd_is_dense_tsvd():
    g, A, B, op, b, e = tiny_problem(7)
    M, rhs = B @ A, B @ b
    U, s, Vt = np.linalg.svd(M)
    for r in (2, 5, 9):
        x = Vt[:r].T @ ((U[:, :r].T @ rhs) / s[:r])
        xo = hy.tsvd(op, oracle.MODE_BA, b, g.n, r).reshape(-1)
        assert np.linalg.norm(xo - x) <= 1e-8 * np.linalg.norm(x), r


@pytest.mark.parametrize("mode", [oracle.MODE_AB, oracle.MODE_BA])
def test_tsvd_at_full_rank_and_dp_with_zero_eta_are_plain_gkb(mode):
    g = synth.par2d(12, 15)
    op = oracle.Operator(A=dense.dense_A(g), B=dense.dense_B(g))
    b = op.A(synth.ellipse_phantom(12, 3)).reshape(-1)
    b, en = synth.add_noise(b, synth.noise_direction(g.m, 3), 0.02)
    K = 10
    plain = oracle.gkb(op, mode, b, K)
    xt = hy.tsvd(op, mode, b, K, K).reshape(-1)
    assert np.linalg.norm(xt - plain.x.reshape(-1)) <= 1e-9 * np.linalg.norm(plain.x)
    res = hy.hybrid(op, mode, b, K, hy.RULE_DP, 1.0, 0.0)
    assert np.all(res.lam == 0.0)
    assert np.linalg.norm(res.x.reshape(-1) - plain.x.reshape(-1)) <= 1e-9 * np.linalg.norm(plain.x)
    assert np.allclose(res.rho, plain.rho, rtol=1e-9)


@pytest.mark.parametrize("mode", [oracle.MODE_AB, oracle.MODE_BA])
def test_hybrid_stopping_rules(mode):
    g = synth.par2d(16, 20)
    op = oracle.Operator(A=dense.dense_A(g), B=dense.dense_B(g))
    xtrue = synth.ellipse_phantom(16, 9)
    b, en = synth.add_noise(op.A(xtrue).reshape(-1), synth.noise_direction(g.m, 9), 0.05)
    full = hy.hybrid(op, mode, b, 20, hy.RULE_GCV)
    assert full.reason in (oracle.STOP_KMAX, oracle.STOP_BREAKDOWN)
    assert np.all(np.isfinite(full.lam)) and np.all(full.lam > 0)
    # each rho_k is the literal residual of the returned iterate
    last = hy.hybrid(op, mode, b, full.k_stop, hy.RULE_GCV)
    assert np.linalg.norm(op.A(last.x).reshape(-1) - b) == pytest.approx(full.rho[-1], rel=1e-12)
    crossed = np.nonzero(full.rho <= 1.0 * en)[0]
    res = hy.hybrid(op, mode, b, 20, hy.RULE_GCV, use_dp=True, tau=1.0, noise_norm=en)
    if crossed.size:
        assert (res.k_stop, res.reason) == (crossed[0] + 1, oracle.STOP_DP)
    else:
        assert res.reason == oracle.STOP_DP_NOT_REACHED
    ch = np.abs(np.diff(full.rho)) / full.rho[:-1]
    eps = 0.5 * (np.sort(ch)[len(ch) // 2] + np.sort(ch)[len(ch) // 2 + 1])
    res = hy.hybrid(op, mode, b, 20, hy.RULE_GCV, rns_eps=eps)
    assert (res.k_stop, res.reason) == (int(np.nonzero(ch < eps)[0][0]) + 2, oracle.STOP_RNS)
