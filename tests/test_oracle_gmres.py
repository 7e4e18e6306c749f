"""Pins of the oracle's AB-GMRES and BA-GMRES (Sec. 2.1, Algs. "AB-GMRES" and
"BA-GMRES"), none of which re-runs the oracle's own formulas:

* brute force: x_k from an orthonormal basis of the Krylov space K_k(M, r_0)
  (QR of the Krylov matrix) and a least-squares solve of the minimisation the
  algorithms state (AB: min ||A B y - b|| over y in K_k(AB, b), x = B y;
  BA: min ||B A x - B b|| over x in K_k(BA, B b));
* the Arnoldi relation M Q_k = Q_{k+1} H_k (eq. (Arn iter)) and QᵀQ = I;
* scipy's GMRES (unrestarted, k steps) on the square systems;
* GMRES minimises over nested spaces: its projected residual never grows, and
  for AB it is the data residual ||A x_k - b|| itself;
* the full space: with M nonsingular, x_n solves the square system exactly;
* the stopping rules: the discrepancy stop at the first crossing, monotone in
  tau; residual norm stagnation at the first small relative change; breakdown
  on an invariant subspace.
"""
import numpy as np
import pytest
from scipy.sparse.linalg import gmres as scipy_gmres

import oracle
from oracle import dense
from paper_2606_31153_amd import synth

GEOMS = {
    "par_over": synth.par2d(8, 9, 13),     # m = 117 > n = 64
    "par_under": synth.par2d(10, 4, 12),   # m = 48 < n = 100
    "fan": synth.fan2d(8, 7, 17, src_dist=20.0),
}
MODES = {"ab": oracle.MODE_AB, "ba": oracle.MODE_BA}


def problem(gname, seed=0):
    g = GEOMS[gname]
    A, B = dense.dense_A(g), dense.dense_B(g)
    b = np.random.default_rng(seed).standard_normal(g.m)
    return A, B, b, oracle.Operator(A=A, B=B)


def krylov_solution(A, B, b, mode, k):
    """x_k by brute force: orthonormal Krylov basis by QR, least squares."""
    if mode == oracle.MODE_AB:
        M, r0 = A @ B, b
    else:
        M, r0 = B @ A, B @ b
    K = np.empty((r0.size, k))
    v = r0.copy()
    for j in range(k):
        K[:, j] = v
        v = M @ v
    V, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(M @ V, r0, rcond=None)
    return (B @ (V @ y)) if mode == oracle.MODE_AB else V @ y


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("gname", list(GEOMS))
def test_gmres_equals_brute_force_krylov_least_squares(gname, mode):
    A, B, b, op = problem(gname)
    for k in range(1, 7):
        r = oracle.gmres(op, MODES[mode], b, k)
        ref = krylov_solution(A, B, b, MODES[mode], k)
        assert r.k_stop == k
        assert np.linalg.norm(r.x - ref) <= 1e-8 * np.linalg.norm(ref), k


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("gname", list(GEOMS))
def test_arnoldi_relation_and_orthonormal_basis(gname, mode):
    A, B, b, op = problem(gname, 1)
    k = 10
    r = oracle.gmres(op, MODES[mode], b, k, want_bases=True)
    M = A @ B if mode == "ab" else B @ A
    Q = r.Q.T  # dimq x (k + 1)
    assert np.linalg.norm(M @ Q[:, :k] - Q @ r.H) <= 1e-12 * np.linalg.norm(M) * np.sqrt(k)
    assert np.max(np.abs(Q.T @ Q - np.eye(k + 1))) <= 1e-10
    # upper Hessenberg: zero below the first subdiagonal
    assert np.all(np.tril(r.H, -2) == 0.0)


@pytest.mark.parametrize("mode", list(MODES))
def test_gmres_matches_scipy(mode):
    A, B, b, op = problem("par_over", 2)
    M, rhs = (A @ B, b) if mode == "ab" else (B @ A, B @ b)
    for k in (3, 5, 8):
        r = oracle.gmres(op, MODES[mode], b, k)
        y, info = scipy_gmres(M, rhs, x0=np.zeros(rhs.size), rtol=0.0, atol=0.0, restart=k, maxiter=1)
        ref = B @ y if mode == "ab" else y
        assert np.linalg.norm(r.x - ref) <= 1e-8 * np.linalg.norm(ref), k


@pytest.mark.parametrize("gname", list(GEOMS))
def test_minimised_residuals(gname):
    A, B, b, op = problem(gname, 3)
    ab = oracle.gmres(op, oracle.MODE_AB, b, 12)
    ba = oracle.gmres(op, oracle.MODE_BA, b, 12)
    # AB-GMRES minimises ||b - A B y||: its projected residual is the data residual
    assert np.allclose(ab.pres, ab.rho, rtol=1e-10)
    assert np.all(np.diff(ab.rho) <= 1e-12 * ab.rho[0])
    # BA-GMRES minimises ||B (b - A x)||
    bres = [np.linalg.norm(B @ (b - A @ oracle.gmres(op, oracle.MODE_BA, b, k).x)) for k in range(1, 13)]
    assert np.allclose(ba.pres, bres, rtol=1e-9)
    assert np.all(np.diff(ba.pres) <= 1e-12 * ba.pres[0])


def test_full_space_solves_the_square_system():
    # 3 x 3 image, 5 views: B A (9 x 9) nonsingular; BA-GMRES after 9 steps
    # solves B A x = B b, and AB-GMRES on the square A B reaches the
    # least-squares solution of A B y = b
    g = synth.par2d(3, 5, 5)
    A, B = dense.dense_A(g), dense.dense_B(g)
    op = oracle.Operator(A=A, B=B)
    b = np.random.default_rng(4).standard_normal(g.m)
    BA = B @ A
    assert np.linalg.matrix_rank(BA) == g.n
    r = oracle.gmres(op, oracle.MODE_BA, b, g.n)
    ref = np.linalg.solve(BA, B @ b)
    assert np.linalg.norm(r.x - ref) <= 1e-9 * np.linalg.norm(ref)
    r = oracle.gmres(op, oracle.MODE_AB, b, g.m)
    y, *_ = np.linalg.lstsq(A @ B, b, rcond=None)
    ref = B @ y
    assert np.linalg.norm(A @ r.x - b) == pytest.approx(np.linalg.norm(A @ ref - b), rel=1e-9)


def test_stopping_rules():
    g = synth.par2d(16, 20)
    A, B = dense.dense_A(g), dense.dense_B(g)
    op = oracle.Operator(A=A, B=B)
    x = synth.ellipse_phantom(16, 7)
    b, en = synth.add_noise(A @ x.reshape(-1), synth.noise_direction(g.m, 7), 0.02)
    for mode in (oracle.MODE_AB, oracle.MODE_BA):
        plain = oracle.gmres(op, mode, b, 30)
        crossed = np.nonzero(plain.rho <= en)[0]
        r = oracle.gmres(op, mode, b, 30, use_dp=True, tau=1.0, noise_norm=en)
        if crossed.size:
            assert (r.k_stop, r.reason) == (crossed[0] + 1, oracle.STOP_DP)
            assert np.array_equal(r.x, oracle.gmres(op, mode, b, r.k_stop).x)
        else:
            assert r.reason == oracle.STOP_DP_NOT_REACHED
        # a looser tau stops no later
        r2 = oracle.gmres(op, mode, b, 30, use_dp=True, tau=1.5, noise_norm=en)
        assert r2.k_stop <= r.k_stop
        # residual norm stagnation: the first k >= 2 with a small relative change
        ch = np.abs(np.diff(plain.rho)) / plain.rho[:-1]
        eps = 0.5 * (np.sort(ch)[len(ch) // 2] + np.sort(ch)[len(ch) // 2 + 1])
        k_rns = int(np.nonzero(ch < eps)[0][0]) + 2
        r = oracle.gmres(op, mode, b, 30, rns_eps=eps)
        assert (r.k_stop, r.reason) == (k_rns, oracle.STOP_RNS)


def test_breakdown_on_an_invariant_subspace():
    # M = B A = I on a 2-pixel problem: r_0 spans the whole Krylov space at k = 1
    A = np.eye(4)[:, :2] * 2.0
    B = np.eye(4)[:2, :] * 0.5
    op = oracle.Operator(A=A, B=B)
    b = np.array([1.0, -2.0, 0.0, 0.0])
    r = oracle.gmres(op, oracle.MODE_BA, b, 5)
    assert (r.k_stop, r.reason) == (1, oracle.STOP_BREAKDOWN)
    assert np.allclose(r.x, [0.5, -1.0], rtol=1e-14)
    # zero right-hand side: nothing to do
    r = oracle.gmres(op, oracle.MODE_AB, np.zeros(4), 5)
    assert (r.k_stop, r.reason) == (0, oracle.STOP_BREAKDOWN)
    assert not r.x.any()
    with pytest.raises(ValueError):
        oracle.gmres(op, oracle.MODE_GKB, b, 5)
