"""Hybrid regularisation and the enlarged-subspace TSVD on AB-/BA-GKB.

Test infrastructure only (the oracle): imported by the test-suite alone, never
by the product library, with which it shares no code.

The paper names hybrid regularisation (a regularisation parameter chosen
inside the Krylov subspace, on the projected problem) as what motivates the
projected SVD solve and as future work (Sec. 1, Sec. 6), and discusses and
declines an enlarged Krylov subspace truncated back to rank k (Sec. 3.1).  It
fixes no rule; the readings here are:

* Iteration k solves the projected Tikhonov problem
  min ||C_k u - t_1 e_1||^2 + lambda_k^2 ||u||^2 (C_k the (k+1) x k lower
  bidiagonal of alpha_1..alpha_k and t_2..t_{k+1}) with lambda_k chosen on
  C_k alone, by one of two rules:

  - discrepancy (RULE_DP): ||C_k u - t_1 e_1|| = tau * eta, eta the noise norm
    in the space of the projected residual (AB: ||e||, since
    ||C_k u - t_1 e_1|| = ||A B Q_k u - b|| for an orthonormal S_{k+1}; BA:
    ||B e||, since it equals ||B A Q_k u - B b||).  The projected residual
    grows with lambda, so the root is unique.  lambda_k = 0 while the residual
    at lambda = 0 is at least tau * eta (the subspace cannot yet fit the data
    to the noise level), lambda_lo or lambda_hi where the root lies outside
    [lambda_lo, lambda_hi];
  - generalised cross validation (RULE_GCV): lambda_k minimises
    G_k(lambda) = ||C_k u - t_1 e_1||^2 / trace(I_{k+1} - H_k(lambda))^2,
    H_k(lambda) = C_k (C_k^T C_k + lambda^2 I)^-1 C_k^T, over
    [lambda_lo, lambda_hi] (the projected GCV function with unit weight).

  with [lambda_lo, lambda_hi] = [1e-10 s, 10 s], s = max_i ||C_k e_i||.
  x_k = Q_k u_k (BA) or B Q_k u_k (AB); rho_k = ||A x_k - b||, evaluated
  literally; the stopping rules of the GKB solves act on rho_k.

* Enlarged subspace (TSVD): K iterations, then x = Q_K u (B Q_K u) with u the
  rank-r truncated SVD solution of min ||C_K u - t_1 e_1||:
  u = sum_{i <= r} (t_1 U_{1i} / sigma_i) v_i.

The Krylov bases do not depend on the projected solve, so the GKB oracle is
run once (with its bases) and every iteration's projected problem is solved
from its alpha and t.  The SVD of C_k is NumPy's.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import MODE_AB, MODE_BA, STOP_BREAKDOWN, STOP_DP, STOP_DP_NOT_REACHED, STOP_KMAX, STOP_RNS, Operator, gkb

RULE_DP, RULE_GCV = 1, 2
LAM_LO, LAM_HI = 1e-10, 1e1


def bidiag(alpha, t, k: int) -> np.ndarray:
    """C_k from the oracle's histories (alpha[i] = alpha_{i+1}, t[i] = t_{i+1})."""
    C = np.zeros((k + 1, k))
    for i in range(k):
        C[i, i] = alpha[i]
        C[i + 1, i] = t[i + 1]
    return C


class Projected:
    """The projected problem min ||C u - beta e_1|| through the full SVD of C."""

    def __init__(self, C: np.ndarray, beta: float):
        self.k = C.shape[1]
        U, self.sig, Vt = np.linalg.svd(C, full_matrices=True)
        self.V = Vt.T
        # g_i = beta U_{1i}: the first k pair with sigma_i, the last is the
        # part of beta e_1 outside the range of C
        self.g = beta * U[0, :]
        self.scale = float(np.max(np.sqrt(np.sum(C * C, axis=0))))

    def residual(self, lam: float) -> float:
        """||C u(lambda) - beta e_1||."""
        s2 = self.sig ** 2
        f = lam * lam / (s2 + lam * lam) if lam > 0 else (s2 == 0).astype(float)
        return float(np.sqrt(np.sum((f * self.g[: self.k]) ** 2) + np.sum(self.g[self.k:] ** 2)))

    def gcv(self, lam: float) -> float:
        s2 = self.sig ** 2
        den = 1.0 + np.sum(lam * lam / (s2 + lam * lam))
        return self.residual(lam) ** 2 / den ** 2

    def u(self, lam: float) -> np.ndarray:
        den = self.sig ** 2 + lam * lam
        d = np.where(den > 0, self.sig / np.where(den > 0, den, 1.0), 0.0)
        return self.V @ (d * self.g[: self.k])

    def u_tsvd(self, r: int) -> np.ndarray:
        return self.V[:, :r] @ (self.g[:r] / self.sig[:r])


def lambda_dp(P: Projected, target: float) -> float:
    lo, hi = LAM_LO * P.scale, LAM_HI * P.scale
    if P.residual(0.0) >= target:
        return 0.0
    if P.residual(lo) >= target:
        return lo
    if P.residual(hi) <= target:
        return hi
    a, b = np.log(lo), np.log(hi)
    for _ in range(200):  # bisection on ln(lambda) down to rounding
        c = 0.5 * (a + b)
        if P.residual(np.exp(c)) < target:
            a = c
        else:
            b = c
        if b - a <= 1e-15 * max(1.0, abs(a)):
            break
    return float(np.exp(0.5 * (a + b)))


def lambda_gcv(P: Projected) -> float:
    lo, hi = np.log(LAM_LO * P.scale), np.log(LAM_HI * P.scale)
    grid = np.linspace(lo, hi, 801)
    vals = np.array([P.gcv(np.exp(z)) for z in grid])
    j = int(np.argmin(vals))
    a, b = grid[max(j - 1, 0)], grid[min(j + 1, grid.size - 1)]
    # golden-section search between the grid neighbours of the grid minimum
    r = 0.5 * (np.sqrt(5.0) - 1.0)
    c, d = b - r * (b - a), a + r * (b - a)
    fc, fd = P.gcv(np.exp(c)), P.gcv(np.exp(d))
    while b - a > 1e-12:
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - r * (b - a)
            fc = P.gcv(np.exp(c))
        else:
            a, c, fc = c, d, fd
            d = a + r * (b - a)
            fd = P.gcv(np.exp(d))
    z = 0.5 * (a + b)
    return float(np.exp(z)) if P.gcv(np.exp(z)) <= vals[j] else float(np.exp(grid[j]))


@dataclass
class HybridResult:
    x: np.ndarray
    k_stop: int
    reason: int
    lam: np.ndarray     # lambda_k, k = 1..k_stop
    rho: np.ndarray     # ||A x_k - b||
    pres: np.ndarray    # ||C_k u_k - t_1 e_1||
    alpha: np.ndarray
    t: np.ndarray


def _assemble(op: Operator, mode: int, Q: np.ndarray, u: np.ndarray) -> np.ndarray:
    z = Q[: u.size].T @ u
    return op.B(z).reshape(-1) if mode == MODE_AB else z


def hybrid(op: Operator, mode: int, b, k_max: int, rule: int, tau_proj: float = 1.0, eta_proj: float = 0.0,
           use_dp: bool = False, tau: float = 1.0, noise_norm: float = 0.0, rns_eps: float = 0.0) -> HybridResult:
    """Hybrid AB-GKB (mode 0) or BA-GKB (mode 1): lambda_k by `rule` on C_k,
    then the discrepancy principle on rho_k (use_dp), residual norm
    stagnation (rns_eps), breakdown or k_max, as for the plain solves."""
    if mode not in (MODE_AB, MODE_BA) or rule not in (RULE_DP, RULE_GCV):
        raise ValueError("hybrid: mode AB or BA, rule DP or GCV")
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    base = gkb(op, mode, b, k_max, want_bases=True)
    beta = base.t1
    K = base.k_stop
    lams, rhos, press = [], [], []
    x = np.zeros(op.n)
    reason = base.reason if base.reason == STOP_BREAKDOWN else STOP_KMAX
    k_stop = K
    for k in range(1, K + 1):
        P = Projected(bidiag(base.alpha, base.t, k), beta)
        lam = lambda_dp(P, tau_proj * eta_proj) if rule == RULE_DP else lambda_gcv(P)
        u = P.u(lam)
        x = _assemble(op, mode, base.Q, u)
        rho = float(np.linalg.norm(op.A(x).reshape(-1) - b))
        lams.append(lam)
        rhos.append(rho)
        press.append(P.residual(lam))
        if use_dp and rho <= tau * noise_norm:
            reason, k_stop = STOP_DP, k
            break
        if rns_eps > 0 and k >= 2 and abs(rhos[-2] - rho) < rns_eps * rhos[-2]:
            reason, k_stop = STOP_RNS, k
            break
    else:
        if use_dp and reason == STOP_KMAX:
            reason = STOP_DP_NOT_REACHED
    return HybridResult(x=x.reshape(op.image_shape), k_stop=k_stop, reason=reason, lam=np.array(lams),
                        rho=np.array(rhos), pres=np.array(press), alpha=base.alpha, t=base.t)


def tsvd(op: Operator, mode: int, b, k_big: int, rank: int) -> np.ndarray:
    """Enlarged-subspace TSVD: k_big GKB iterations (fewer on breakdown),
    then the rank-`rank` truncated SVD solution of the projected problem."""
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    base = gkb(op, mode, b, k_big, want_bases=True)
    K = base.k_stop
    if not 1 <= rank <= K:
        raise ValueError("tsvd: rank must be in [1, k_stop]")
    P = Projected(bidiag(base.alpha, base.t, K), base.t1)
    return _assemble(op, mode, base.Q, P.u_tsvd(rank)).reshape(op.image_shape)
