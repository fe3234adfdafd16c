"""Algorithm 1 (mixed-precision PINVIT) and the rate of Theorem 1 (sections 3.1 and 4).

Algorithm 1: X = Q of X~; Theta = X^T A X; R = A X - X Theta; return once the
k smallest pairs pass the test; W = working(f_T(lower(R))); X~ = X - W.

Theorem 1 bounds one step for k = 1: with rho the Rayleigh quotient,
  (rho_{i+1} - lambda_1)/(lambda_2 - rho_{i+1}) <= q^2 (rho_i - lambda_1)/(lambda_2 - rho_i),
  q = gamma + (1 - gamma) lambda_1 / lambda_2,  gamma = ||I - A^{1/2} T A^{1/2}||_2,
when rho_i lies in [lambda_1, lambda_2).
"""
from __future__ import annotations

import numpy as np


def pinvit_k1(A, x0: np.ndarray, precond, steps: int):
    """Single-vector PINVIT; returns the list of Rayleigh quotients rho_0..rho_steps."""
    x = np.asarray(x0, dtype=np.float64).reshape(-1, 1)
    rhos = []
    for _ in range(steps + 1):
        x = x / np.linalg.norm(x)
        Ax = A @ x
        rho = float((x.T @ Ax)[0, 0])
        rhos.append(rho)
        r = Ax - rho * x
        x = x - precond(r)
    return rhos


def rate_bound(gamma: float, lam1: float, lam2: float) -> float:
    q = gamma + (1.0 - gamma) * lam1 / lam2
    return q * q


def ratio(rho: float, lam1: float, lam2: float) -> float:
    return (rho - lam1) / (lam2 - rho)


def mixed_pinvit(A, X0: np.ndarray, k: int, tol: float, precond, norm_a: float, maxit: int = 1000):
    """Block Algorithm 1; returns (theta[:k], X[:, :k], iterations)."""
    Xt = np.asarray(X0, dtype=np.float64)
    for it in range(1, maxit + 1):
        X, _ = np.linalg.qr(Xt)
        AX = A @ X
        H = 0.5 * (X.T @ AX + (X.T @ AX).T)
        th, Y = np.linalg.eigh(H)           # rotate so Theta is diagonal (per-column test)
        X = X @ Y
        AX = AX @ Y
        R = AX - X * th
        res = np.linalg.norm(R, axis=0) / (norm_a * np.linalg.norm(X, axis=0))
        if np.all(res[:k] <= tol):
            return th[:k], X[:, :k], it
        Xt = X - precond(R)
    return th[:k], X[:, :k], maxit
