"""Plain FP64 LOBPCG following Algorithm 3's working-precision loop (section 3.3).

Steps, in the algorithm's order and notation:
  line 2      P = [], Theta = X^T A X.  Reading: X0 is orthonormalised (Householder
              QR) and one Rayleigh-Ritz step on span(X0) makes Theta diagonal and
              X Ritz vectors, so the per-column test uses Theta(j, j).
  line 4      R = A X - X Theta.
  line 5      n_c = length of the leading run of columns satisfying the
              convergence test (eq. (stop) of section 5.1, or the normalised
              residual ||r_j|| / (||A||_2 ||x_j||) <= tol).
  line 6-8    return X(:, 1:k), Theta(1:k, 1:k) once n_c >= k.
  line 9-10   W = working(f_T(lower(R))) (oracle.precond).
  line 11     W -= [X, P]([X, P]^T W), twice (block classical Gram-Schmidt).
  line 12     W = Q of a QR factorization of W (Householder here, so the oracle
              stays independent of Algorithm 2 and is orthonormal even for a
              rank-deficient W).
  line 13     A_p = S^T A S with S = [X, P, W]; A S is formed explicitly.
  line 14     A_p C = C D, eigenvalues ascending.
  line 15     V = orthonormal factor of C(1:m, m+1:c)^T, c = columns of S.
  line 16     X = S C(:, 1:m), P = S C(:, m+1:c) V, Theta = D(1:m, 1:m).
Lines 15-16 print the column ranges as m+1:n and m+1:2m; with c = 3m columns the
consistent reading (the improved Hetmaniuk-Lehoucq trick of section 2) is
m+1:c for both, which is the printed text at the first iteration (c = 2m).

Everything is float64 except the preconditioner, which runs in the factor's
precision.

Line 1 (mixed_lobpcg): the start block of the working-precision loop is computed
by the same LOBPCG run entirely in single precision (every array float32:
single(A), single(X0), products, QR, Rayleigh-Ritz, residual, and the
preconditioner's output) until the test holds with the first-stage tolerance
(section 5.1 sets it to 5e-6); that X, widened to float64, then enters line 2
with P = [].
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .precond import Preconditioner


@dataclasses.dataclass
class Result:
    evals: np.ndarray
    evecs: np.ndarray
    iters: int
    converged: bool
    residuals: np.ndarray
    history: list
    block: np.ndarray = None   # all m columns of X at exit


def _sym(H):
    return 0.5 * (H + H.T)


def residual_norms(A, X, theta, norm_a, mode="bj"):
    """Per-column normalised residuals.

    mode "bj":    ||A x_j - theta_j x_j|| / (||A||_2 ||x_j||)
    mode "paper": ||A x_j - theta_j x_j|| / ((||A||_2 + |theta_j|) ||x_j||)   (eq. (stop))
    """
    R = A @ X - X * theta
    rn = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(X, axis=0)
    if mode == "paper":
        return rn / ((norm_a + np.abs(theta)) * xn)
    return rn / (norm_a * xn)


def leading_converged(flags) -> int:
    """n_c: number of leading columns that all satisfy the test (reading of line 5)."""
    nc = 0
    for f in flags:
        if not f:
            break
        nc += 1
    return nc


def rayleigh_ritz_start(A, X0, dtype=np.float64):
    """Line 2 with the diagonal-Theta reading: orthonormalise X0, then Rayleigh-Ritz on span(X0)."""
    X, _ = np.linalg.qr(np.asarray(X0, dtype=dtype))
    AX = A @ X
    theta, Y = np.linalg.eigh(_sym(X.T @ AX))
    return X @ Y, theta


def hl_update(S, C, D, m):
    """Lines 15-16: X = S C(:,1:m); P = S C(:,m+1:c) V with V = Q of C(1:m, m+1:c)^T."""
    V, _ = np.linalg.qr(C[:m, m:].T)           # (c-m) x m, orthonormal columns
    X = S @ C[:, :m]
    P = S @ (C[:, m:] @ V)
    return X, P, D[:m].copy()


def lobpcg(A, X0, k: int, tol: float, *, precond=None, precond_precision="fp64",
           norm_a: float, maxit: int = 1000, stop: str = "bj", eig_tol: float = 0.0,
           callback=None, dtype=np.float64) -> Result:
    """k smallest eigenpairs of the SPD matrix A (dense ndarray or scipy sparse).

    dtype=np.float32 runs every step in single precision (the lower-precision LOBPCG of line 1):
    A and X0 are rounded to float32 and the preconditioner's output too."""
    n, m = X0.shape
    if not (1 <= k <= m) or 3 * m > n:
        raise ValueError("need 1 <= k <= m and 3m <= n")
    if precond is None:
        precond = Preconditioner(A, precond_precision)
    if dtype != np.float64:
        A = A.astype(dtype)
        f_t = precond
        precond = lambda R: f_t(R).astype(dtype)            # noqa: E731
    X, theta = rayleigh_ritz_start(A, X0, dtype)
    P = None
    history = []
    res = None
    for it in range(1, maxit + 1):
        AX = A @ X
        R = AX - X * theta                                           # line 4
        rn = np.linalg.norm(R, axis=0)
        xn = np.linalg.norm(X, axis=0)
        if stop == "paper":
            res = rn / ((norm_a + np.abs(theta)) * xn)
        else:
            res = rn / (norm_a * xn)
        ok = res <= tol
        if eig_tol > 0.0:
            gap = np.maximum(theta[m - 1] - theta, 0.0)
            ok &= rn ** 2 <= eig_tol * np.abs(theta) * gap
        nc = leading_converged(ok)                                   # line 5
        history.append((it, nc, float(res[:k].max())))
        if callback is not None:
            callback(it, X, P, theta, res)
        if nc >= k:                                                  # lines 6-8
            return Result(theta[:k].copy(), X[:, :k].copy(), it, True, res[:k].copy(), history, X.copy())
        W = precond(R)                                               # lines 9-10
        B = X if P is None else np.hstack([X, P])
        for _ in range(2):                                           # line 11
            W = W - B @ (B.T @ W)
        W, _ = np.linalg.qr(W)                                       # line 12
        S = np.hstack([X, W]) if P is None else np.hstack([X, P, W])
        AS = A @ S                                                   # line 13
        D, C = np.linalg.eigh(_sym(S.T @ AS))                        # line 14
        X, P, theta = hl_update(S, C, D, m)                          # lines 15-16
    return Result(theta[:k].copy(), X[:, :k].copy(), maxit, False,
                  res[:k].copy() if res is not None else None, history, X.copy())


@dataclasses.dataclass
class MixedResult:
    evals: np.ndarray
    evecs: np.ndarray
    iters: int            # working-precision loop (lines 2-17)
    stage1_iters: int     # single-precision LOBPCG of line 1
    converged: bool
    stage1_converged: bool
    stage1_X: np.ndarray  # the float32 start block line 1 produced
    residuals: np.ndarray


def mixed_lobpcg(A, X0, k: int, tol: float, tol1: float, *, precond, norm_a: float, maxit: int = 1000,
                 stop: str = "paper") -> MixedResult:
    """Algorithm 3 with line 1: a single-precision LOBPCG from single(X0) to tol1, then the
    working-precision loop from working(X) with P = [] (MPLOBPCG-schol of section 5.1)."""
    s1 = lobpcg(A, X0, k, tol1, precond=precond, norm_a=norm_a, maxit=maxit, stop=stop, dtype=np.float32)
    X1 = s1.block
    s2 = lobpcg(A, X1.astype(np.float64), k, tol, precond=precond, norm_a=norm_a, maxit=maxit, stop=stop)
    return MixedResult(s2.evals, s2.evecs, s2.iters, s1.iters, s2.converged, s1.converged, X1, s2.residuals)
