"""Dense gradient of eigenvalue/eigenvector losses with respect to a diagonal potential.

For A(V) = A0 + diag(V) with full eigendecomposition A = U Lambda U^T (simple
eigenvalues at the indices used), first-order perturbation theory gives
  d lambda_i / d V_j        = U[j, i]^2
  d x_1 / d V_j             = - sum_{l != 1} u_l u_l[j] x_1[j] / (lambda_l - lambda_1)
so for the loss  L = sum_{i<=k} lambda_i + <x_1, g>^2
  dL/dV_j = sum_{i<=k} U[j, i]^2  -  x_1[j] * y_j,
  y = sum_{l != 1} u_l (u_l^T b) / (lambda_l - lambda_1),  b = 2 <g, x_1> g.
The chain to bump amplitudes a_g is dL/da_g = sum_j dL/dV_j phi_g(x_j).
This is the plain definition (dense eigensolver, explicit sums); it is not
part of the paper and follows textbook eigenvalue perturbation theory.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def loss_and_grad_diag(A, k: int, g: np.ndarray):
    """Return (loss, dL/dV (n,), lam[:k], U[:, :k]) for L = sum lam_1..k + <x_1, g>^2."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    lam, U = np.linalg.eigh(0.5 * (Ad + Ad.T))
    x1 = U[:, 0]
    gx = float(g @ x1)
    loss = float(lam[:k].sum() + gx * gx)
    grad = (U[:, :k] ** 2).sum(axis=1)
    b = 2.0 * gx * g
    coef = (U[:, 1:].T @ b) / (lam[1:] - lam[0])
    y = U[:, 1:] @ coef
    grad = grad - x1 * y
    return loss, grad, lam[:k].copy(), U[:, :k].copy()


def loss_value(A, k: int, g: np.ndarray) -> float:
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    lam, U = np.linalg.eigh(0.5 * (Ad + Ad.T))
    return float(lam[:k].sum() + (g @ U[:, 0]) ** 2)


def grad_amplitudes(grad_v: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """dL/da_g = sum_j dL/dV_j phi[j, g]."""
    return phi.T @ grad_v
