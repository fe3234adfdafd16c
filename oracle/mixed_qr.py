"""Algorithm 2 (mixed-precision QR factorization), section 3.2.

Given W (n x m, full column rank) in working precision:
  1. lower(W) = Q_l R_l by Householder QR in the lower precision;
  2. V = W * working(R_l)^{-1}, an upper triangular solve in working precision;
  3. V^T V = L L^T, Cholesky in working precision;
  4. Q = V L^{-T}, an upper triangular solve in working precision.
Then W = Q R with R = L^T working(R_l) and Q^T Q = I (the algorithm's ENSURE).

Step 1 uses LAPACK geqrf in float32 (numpy.linalg.qr), the Householder QR that
section 3.2 names; steps 2-4 use float64 LAPACK triangular solves and potrf.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def mixed_qr(W: np.ndarray):
    """Return (Q, R) of Algorithm 2 for W (float64, n x m)."""
    W = np.asarray(W, dtype=np.float64)
    _, Rl = np.linalg.qr(W.astype(np.float32), mode="reduced")      # step 1, float32 Householder
    Rw = Rl.astype(np.float64)                                        # working(R_l)
    # step 2: V = W Rw^{-1}  <=>  Rw^T V^T = W^T
    V = sla.solve_triangular(Rw, W.T, trans="T", lower=False).T
    # step 3: V^T V = L L^T
    L = np.linalg.cholesky(V.T @ V)
    # step 4: Q = V L^{-T}  <=>  L Q^T = V^T
    Q = sla.solve_triangular(L, V.T, lower=True).T
    R = L.T @ Rw
    return Q, R


def householder_qr(W: np.ndarray):
    """FP64 Householder QR (LAPACK geqrf/orgqr), the working-precision comparison."""
    return np.linalg.qr(np.asarray(W, dtype=np.float64), mode="reduced")
