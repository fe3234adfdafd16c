"""The preconditioner of section 5.1: T = Pi L^{-T} L^{-1} Pi^T with Pi^T A Pi = L L^T.

Section 5.1 applies T by two triangular solves with a Cholesky factor computed
in single precision (DLOBPCG-schol, MPLOBPCG-schol) or double precision
(DLOBPCG-dchol).  Section 3.1 applies the whole of f_T in the lower precision:
W_l = f_T(lower(R)), W = working(W_l).

Dense A: LAPACK potrf/potrs in the factor's precision (scipy.linalg.cho_factor).
Sparse A: an LU factorization without pivoting of the symmetric positive
definite matrix (SuperLU with a symmetric minimum-degree ordering and diagonal
pivots only).  For SPD A, LU without pivoting equals L D L^T, so (LU)^{-1} is
the same operator A^{-1} as (L L^T)^{-1} up to rounding, in the same precision.
The ordering Pi is a fill-reducing symmetric permutation; the eigenpairs do not
depend on it.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class Preconditioner:
    """Callable R (n x m float64) -> W (n x m float64), applying T in `precision`."""

    def __init__(self, A, precision: str = "fp64"):
        if precision not in ("fp64", "fp32"):
            raise ValueError(precision)
        self.precision = precision
        self.dtype = np.float64 if precision == "fp64" else np.float32
        self.sparse = sp.issparse(A)
        if self.sparse:
            Al = sp.csc_matrix(A, dtype=self.dtype)
            self.lu = spla.splu(Al, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                                options={"SymmetricMode": True})
        else:
            Al = np.asarray(A, dtype=self.dtype)
            self.cf = sla.cho_factor(Al, lower=True, check_finite=True)

    def __call__(self, R: np.ndarray) -> np.ndarray:
        Rl = np.asarray(R).astype(self.dtype)          # lower(R), round to nearest
        if self.sparse:
            Wl = self.lu.solve(Rl)
        else:
            Wl = sla.cho_solve(self.cf, Rl)
        return np.asarray(Wl, dtype=self.dtype).astype(np.float64)   # working(W_l)


def lower_factor_dense(A: np.ndarray, precision: str = "fp32") -> np.ndarray:
    """Lower Cholesky factor of dense A computed in `precision` (returned in that precision)."""
    dt = np.float32 if precision == "fp32" else np.float64
    return np.linalg.cholesky(np.asarray(A, dtype=dt))


def preconditioner_gamma(A: np.ndarray, precision: str = "fp32") -> float:
    """gamma = ||I - A^{1/2} T_E A^{1/2}||_2 for the dense Cholesky preconditioner (Lemma 2).

    T_E is formed column by column by applying the lower-precision solves to the
    unit vectors (so it includes the rounding of the solves, as in eq. (wm)).
    """
    n = A.shape[0]
    Pc = Preconditioner(A, precision)
    T = Pc(np.eye(n))
    T = 0.5 * (T + T.T)
    lam, U = np.linalg.eigh(A)
    Ah = (U * np.sqrt(lam)) @ U.T
    M = np.eye(n) - Ah @ T @ Ah
    return float(np.linalg.norm(0.5 * (M + M.T), 2))
