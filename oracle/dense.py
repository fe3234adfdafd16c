"""Brute-force eigenpairs: the plain definition of what the method computes.

Section 1 poses the problem: the k smallest eigenvalues of a Hermitian positive
definite A and eigenvectors with A X = X Lambda.  For n small enough for a dense
symmetric eigensolver this is computed directly (LAPACK syevd via numpy).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _dense_hermitian(A):
    """A as a dense array, made exactly Hermitian ((A + A^H) / 2; the transpose for real A)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    Ad = Ad.astype(np.complex128 if np.iscomplexobj(Ad) else np.float64)
    return 0.5 * (Ad + Ad.conj().T)


def smallest_eigenpairs(A, k: int):
    """Return (lam[:k] ascending, U[:, :k]) of the symmetric or Hermitian matrix A (dense or sparse)."""
    lam, U = np.linalg.eigh(_dense_hermitian(A))
    return lam[:k].copy(), U[:, :k].copy()


def all_eigenpairs(A):
    return np.linalg.eigh(_dense_hermitian(A))


def norm2(A) -> float:
    """||A||_2 of a symmetric positive definite A (largest eigenvalue), by Lanczos for sparse A."""
    if sp.issparse(A):
        if A.shape[0] <= 2000:
            return float(np.linalg.eigvalsh(A.toarray())[-1])
        from scipy.sparse.linalg import eigsh
        v0 = np.random.default_rng(0).standard_normal(A.shape[0])
        return float(eigsh(A, k=1, which="LA", v0=v0, tol=1e-12, return_eigenvectors=False)[0])
    return float(np.linalg.eigvalsh(0.5 * (A + A.T))[-1])
