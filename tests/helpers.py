"""Shared checks for the GPU parity tests (host-side definitions, no oracle arithmetic)."""
import numpy as np
import scipy.sparse as sp


def residuals(A, X, lam, norm_a):
    """||A x_j - lam_j x_j|| / (||A||_2 ||x_j||) computed in FP64 on the host."""
    R = A @ X - X * lam
    return np.linalg.norm(R, axis=0) / (norm_a * np.linalg.norm(X, axis=0))


def clusters(lam, rel=1e-8):
    """Group indices of (sorted) eigenvalues whose relative gap is below rel."""
    groups, cur = [], [0]
    for i in range(1, len(lam)):
        if abs(lam[i] - lam[i - 1]) <= rel * max(abs(lam[i]), 1e-300):
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups


def subspace_cos(U, X):
    """Smallest cosine of the principal angles between span(U) and span(X) (both orthonormal)."""
    return float(np.linalg.svd(U.T @ X, compute_uv=False).min())


def permuted(A, perm):
    if sp.issparse(A):
        return sp.csr_matrix(A)[perm][:, perm]
    return A[np.ix_(perm, perm)]
