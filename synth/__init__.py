"""Seeded synthetic eigenproblems shaped like the paper's workloads.

This module builds input matrices and start blocks only.  It holds none of the
eigensolver's arithmetic, so both the CPU oracle and the GPU path can use it.
Every random draw goes through ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed order, and arrays are created once on the host; the same arrays are fed
to both sides.

Grid numbering (0-based):
  2D  p = i*s + j                       (grid hint (s, s, 1))
  3D  p = (i*N + j)*N + l               (grid hint (N, N, N))

Workloads (the paper tests sparse SPD matrices with 5-7 nonzeros per row and
dense SPD matrices with n up to 8192, m = 8n/1024; section 5.3, section 5.4):
  laplace2d        : 5-point Dirichlet Laplacian, unscaled (4 / -1)
  diffusion3d      : 7-point cell-centred variable-coefficient diffusion,
                     harmonic-mean face coefficients, Dirichlet faces add a_p
  dense_spd        : Q diag(lambda) Q^T, Q from QR of a Gaussian matrix,
                     lambda geometric in [1, 1e6]
  schrodinger2d/3d : h^-2 * Laplacian + diag(V), V a sum of Gaussian bumps
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Problem:
    name: str
    A: object                 # scipy.sparse.csr_matrix (float64) or np.ndarray (dense, C-order)
    X0: np.ndarray            # n x m float64, C-order
    k: int
    m: int
    tol: float
    factor_precision: str     # "fp32" or "fp64"
    grid: tuple = (0, 0, 0)   # geometry hint for nested dissection (0 = none)
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def dense(self) -> bool:
        return isinstance(self.A, np.ndarray)


def _csr_sorted(A) -> sp.csr_matrix:
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def laplace2d(s: int) -> sp.csr_matrix:
    """5-point Dirichlet Laplacian on an s x s interior grid, diagonal 4, off-diagonal -1."""
    n = s * s
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(s, s)
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(np.full(n, 4.0))
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        i0, i1 = max(0, -di), s - max(0, di)
        j0, j1 = max(0, -dj), s - max(0, dj)
        a = idx[i0:i1, j0:j1].ravel()
        b = idx[i0 + di:i1 + di, j0 + dj:j1 + dj].ravel()
        rows.append(a); cols.append(b); vals.append(np.full(a.size, -1.0))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return _csr_sorted(A)


def laplace2d_rect(p: int, q: int) -> sp.csr_matrix:
    """5-point Dirichlet Laplacian on a p x q interior grid (index i q + j), diagonal 4, off-diagonal -1."""
    n = p * q
    idx = np.arange(n).reshape(p, q)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [np.full(n, 4.0)]
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        i0, i1 = max(0, -di), p - max(0, di)
        j0, j1 = max(0, -dj), q - max(0, dj)
        a = idx[i0:i1, j0:j1].ravel()
        b = idx[i0 + di:i1 + di, j0 + dj:j1 + dj].ravel()
        rows.append(a); cols.append(b); vals.append(np.full(a.size, -1.0))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return _csr_sorted(A)


def laplace2d_rect_eigs(p: int, q: int) -> np.ndarray:
    """All eigenvalues of laplace2d_rect(p, q), ascending: 4 - 2 cos(a pi/(p+1)) - 2 cos(b pi/(q+1))."""
    a = np.arange(1, p + 1)[:, None]
    b = np.arange(1, q + 1)[None, :]
    lam = 4.0 - 2.0 * np.cos(a * np.pi / (p + 1)) - 2.0 * np.cos(b * np.pi / (q + 1))
    return np.sort(lam.ravel())


def diffusion3d(a: np.ndarray) -> sp.csr_matrix:
    """Cell-centred 7-point diffusion on an N^3 grid with cell coefficients a (N,N,N).

    Interior face between cells p, q has coefficient 2 a_p a_q / (a_p + a_q);
    a Dirichlet boundary face of cell p adds a_p to its diagonal.  With a == 1
    this is the 7-point Laplacian (diagonal 6, off-diagonal -1).
    """
    N = a.shape[0]
    assert a.shape == (N, N, N)
    n = N ** 3
    idx = np.arange(n).reshape(N, N, N)
    diag = np.zeros((N, N, N))
    rows, cols, vals = [], [], []
    for ax in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, N - 1)
        sl_hi[ax] = slice(1, N)
        ap = a[tuple(sl_lo)]
        aq = a[tuple(sl_hi)]
        f = 2.0 * ap * aq / (ap + aq)
        p = idx[tuple(sl_lo)].ravel()
        q = idx[tuple(sl_hi)].ravel()
        rows += [p, q]; cols += [q, p]; vals += [-f.ravel(), -f.ravel()]
        diag[tuple(sl_lo)] += f
        diag[tuple(sl_hi)] += f
        # Dirichlet faces on both ends of this axis
        b0 = [slice(None)] * 3; b0[ax] = 0
        b1 = [slice(None)] * 3; b1[ax] = N - 1
        diag[tuple(b0)] += a[tuple(b0)]
        diag[tuple(b1)] += a[tuple(b1)]
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return _csr_sorted(A)


def gaussian_bumps(points: np.ndarray, centers: np.ndarray, widths: np.ndarray, amps: np.ndarray) -> np.ndarray:
    """V(x) = sum_g amps[g] * exp(-|x - c_g|^2 / (2 w_g^2)) at each point (rows of `points`)."""
    return bump_basis(points, centers, widths) @ amps


def bump_basis(points: np.ndarray, centers: np.ndarray, widths: np.ndarray) -> np.ndarray:
    """phi[p, g] = exp(-|x_p - c_g|^2 / (2 w_g^2)), so that V = phi @ amps."""
    d2 = ((points[:, None, :] - centers[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2.0 * widths[None, :] ** 2))


def grid_points(dims) -> np.ndarray:
    """Interior nodes ((i+1)h, ...) of the unit square/cube, h = 1/(s+1), in grid numbering."""
    axes = [(np.arange(s) + 1.0) / (s + 1.0) for s in dims]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in mesh], axis=1)


def laplace_scaled(dims) -> sp.csr_matrix:
    """h^-2 * (Dirichlet Laplacian stencil) on a 2D or 3D interior grid with equal sides."""
    s = dims[0]
    h = 1.0 / (s + 1.0)
    if len(dims) == 2:
        L = laplace2d(s)
    else:
        L = diffusion3d(np.ones((s, s, s)))
    return _csr_sorted(L * (1.0 / (h * h)))


def schrodinger(dims, centers, widths, amps) -> sp.csr_matrix:
    """-Laplacian + diag(V) on the unit square/cube interior grid (h^-2 scaled stencil)."""
    L = laplace_scaled(dims)
    V = gaussian_bumps(grid_points(dims), centers, widths, amps)
    return _csr_sorted(L + sp.diags(V))


def dense_spd(n: int, seed: int = 3, lo: float = 1.0, hi: float = 1e6):
    """A = Q diag(lambda) Q^T with Q from QR of a seeded Gaussian and lambda = geomspace(lo, hi, n)."""
    G = np.random.default_rng(seed).standard_normal((n, n))
    Q, _ = np.linalg.qr(G)
    lam = np.geomspace(lo, hi, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return np.ascontiguousarray(A), lam


# ---------------------------------------------------------------------------
# The five workloads.  `scale` shrinks a workload (for tests) while keeping its recipe.
# ---------------------------------------------------------------------------

def cfg1() -> Problem:
    """2D 5-point Dirichlet Laplacian on 32x32 (n=1024), k=4, m=8, FP64 factor, tol 1e-10."""
    A = laplace2d(32)
    X0 = np.random.default_rng(101).standard_normal((1024, 8))
    return Problem("laplace2d_32", A, X0, 4, 8, 1e-10, "fp64", (32, 32, 1))


def cfg2(N: int = 64, coeff_seed: int = 2, x0_seed: int = 102, k: int = 16, m: int = 32,
         constant: bool = False, factor_precision: str = "fp32") -> Problem:
    """3D 7-point variable-coefficient diffusion, a = exp(N(0,1)) per cell (n = N^3), k=16, m=32."""
    if constant:
        a = np.ones((N, N, N))
    else:
        a = np.exp(np.random.default_rng(coeff_seed).standard_normal((N, N, N)))
    A = diffusion3d(a)
    X0 = np.random.default_rng(x0_seed).standard_normal((N ** 3, m))
    return Problem(f"diffusion3d_{N}", A, X0, k, m, 1e-10, factor_precision, (N, N, N))


def cfg3(n: int = 8192, k: int = 32, m: int = 64, factor_precision: str = "fp32") -> Problem:
    """Dense SPD n=8192 with a geometric spectrum in [1, 1e6], k=32, m=64."""
    A, lam = dense_spd(n, seed=3)
    X0 = np.random.default_rng(103).standard_normal((n, m))
    return Problem(f"dense_spd_{n}", A, X0, k, m, 1e-10, factor_precision, (0, 0, 0),
                   extra={"spectrum": lam})


def cfg4_params(count: int = 256, seed: int = 4):
    """Per-instance (side, centers, widths, amplitudes), drawn in a fixed order from rng(seed)."""
    r = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = int(r.integers(48, 129))
        c = r.uniform(0, 1, (8, 2))
        w = r.uniform(0.05, 0.2, 8)
        amp = r.uniform(0, 50, 8)
        out.append((s, c, w, amp))
    return out


def cfg4(count: int = 256, k: int = 8, m: int = 16, side_override=None) -> list:
    """256 2D Schrodinger operators, side U{48..128}, 8 Gaussian bumps each, k=8, m=16, FP32 factors."""
    probs = []
    for b, (s, c, w, amp) in enumerate(cfg4_params(count)):
        if side_override is not None:
            s = side_override(s)
        A = schrodinger((s, s), c, w, amp)
        X0 = np.random.default_rng(10_000 + b).standard_normal((s * s, m))
        probs.append(Problem(f"schrodinger2d_{b}_{s}", A, X0, k, m, 1e-10, "fp32", (s, s, 1),
                             extra={"centers": c, "widths": w, "amps": amp}))
    return probs


def cfg5(N: int = 48, k: int = 8, m: int = 16) -> Problem:
    """3D Schrodinger, 32 learnable Gaussian bumps with amplitudes U(0,20), k=8, m=16."""
    r = np.random.default_rng(5)
    c = r.uniform(0, 1, (32, 3))
    w = r.uniform(0.05, 0.2, 32)
    a0 = r.uniform(0, 20, 32)
    n = N ** 3
    g = np.random.default_rng(105).standard_normal(n)
    g /= np.linalg.norm(g)
    X0 = np.random.default_rng(205).standard_normal((n, m))
    A = schrodinger((N, N, N), c, w, a0)
    phi = bump_basis(grid_points((N, N, N)), c, w)
    L0 = laplace_scaled((N, N, N))
    return Problem(f"schrodinger3d_{N}", A, X0, k, m, 1e-10, "fp32", (N, N, N),
                   extra={"centers": c, "widths": w, "amps": a0, "g": g, "phi": phi, "L0": L0})


def paper2d(x0_seed: int = 106) -> Problem:
    """The 2D-Laplace matrix of the paper's sparse tests, reconstructed from its size: n = 25,000 and
    nnz = 114,990 are those of a 5 x 5000 Dirichlet 5-point grid (5pq - 2(p + q) with pq = 25,000);
    k = 30, m = 45, tol = 1e-12 under the paper's stopping rule.  The start block is a seeded N(0,1)
    block (the paper's is not given)."""
    A = laplace2d_rect(5, 5000)
    X0 = np.random.default_rng(x0_seed).standard_normal((25000, 45))
    return Problem("laplace2d_5x5000", A, X0, 30, 45, 1e-12, "fp32", (0, 0, 0),
                   extra={"eigs": laplace2d_rect_eigs(5, 5000)})


def gauge_laplace2d(p: int, q: int, seed: int = 7) -> sp.csr_matrix:
    """A complex Hermitian positive definite matrix with a known spectrum: D L D^H for the p x q Dirichlet
    5-point Laplacian L and D = diag(exp(i phi)) with phases phi ~ U(0, 2 pi) per node (seeded).  Every
    coupling L_jk = -1 becomes -exp(i (phi_j - phi_k)); D is unitary, so the eigenvalues are those of L
    (laplace2d_rect_eigs) and the eigenvectors D u."""
    L = laplace2d_rect(p, q).tocoo()
    phi = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, p * q)
    vals = L.data * np.exp(1j * (phi[L.row] - phi[L.col]))
    A = sp.csr_matrix(sp.coo_matrix((vals, (L.row, L.col)), shape=L.shape), dtype=np.complex128)
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def dense_hpd(n: int, seed: int = 13, lo: float = 1.0, hi: float = 1e3):
    """A = Q diag(lambda) Q^H with Q from QR of a seeded complex Gaussian, lambda = geomspace(lo, hi, n)."""
    r = np.random.default_rng(seed)
    G = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    Q, _ = np.linalg.qr(G)
    lam = np.geomspace(lo, hi, n)
    A = (Q * lam) @ Q.conj().T
    return 0.5 * (A + A.conj().T), lam


def complex_block(n: int, m: int, seed: int) -> np.ndarray:
    r = np.random.default_rng(seed)
    return r.standard_normal((n, m)) + 1j * r.standard_normal((n, m))


def random_block(n: int, m: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((n, m))
