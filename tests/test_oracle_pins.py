"""Pins for the CPU oracle: closed forms, brute force, invariants and planted mistakes.

These tests check the oracle against facts fixed by the mathematics and the
paper, not against itself:
  * Dirichlet Laplacian spectra in closed form (2D and 3D);
  * a dense matrix with a prescribed spectrum;
  * brute-force dense eigenpairs on small random SPD matrices;
  * Algorithm 2's ENSURE (A = QR, Q^T Q = I) and agreement with FP64 Householder R;
  * the Hetmaniuk-Lehoucq update keeps [X, P] orthonormal and contains span(X_old);
  * the residual test of eq. (stop);
  * Lemma 2's bound on gamma where its hypothesis holds, and Theorem 1's rate;
  * eigen-gradients against central finite differences and shift invariants.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import dense, grad, lobpcg as ol, mixed_qr, pinvit, precond

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def closed_form_2d(s, count):
    t = 4.0 * np.sin(np.arange(1, s + 1) * np.pi / (2 * (s + 1))) ** 2
    return np.sort((t[:, None] + t[None, :]).ravel())[:count]


def closed_form_3d(N, count):
    t = 4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    return np.sort((t[:, None, None] + t[None, :, None] + t[None, None, :]).ravel())[:count]


def test_golden_closed_forms_match_formula():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        g = json.load(f)
    np.testing.assert_allclose(closed_form_2d(32, 6), g["laplace2d_32"]["eigs"], rtol=1e-13)
    np.testing.assert_allclose(closed_form_3d(64, 33)[[0, 15, 16, 31, 32]], g["laplace3d_64"]["eigs"], rtol=1e-13)


def test_cfg1_closed_form():
    p = synth.cfg1()
    na = dense.norm2(p.A)
    assert abs(na - 8 * np.sin(32 * np.pi / 66) ** 2) < 1e-12
    r = ol.lobpcg(p.A, p.X0, p.k, p.tol, norm_a=na)
    assert r.converged
    ref = closed_form_2d(32, 4)
    assert np.max(np.abs(r.evals - ref) / ref) < 1e-12
    # invariants: orthonormal X and the residual gate
    assert np.max(np.abs(r.evecs.T @ r.evecs - np.eye(4))) < 1e-13
    res = ol.residual_norms(p.A, r.evecs, r.evals, na)
    assert np.all(res <= p.tol)


def test_laplace3d_closed_form_fp32_factor():
    p = synth.cfg2(N=12, constant=True, k=8, m=16)
    na = dense.norm2(p.A)
    r = ol.lobpcg(p.A, p.X0, p.k, p.tol, precond_precision="fp32", norm_a=na)
    ref = closed_form_3d(12, 8)
    assert r.converged
    assert np.max(np.abs(r.evals - ref) / ref) < 1e-11


def test_dense_prescribed_spectrum():
    A, lam = synth.dense_spd(256, seed=3)
    X0 = synth.random_block(256, 16, 7)
    r = ol.lobpcg(A, X0, 8, 1e-12, precond_precision="fp32", norm_a=1e6)
    assert r.converged
    assert np.max(np.abs(r.evals - lam[:8]) / lam[:8]) < 1e-9


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_random_sparse(seed):
    rng = np.random.default_rng(seed)
    n = 300
    B = sp.random(n, n, density=0.02, random_state=seed)
    A = (B @ B.T + sp.eye(n) * 0.5).tocsr()
    X0 = rng.standard_normal((n, 10))
    na = dense.norm2(A)
    r = ol.lobpcg(A, X0, 5, 1e-11, norm_a=na)
    lam, U = dense.smallest_eigenpairs(A, 5)
    assert r.converged
    assert np.max(np.abs(r.evals - lam) / lam) < 1e-10
    # sign-invariant eigenvector agreement (eigenvalues are simple here)
    gaps = np.diff(dense.all_eigenpairs(A)[0][:7])
    if gaps.min() > 1e-6:
        cosines = np.abs(np.sum(r.evecs * U, axis=0))
        assert np.all(cosines > 1 - 1e-9)


def test_degenerate_cluster_subspace():
    # cfg1 has lambda_2 = lambda_3 exactly: compare the invariant subspace, not vectors.
    p = synth.cfg1()
    r = ol.lobpcg(p.A, p.X0, 4, 1e-10, norm_a=dense.norm2(p.A))
    lam, U = dense.smallest_eigenpairs(p.A, 4)
    Xc, Uc = r.evecs[:, 1:3], U[:, 1:3]
    s = np.linalg.svd(Uc.T @ Xc, compute_uv=False)
    assert s.min() > 1 - 1e-12


def test_stop_paper_form_is_looser_than_bj():
    A = synth.laplace2d(20)
    X0 = synth.random_block(400, 8, 1)
    na = dense.norm2(A)
    r1 = ol.lobpcg(A, X0, 4, 1e-8, norm_a=na, stop="bj")
    r2 = ol.lobpcg(A, X0, 4, 1e-8, norm_a=na, stop="paper")
    assert r2.iters <= r1.iters
    res = ol.residual_norms(A, r2.evecs, r2.evals, na, mode="paper")
    assert np.all(res <= 1e-8)


@pytest.mark.parametrize("kappa", [1.0, 1e3, 1e6])
def test_mixed_qr_ensure(kappa):
    rng = np.random.default_rng(11)
    n, m = 2000, 24
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    W = (U * np.geomspace(1.0, 1.0 / kappa, m)) @ V.T
    Q, R = mixed_qr.mixed_qr(W)
    u = np.finfo(np.float64).eps / 2
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 10 * m * u
    assert np.linalg.norm(W - Q @ R) / np.linalg.norm(W) <= 10 * u * 10
    assert np.allclose(np.tril(R, -1), 0.0)
    # R equals the FP64 Householder R up to row signs
    _, Rh = mixed_qr.householder_qr(W)
    sgn = np.sign(np.diag(R)) * np.sign(np.diag(Rh))
    assert np.linalg.norm(R - sgn[:, None] * Rh) / np.linalg.norm(Rh) < 50 * kappa * u


def test_hl_update_invariants():
    A = synth.laplace2d(24)
    X0 = synth.random_block(576, 6, 3)
    m = 6
    seen = []

    def cb(it, X, P, theta, res):
        if P is not None:
            B = np.hstack([X, P])
            seen.append(np.max(np.abs(B.T @ B - np.eye(2 * m))))

    ol.lobpcg(A, X0, 3, 1e-10, norm_a=dense.norm2(A), callback=cb)
    assert seen and max(seen) < 1e-12

    # span(X_old) is contained in span([X_new, P_new]) after one update
    rng = np.random.default_rng(0)
    S, _ = np.linalg.qr(rng.standard_normal((576, 3 * m)))
    H = S.T @ (A @ S)
    D, C = np.linalg.eigh(0.5 * (H + H.T))
    X, P, _ = ol.hl_update(S, C, D, m)
    B = np.hstack([X, P])
    Xold = S[:, :m]
    assert np.linalg.norm(Xold - B @ (B.T @ Xold)) < 1e-12


def test_lemma2_bound_and_theorem1_rate():
    # Lemma 2 hypothesis eps_T = 4n(3n+1) kappa u_l < 1 holds for tiny n and small kappa.
    n = 8
    A, _ = synth.dense_spd(n, seed=5, lo=1.0, hi=4.0)
    ul = np.finfo(np.float32).eps / 2
    kappa = np.linalg.cond(A)
    eps_t = 4 * n * (3 * n + 1) * kappa * ul
    assert eps_t < 1
    gamma = precond.preconditioner_gamma(A, "fp32")
    assert gamma <= eps_t / (1 - eps_t)
    # Theorem 1: per-step contraction of PINVIT with a deliberately weak preconditioner.
    A2, lam = synth.dense_spd(60, seed=9, lo=1.0, hi=50.0)
    Tw = np.linalg.inv(A2 + 5.0 * np.eye(60))
    Ah = np.linalg.cholesky(A2)
    evals, U = np.linalg.eigh(A2)
    Ahalf = (U * np.sqrt(evals)) @ U.T
    g = np.linalg.norm(np.eye(60) - Ahalf @ Tw @ Ahalf, 2)
    assert g < 1
    q2 = pinvit.rate_bound(g, lam[0], lam[1])
    rhos = pinvit.pinvit_k1(A2, U[:, 0] + 0.05 * U[:, 1] + 0.01 * U[:, 5], lambda r: Tw @ r, 6)
    for a, b in zip(rhos[:-1], rhos[1:]):
        if lam[0] < a < lam[1] and b - lam[0] > 1e-13:
            assert pinvit.ratio(b, lam[0], lam[1]) <= q2 * pinvit.ratio(a, lam[0], lam[1]) * (1 + 1e-6)
    del Ah


def test_fp32_factor_gamma_small_on_diffusion():
    p = synth.cfg2(N=8)
    A = p.A.toarray()
    gamma = precond.preconditioner_gamma(A, "fp32")
    assert gamma < 1e-4


def test_gradient_oracle_fd_and_invariants():
    s = 7
    rng = np.random.default_rng(4)
    c = rng.uniform(0, 1, (4, 2)); w = rng.uniform(0.1, 0.2, 4); a = rng.uniform(0, 20, 4)
    L0 = synth.laplace_scaled((s, s)).toarray()
    phi = synth.bump_basis(synth.grid_points((s, s)), c, w)
    g = rng.standard_normal(s * s); g /= np.linalg.norm(g)
    k = 3

    def A_of(amp):
        return L0 + np.diag(phi @ amp)

    loss, gv, lam, U = grad.loss_and_grad_diag(A_of(a), k, g)
    # shift invariants: sum_j dlambda_i/dV_j = 1, sum_j dLvec/dV_j = 0
    assert abs(gv.sum() - k) < 1e-10
    ga = grad.grad_amplitudes(gv, phi)
    h = 1e-5
    fd = np.array([(grad.loss_value(A_of(a + h * e), k, g) - grad.loss_value(A_of(a - h * e), k, g)) / (2 * h)
                   for e in np.eye(4)])
    np.testing.assert_allclose(ga, fd, rtol=1e-6, atol=1e-9)


def test_table3_laplace_shape():
    # Table 3: 2D-Laplace has n = 25,000 and nnz = 114,990; a 5 x 5000 5-point grid gives both.
    p, q = 5, 5000
    nnz = 5 * p * q - 2 * (p + q)
    assert p * q == 25000 and nnz == 114990
    A = synth.paper2d().A
    assert A.shape == (25000, 25000) and A.nnz == 114990


def test_rect_laplace_closed_form():
    # the separable spectrum of the p x q grid against a dense symmetric eigensolver
    A = synth.laplace2d_rect(5, 60).toarray()
    np.testing.assert_allclose(np.linalg.eigvalsh(A), synth.laplace2d_rect_eigs(5, 60), rtol=0, atol=1e-12)
    assert np.allclose(A, A.T) and np.all(np.diag(A) == 4.0)


# ---------------------------------------------------------------------------
# Planted mistakes: each mutation of the oracle must be caught by a pin above.
# ---------------------------------------------------------------------------

def test_planted_mistake_hl_without_v_is_caught(monkeypatch):
    def bad_hl(S, C, D, m):
        return S @ C[:, :m], S @ C[:, m:2 * m], D[:m].copy()   # drops V: P no longer spans X_old's remainder
    monkeypatch.setattr(ol, "hl_update", bad_hl)
    A = synth.laplace2d(24)
    rng = np.random.default_rng(0)
    S, _ = np.linalg.qr(rng.standard_normal((576, 18)))
    H = S.T @ (A @ S)
    D, C = np.linalg.eigh(0.5 * (H + H.T))
    X, P, _ = ol.hl_update(S, C, D, 6)
    B = np.hstack([X, P])
    assert np.linalg.norm(S[:, :6] - B @ (B.T @ S[:, :6])) > 1e-3


def test_planted_mistake_residual_sign_is_caught():
    p = synth.cfg1()
    na = dense.norm2(p.A)
    r = ol.lobpcg(p.A, p.X0, p.k, p.tol, norm_a=na)
    R_bad = p.A @ r.evecs + r.evecs * r.evals      # wrong sign
    res_bad = np.linalg.norm(R_bad, axis=0) / na
    assert np.all(res_bad > p.tol)


def test_planted_mistake_qr_transpose_is_caught():
    rng = np.random.default_rng(2)
    W = rng.standard_normal((500, 12))
    Q, R = mixed_qr.mixed_qr(W)
    assert np.linalg.norm(W - Q @ R.T) / np.linalg.norm(W) > 1e-3


# ---------------------------------------------------------------------------
# Algorithm 1 (block PINVIT, mixed precision) and the sparse preconditioner of section 5.1.
# ---------------------------------------------------------------------------

def _cfg1_closed(count):
    return closed_form_2d(32, count)


def test_mixed_pinvit_reaches_closed_form_cfg1():
    # Algorithm 1 with the FP32 sparse factor of section 5.1 on the 32 x 32 Laplacian: the four
    # smallest eigenvalues in closed form (4 sin^2(i pi/66) + 4 sin^2(j pi/66)) to 1e-10.
    p = synth.cfg1()
    na = dense.norm2(p.A)
    T = precond.Preconditioner(p.A, "fp32")
    th, X, it = pinvit.mixed_pinvit(p.A, p.X0, p.k, p.tol, T, na, maxit=300)
    ref = _cfg1_closed(4)
    assert it < 300
    assert np.max(np.abs(th - ref) / ref) <= 1e-10
    res = ol.residual_norms(p.A, X, th, na)
    assert np.all(res <= p.tol)
    assert np.max(np.abs(X.T @ X - np.eye(p.k))) < 1e-12


def test_mixed_pinvit_theorem1_rate_with_measured_gamma():
    # Theorem 1 (k = 1): with gamma = ||I - A^{1/2} T A^{1/2}||_2 measured for the FP32 factor, every step
    # with rho in [lambda_1, lambda_2) contracts (rho - lambda_1)/(lambda_2 - rho) by at most
    # (gamma + (1 - gamma) lambda_1/lambda_2)^2.  The Rayleigh quotient of iteration j is the theta that
    # mixed_pinvit returns when stopped after j iterations (the iteration is deterministic).
    p = synth.cfg1()
    na = dense.norm2(p.A)
    T = precond.Preconditioner(p.A, "fp32")
    gamma = precond.preconditioner_gamma(p.A.toarray(), "fp32")
    assert 0 < gamma < 1e-4
    l1, l2 = _cfg1_closed(2)
    q2 = pinvit.rate_bound(gamma, l1, l2)
    x0 = p.X0[:, :1]
    rhos = [pinvit.mixed_pinvit(p.A, x0, 1, 1e-300, T, na, maxit=j)[0][0] for j in range(1, 12)]
    checked = 0
    for a, b in zip(rhos[:-1], rhos[1:]):
        ra, rb = pinvit.ratio(a, l1, l2), pinvit.ratio(b, l1, l2)
        if l1 <= a < l2 and ra > 1e-6:
            assert rb <= q2 * ra * (1 + 1e-6)
            checked += 1
    assert checked >= 4
    # the bound is sharp for an almost exact preconditioner: the last contractions approach it
    assert rb / ra > 0.95 * q2


def test_planted_mistake_pinvit_update_sign_is_caught():
    # X~ = X + W instead of X - W: the closed-form pin above fails
    p = synth.cfg1()
    na = dense.norm2(p.A)
    T = precond.Preconditioner(p.A, "fp32")
    th, _, it = pinvit.mixed_pinvit(p.A, p.X0, p.k, p.tol, lambda r: -T(r), na, maxit=100)
    ref = _cfg1_closed(4)
    assert it == 100 or np.max(np.abs(th - ref) / ref) > 1e-3


def _sparse_case(N):
    A = synth.cfg2(N=N).A
    lam = np.linalg.eigvalsh(A.toarray())
    R = np.random.default_rng(3).standard_normal((A.shape[0], 8))
    return A, lam[-1], lam[-1] / lam[0], R


@pytest.mark.parametrize("N", [12, 16])
def test_sparse_preconditioner_solve_accuracy(N):
    # The sparse branch (SuperLU, no pivoting, minimum-degree order) against the mathematics of a
    # backward-stable solve: ||A W - R||_F <= 10 u ||A||_2 ||W||_F, and against a second, independent
    # library route (dense LAPACK Cholesky in FP64): every column within kappa u of A^{-1} R, for the
    # FP64 factor with u = u64 and the FP32 factor (lower(R), FP32 solves, working(W)) with u = u32.
    import scipy.linalg as sla
    A, na, kappa, R = _sparse_case(N)
    Wex = sla.cho_solve(sla.cho_factor(A.toarray()), R)
    for prec, u in (("fp64", np.finfo(np.float64).eps / 2), ("fp32", np.finfo(np.float32).eps / 2)):
        W = precond.Preconditioner(A, prec)(R)
        assert W.dtype == np.float64
        assert np.linalg.norm(A @ W - R) <= 10 * u * na * np.linalg.norm(W), prec
        col = np.linalg.norm(W - Wex, axis=0) / np.linalg.norm(Wex, axis=0)
        assert col.max() <= kappa * u, prec
        if prec == "fp32":
            # and not better than FP32 allows: the factor really is held in single precision
            assert col.max() >= 1e-3 * kappa * u


def test_planted_mistake_preconditioner_one_triangular_solve_is_caught():
    # applying only the lower triangular solve (the SuperLU L factor) is far outside the pin
    import scipy.sparse.linalg as spla
    A, na, kappa, R = _sparse_case(12)
    Pc = precond.Preconditioner(A, "fp64")
    lu = Pc.lu
    Wbad = np.zeros_like(R)
    Wbad[lu.perm_c] = spla.spsolve_triangular(lu.L.tocsr(), R[lu.perm_r], lower=True)
    u = np.finfo(np.float64).eps / 2
    assert np.linalg.norm(A @ Wbad - R) > 1e6 * 10 * u * na * np.linalg.norm(Wbad)


def test_planted_mistake_preconditioner_half_precision_is_caught():
    # lower(R) rounded to half precision instead of single: the FP32 branch's kappa u32 pin fails
    import scipy.linalg as sla
    A, na, kappa, R = _sparse_case(12)
    Wex = sla.cho_solve(sla.cho_factor(A.toarray()), R)
    Pc = precond.Preconditioner(A, "fp32")
    Wbad = Pc(R.astype(np.float16).astype(np.float64))
    col = np.linalg.norm(Wbad - Wex, axis=0) / np.linalg.norm(Wex, axis=0)
    assert col.max() > kappa * np.finfo(np.float32).eps / 2


# ---------------------------------------------------------------------------
# Algorithm 3 line 1: the single-precision LOBPCG that computes the start block (MPLOBPCG-schol with
# the first-stage tolerance 5e-6 of section 5.1).
# ---------------------------------------------------------------------------

def _stage1_case():
    p = synth.cfg1()
    na = dense.norm2(p.A)
    T = precond.Preconditioner(p.A, "fp32")
    return p, na, T


def test_stage1_single_precision_meets_its_tolerance_and_closed_form():
    # The first stage runs in float32 end to end and stops once eq. (stop) holds with 5e-6; its Ritz values
    # then lie within the Kato-Temple bound ||r||^2 / gap plus the float32 rounding of A X (about
    # u32 ||A|| absolute) of the closed form 4 sin^2(i pi/66) + 4 sin^2(j pi/66).
    p, na, T = _stage1_case()
    s1 = ol.lobpcg(p.A, p.X0, p.k, 5e-6, precond=T, norm_a=na, stop="paper", dtype=np.float32)
    assert s1.converged and s1.block.dtype == np.float32 and s1.block.shape == (p.n, p.m)
    X = s1.block.astype(np.float64)
    theta = np.diag(X.T @ (p.A @ X)) / np.sum(X * X, axis=0)
    res = ol.residual_norms(p.A, X[:, :p.k], theta[:p.k], na, mode="paper")
    assert np.all(res <= 2 * 5e-6)                       # recomputed in FP64: float32 rounding stays well inside
    ref = _cfg1_closed(p.k)
    u32 = np.finfo(np.float32).eps / 2
    gap = _cfg1_closed(p.m + 1)[p.m] - ref               # distance to the spectrum outside the block
    bound = (5e-6 * (na + ref)) ** 2 / gap + 4 * u32 * na
    assert np.all(np.abs(theta[:p.k] - ref) <= bound)
    assert np.max(np.abs(theta[:p.k] - ref) / ref) > 1e-12   # single precision: not FP64-accurate


def test_mixed_lobpcg_two_stages_reach_closed_form():
    # Line 1 then lines 2-17: the FP64 loop from working(X) reaches the closed form to 1e-10 and the residual
    # gate, and needs fewer working-precision iterations than the loop started from X0 itself.
    p, na, T = _stage1_case()
    r = ol.mixed_lobpcg(p.A, p.X0, p.k, p.tol, 5e-6, precond=T, norm_a=na, stop="paper")
    assert r.converged and r.stage1_converged
    ref = _cfg1_closed(p.k)
    assert np.max(np.abs(r.evals - ref) / ref) <= 1e-10
    assert np.all(ol.residual_norms(p.A, r.evecs, r.evals, na, mode="paper") <= p.tol)
    single = ol.lobpcg(p.A, p.X0, p.k, p.tol, precond=T, norm_a=na, stop="paper")
    assert r.iters < single.iters


def test_planted_mistake_stage1_result_dropped_is_caught(monkeypatch):
    # A first stage whose result is lost (the second stage restarts from X0) takes as many
    # working-precision iterations as no first stage at all, which the two-stage pin rejects.
    p, na, T = _stage1_case()
    single = ol.lobpcg(p.A, p.X0, p.k, p.tol, precond=T, norm_a=na, stop="paper")
    real = ol.lobpcg

    def lossy(A, X0, k, tol, **kw):
        r = real(A, X0, k, tol, **kw)
        if kw.get("dtype") == np.float32:
            r.block = np.asarray(X0, dtype=np.float32)
        return r
    monkeypatch.setattr(ol, "lobpcg", lossy)
    r = ol.mixed_lobpcg(p.A, p.X0, p.k, p.tol, 5e-6, precond=T, norm_a=na, stop="paper")
    assert not r.iters < single.iters


def test_planted_mistake_stage1_in_double_is_caught():
    # Running the first stage in float64 gives Ritz values accurate far beyond single precision: the
    # last assertion of the first pin rejects it.
    p, na, T = _stage1_case()
    s1 = ol.lobpcg(p.A, p.X0, p.k, 1e-11, precond=T, norm_a=na, stop="paper", dtype=np.float64)
    ref = _cfg1_closed(p.k)
    assert not np.max(np.abs(s1.evals - ref) / ref) > 1e-12


# ---------------------------------------------------------------------------
# Complex Hermitian matrices (section 1): the brute-force path of the oracle on Hermitian inputs, and the
# real symmetric embedding the GPU path solves.
# ---------------------------------------------------------------------------

def test_gauge_laplacian_closed_form():
    # D L D^H with a unitary diagonal D has the spectrum of L: 4 sin^2(i pi/(2(p+1))) + 4 sin^2(j pi/(2(q+1)))
    A = synth.gauge_laplace2d(9, 11)
    assert np.iscomplexobj(A.data) and np.abs(A.imag).max() > 0.1
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.conj().T, atol=0, rtol=0)
    lam, U = dense.smallest_eigenpairs(A, 12)
    np.testing.assert_allclose(lam, synth.laplace2d_rect_eigs(9, 11)[:12], rtol=1e-13)
    R = Ad @ U - U * lam
    assert np.linalg.norm(R) < 1e-12 and np.allclose(U.conj().T @ U, np.eye(12), atol=1e-13)


def test_dense_hpd_prescribed_spectrum():
    A, lam = synth.dense_hpd(120)
    got, _ = dense.smallest_eigenpairs(A, 10)
    np.testing.assert_allclose(got, lam[:10], rtol=1e-12)


def test_real_embedding_doubles_each_eigenvalue():
    # M = [[B, -C], [C, B]] for A = B + iC: every eigenvalue of A twice, and [u; v] for x = u + iv
    A = synth.gauge_laplace2d(6, 7).toarray()
    B, C = A.real, A.imag
    M = np.block([[B, -C], [C, B]])
    assert np.allclose(M, M.T)
    lamA, UA = np.linalg.eigh(A)
    lamM = np.linalg.eigvalsh(M)
    np.testing.assert_allclose(lamM[0::2], lamA, rtol=1e-12)
    np.testing.assert_allclose(lamM[1::2], lamA, rtol=1e-12)
    x = UA[:, 0]
    z = np.concatenate([x.real, x.imag])
    assert np.linalg.norm(M @ z - lamA[0] * z) < 1e-12


def test_planted_mistake_embedding_sign_is_caught():
    # the wrong sign on the off-diagonal blocks ([[B, C], [C, B]]) is not even symmetric
    A = synth.gauge_laplace2d(6, 7).toarray()
    B, C = A.real, A.imag
    M_bad = np.block([[B, C], [C, B]])
    assert not np.allclose(M_bad, M_bad.T)
