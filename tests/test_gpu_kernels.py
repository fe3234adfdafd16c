"""Per-step GPU parity through the C-ABI: SpMM, Gram, small eigensolver, Algorithm 2, preconditioner."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import mixed_qr as oqr
from oracle import precond as opc
from tests.helpers import permuted

pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2
U32 = np.finfo(np.float32).eps / 2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("shape", [(1000, 8, 8), (3001, 24, 40), (70000, 96, 96), (17, 3, 5), (5000, 192, 192)])
def test_gram(torch_cuda, shape):
    import paper_2302_12528_amd as pk
    n, c1, c2 = shape
    print(f"gram n={n} c1={c1} c2={c2}", flush=True)
    rng = np.random.default_rng(n + c1)
    X = rng.standard_normal((n, c1))
    Y = rng.standard_normal((n, c2))
    G = _np(pk.gram(X, Y))
    ref = X.T @ Y
    bound = n * U64 * 1.01 * (np.abs(X).T @ np.abs(Y)) + 1e-300
    assert np.all(np.abs(G - ref) <= 4 * bound)


def test_gram_deterministic(torch_cuda):
    import paper_2302_12528_amd as pk
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50000, 48))
    G1 = _np(pk.gram(X, X))
    G2 = _np(pk.gram(X, X))
    assert np.array_equal(G1, G2)


@pytest.mark.parametrize("c", [1, 2, 3, 8, 16, 17, 24, 33, 47, 48, 95, 96, 128, 192])
def test_syev_small(torch_cuda, c):
    import paper_2302_12528_amd as pk
    print(f"syev c={c}", flush=True)
    rng = np.random.default_rng(c)
    Q, _ = np.linalg.qr(rng.standard_normal((c, c)))
    lam = np.sort(rng.standard_normal(c))
    if c >= 3:
        lam[1] = lam[2]                   # an exact double eigenvalue
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    w, V = pk.syev_small(H)
    w, V = _np(w), _np(V)
    ref = np.linalg.eigvalsh(H)
    hn = np.linalg.norm(H, 2)
    assert np.max(np.abs(w - ref)) <= 50 * c * U64 * hn
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(V.T @ V - np.eye(c))) <= 100 * c * U64
    assert np.max(np.abs(H @ V - V * w)) <= 100 * c * U64 * hn


@pytest.mark.parametrize("c", [24, 48, 96])
def test_syev_clusters(torch_cuda, c):
    # a six-fold eigenvalue, a pair 1e-12 apart and a zero eigenvalue: the bisection brackets reach
    # ulp level and inverse iteration has to orthogonalise inside the clusters
    import paper_2302_12528_amd as pk
    print(f"syev clusters c={c}", flush=True)
    rng = np.random.default_rng(100 + c)
    Q, _ = np.linalg.qr(rng.standard_normal((c, c)))
    lam = np.sort(rng.uniform(-2.0, 3.0, c))
    lam[2:8] = 0.75
    lam[10] = lam[11] + 1e-12
    lam[12] = 0.0
    lam = np.sort(lam)
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    w, V = pk.syev_small(H)
    w, V = _np(w), _np(V)
    hn = np.linalg.norm(H, 2)
    assert np.max(np.abs(w - np.linalg.eigvalsh(H))) <= 50 * c * U64 * hn
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(V.T @ V - np.eye(c))) <= 100 * c * U64
    assert np.max(np.abs(H @ V - V * w)) <= 100 * c * U64 * hn


@pytest.mark.parametrize("kappa", [1.0, 1e3, 1e6])
@pytest.mark.parametrize("lower", [True, False])
@pytest.mark.parametrize("nc", [(20000, 32), (5000, 16), (1000, 64), (64, 64)])
def test_mixed_qr(torch_cuda, kappa, lower, nc):
    import paper_2302_12528_amd as pk
    n, c = nc
    print(f"mixed_qr n={n} c={c} kappa={kappa} lower={lower}", flush=True)
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(rng.standard_normal((n, c)))
    V, _ = np.linalg.qr(rng.standard_normal((c, c)))
    W = (U * np.geomspace(1.0, 1.0 / kappa, c)) @ V.T
    Q, R = pk.mixed_qr(W, lower=lower)
    Q, R = _np(Q), _np(R)
    assert np.linalg.norm(Q.T @ Q - np.eye(c)) <= 10 * c * U64
    assert np.linalg.norm(W - Q @ R) / np.linalg.norm(W) <= 100 * U64
    assert np.allclose(np.tril(R, -1), 0.0)
    # same R as the oracle's Algorithm 2 / FP64 Householder, up to row signs
    _, Rh = oqr.householder_qr(W)
    sgn = np.sign(np.diag(R)) * np.sign(np.diag(Rh))
    assert np.linalg.norm(R - sgn[:, None] * Rh) / np.linalg.norm(Rh) < 100 * kappa * U64


def _solver(A, k, m, prec, grid=(0, 0, 0), **kw):
    import paper_2302_12528_amd as pk
    return pk.Solver(A, k, m, 1e-10, factor_precision=prec, grid=grid, **kw)


@pytest.mark.parametrize("case", ["laplace2d_32", "diffusion3d_12", "dense_300"])
def test_apply_a(torch_cuda, case):
    print(f"apply_a {case}", flush=True)
    if case == "laplace2d_32":
        A, grid = synth.laplace2d(32), (32, 32, 1)
    elif case == "diffusion3d_12":
        A, grid = synth.cfg2(N=12).A, (12, 12, 12)
    else:
        A, grid = synth.dense_spd(300)[0], (0, 0, 0)
    s = _solver(A, 2, 4, "fp64", grid)
    perm = s.permutation()
    Ap = permuted(A, perm)
    rng = np.random.default_rng(1)
    for c in (1, 5, 8, 16, 33, 64, 96):
        X = rng.standard_normal((A.shape[0], c))
        Y = _np(s.apply_a(X))
        ref = Ap @ X
        absA = abs(Ap) if sp.issparse(Ap) else np.abs(Ap)
        bound = (A.shape[0] if not sp.issparse(A) else 8) * U64 * 1.01 * (absA @ np.abs(X))
        assert np.all(np.abs(Y - ref) <= 4 * bound + 1e-300), c
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["laplace2d_32", "diffusion3d_16", "diffusion3d_16_graph", "dense_500",
                                  "laplace2d_33x31"])
def test_apply_precond(torch_cuda, prec, case):
    print(f"precond {case} {prec}", flush=True)
    if case == "laplace2d_32":
        A, grid, m = synth.laplace2d(32), (32, 32, 1), 8
    elif case == "diffusion3d_16":
        A, grid, m = synth.cfg2(N=16).A, (16, 16, 16), 32
    elif case == "diffusion3d_16_graph":
        A, grid, m = synth.cfg2(N=16).A, (0, 0, 0), 16
    elif case == "laplace2d_33x31":
        L1 = synth.laplace2d(33)
        A, grid, m = L1, (0, 0, 0), 13
    else:
        A, grid, m = synth.dense_spd(500, seed=4, hi=1e3)[0], (0, 0, 0), 24
    s = _solver(A, 1, m, prec, grid)
    perm = s.permutation()
    Ap = permuted(A, perm)
    rng = np.random.default_rng(2)
    R = rng.standard_normal((A.shape[0], m))
    W = _np(s.apply_precond(R))
    Wref = opc.Preconditioner(Ap, "fp64")(R)
    err = np.linalg.norm(W - Wref) / np.linalg.norm(Wref)
    tol = 1e-9 if prec == "fp64" else 5e-4
    assert err < tol, err
    s.close()
