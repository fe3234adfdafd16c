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


@pytest.mark.parametrize("c,nev", [(72, 16), (96, 32), (100, 8), (128, 40), (160, 48), (192, 32), (192, 64),
                                   (192, 65)])
@pytest.mark.parametrize("clustered", [False, True])
def test_syev_partial(torch_cuda, c, nev, clustered):
    # the nev smallest pairs, as the Rayleigh-Ritz step asks for them (c = 3m, nev = m); for c > 96 and
    # nev <= 64 this is the inverse-iteration kernel with the factors in global memory and the separate
    # back-transformation, nev = 65 takes the one-workgroup form
    import paper_2302_12528_amd as pk
    print(f"syev partial c={c} nev={nev} clustered={clustered}", flush=True)
    rng = np.random.default_rng(200 + c + nev)
    Q, _ = np.linalg.qr(rng.standard_normal((c, c)))
    lam = np.sort(rng.uniform(0.0, 10.0, c))
    if clustered:
        # the wanted eigenvalues inside one cluster (gaps below 1e-3 ||T||), with a triple eigenvalue
        lam[:nev] = np.sort(rng.uniform(0.001, 0.005, nev))
        lam[3:6] = lam[3]
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    w, V = pk.syev_small(H, nev)
    w, V = _np(w), _np(V)
    assert w.shape == (nev,) and V.shape == (c, nev)
    hn = np.linalg.norm(H, 2)
    assert np.max(np.abs(w - np.linalg.eigvalsh(H)[:nev])) <= 50 * c * U64 * hn
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(V.T @ V - np.eye(nev))) <= 100 * c * U64
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


@pytest.mark.parametrize("lower", [True, False])
@pytest.mark.parametrize("ncl", [(3001, 32, 33), (2000, 16, 21), (777, 8, 96), (4100, 32, 96)])
def test_mixed_qr_strided(torch_cuda, lower, ncl):
    """Algorithm 2 on a block inside a wider buffer (odd leading dimensions take the element-wise
    paths of the row solves, a ragged last tile their range limits)."""
    import paper_2302_12528_amd as pk
    n, c, ld = ncl
    print(f"mixed_qr_strided n={n} c={c} ld={ld} lower={lower}", flush=True)
    rng = np.random.default_rng(n + ld)
    W = rng.standard_normal((n, c)) * np.geomspace(1.0, 1e-3, c)
    Q, R = pk.mixed_qr(W, lower=lower, ld=ld)
    Q, R = _np(Q), _np(R)
    assert np.linalg.norm(Q.T @ Q - np.eye(c)) <= 10 * c * U64
    assert np.linalg.norm(W - Q @ R) / np.linalg.norm(W) <= 100 * U64
    _, Rh = oqr.householder_qr(W)
    sgn = np.sign(np.diag(R)) * np.sign(np.diag(Rh))
    assert np.linalg.norm(R - sgn[:, None] * Rh) / np.linalg.norm(Rh) < 100 * 1e3 * U64


def _solver(A, k, m, prec, grid=(0, 0, 0), **kw):
    import paper_2302_12528_amd as pk
    return pk.Solver(A, k, m, 1e-10, factor_precision=prec, grid=grid, **kw)


@pytest.mark.parametrize("case", ["laplace2d_32", "diffusion3d_12", "dense_300", "dense_1031", "dense_4096"])
def test_apply_a(torch_cuda, case):
    print(f"apply_a {case}", flush=True)
    if case == "laplace2d_32":
        A, grid = synth.laplace2d(32), (32, 32, 1)
    elif case == "diffusion3d_12":
        A, grid = synth.cfg2(N=12).A, (12, 12, 12)
    else:
        A, grid = synth.dense_spd(int(case.split("_")[1]))[0], (0, 0, 0)
    s = _solver(A, 2, 4, "fp64", grid)
    perm = s.permutation()
    Ap = permuted(A, perm)
    rng = np.random.default_rng(1)
    for c in (1, 5, 8, 16, 32, 33, 48, 64, 96):
        X = rng.standard_normal((A.shape[0], c))
        Y = _np(s.apply_a(X))
        ref = Ap @ X
        absA = abs(Ap) if sp.issparse(Ap) else np.abs(Ap)
        bound = (A.shape[0] if not sp.issparse(A) else 8) * U64 * 1.01 * (absA @ np.abs(X))
        assert np.all(np.abs(Y - ref) <= 4 * bound + 1e-300), c
    s.close()


_KAPPA = {}


def _precond_case(case):
    if case == "laplace2d_32":
        return synth.laplace2d(32), (32, 32, 1), 8
    if case == "diffusion3d_16":
        return synth.cfg2(N=16).A, (16, 16, 16), 32
    if case == "diffusion3d_16_graph":
        return synth.cfg2(N=16).A, (0, 0, 0), 16
    if case == "diffusion3d_32":
        return synth.cfg2(N=32).A, (32, 32, 32), 32
    if case == "laplace2d_33x31":
        return synth.laplace2d(33), (0, 0, 0), 13
    return synth.dense_spd(500, seed=4, hi=1e3)[0], (0, 0, 0), 24


def _kappa(case, A):
    """2-norm condition number of A (extreme eigenvalues by Lanczos, the smallest by shift-invert)."""
    if case not in _KAPPA:
        import scipy.sparse.linalg as spla
        if sp.issparse(A):
            lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
            lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
        else:
            lam = np.linalg.eigvalsh(A)
            lmin, lmax = lam[0], lam[-1]
        _KAPPA[case] = lmax / lmin
    return _KAPPA[case]


# Launch plans of the preconditioner: "auto" (what setup picks: one workgroup for the whole tree when the
# panels are small, else one launch sequence per level), "levels" (the per-level gather / tile / split /
# finalize sweeps that large factors take, forced on small ones) and "wide" (per-level sweeps and a
# factor whose every Schur complement runs on 128 x 128 blocks).
_PLANS = {"auto": {}, "levels": {"subtree_levels": -1}, "wide": {"subtree_levels": -1, "schur_wide_tiles": 1}}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case,plan", [("laplace2d_32", "auto"), ("laplace2d_32", "levels"), ("laplace2d_32", "wide"),
                                       ("diffusion3d_16", "auto"), ("diffusion3d_16", "levels"),
                                       ("diffusion3d_16", "wide"), ("diffusion3d_16_graph", "auto"),
                                       ("diffusion3d_16_graph", "levels"), ("dense_500", "auto"),
                                       ("laplace2d_33x31", "auto"), ("laplace2d_33x31", "wide"),
                                       ("diffusion3d_32", "auto")])
def test_apply_precond(torch_cuda, prec, case, plan):
    # Section 5.1's two triangular solves (Algorithm 3 lines 9-10) against the oracle's FP64 solve, column by
    # column: an FP64 factor to 1e-9 relative; an FP32 factor within 4 kappa(A) u32 (a backward-stable
    # Cholesky and solve in single precision; the oracle's own FP32 branch is pinned to the same bound).
    print(f"precond {case} {plan} {prec}", flush=True)
    A, grid, m = _precond_case(case)
    s = _solver(A, 1, m, prec, grid, **_PLANS[plan])
    perm = s.permutation()
    Ap = permuted(A, perm)
    rng = np.random.default_rng(2)
    R = rng.standard_normal((A.shape[0], m))
    W = _np(s.apply_precond(R))
    s.close()
    Wref = opc.Preconditioner(Ap, "fp64")(R)
    col = np.linalg.norm(W - Wref, axis=0) / np.linalg.norm(Wref, axis=0)
    bound = 1e-9 if prec == "fp64" else 4 * _kappa(case, A) * U32
    print(f"  max column error {col.max():.3e} (bound {bound:.3e})", flush=True)
    assert np.all(np.isfinite(W))
    assert col.max() <= bound, (col.max(), bound)
