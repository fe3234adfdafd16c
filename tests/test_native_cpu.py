"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
validates arguments before touching the GPU, and its host symbolic analysis
produces a valid ordering whose supernodal fill contains the exact fill."""
import ctypes as ct
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from paper_2302_12528_amd import native as nv
from paper_2302_12528_amd import solver as sv

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lobpcg.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lobpcg_status|const char\*|int32_t)\s+(lobpcg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in nv.SIGNATURES, name


def test_status_strings(lib):
    for s in range(9):
        assert lib.lobpcg_status_string(s)


def _setup(A, k, m, tol, prec=nv.LOBPCG_FP32, grid=(0, 0, 0)):
    lib = nv.load()
    M, keep = sv.make_matrix(A, grid)
    ctx = ct.c_void_p()
    st = lib.lobpcg_setup(ct.byref(M), k, m, tol, prec, None, None, ct.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("k,m,tol,msg", [(0, 8, 1e-8, "k <= m"), (9, 8, 1e-8, "k <= m"), (4, 8, 0.0, "tol"),
                                         (4, 8, float("nan"), "tol"), (4, 65, 1e-8, "<= 64"),
                                         (4, 40, 1e-8, "3m <= n")])
def test_setup_rejects_bad_arguments(lib, k, m, tol, msg):
    A = synth.laplace2d(10)
    st, ctx = _setup(A, k, m, tol)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and not ctx.value
    assert msg in nv.last_error()


def test_setup_rejects_bad_matrices(lib):
    A = synth.laplace2d(10).tolil()
    A[0, 5] = 1.0                           # asymmetric pattern
    st, _ = _setup(A.tocsr(), 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "symmetric" in nv.last_error()
    B = synth.laplace2d(10).copy()
    B.data[3] = np.nan
    st, _ = _setup(B, 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "non-finite" in nv.last_error()
    C = synth.laplace2d(10).tolil()
    C[3, 3] = -1.0
    st, _ = _setup(C.tocsr(), 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "diagonal" in nv.last_error()
    D = np.eye(40)
    D[0, 1] = 0.5
    st, _ = _setup(D, 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "symmetric" in nv.last_error()
    st, _ = _setup(synth.laplace2d(10), 2, 4, 1e-8, prec=7)
    assert st == nv.LOBPCG_ERR_INVALID_ARG


def _setup_batched(mats, k, m, tol, prec=nv.LOBPCG_FP32):
    lib = nv.load()
    arr = (nv.Matrix * max(1, len(mats)))()
    keep = []
    for b, A in enumerate(mats):
        M, kp = sv.make_matrix(A)
        arr[b] = M
        keep.append(kp)
    ctx = ct.c_void_p()
    st = lib.lobpcg_setup_batched(arr, len(mats), k, m, tol, prec, None, None, ct.byref(ctx))
    return st, ctx


def test_batched_setup_rejects_bad_arguments(lib):
    L = synth.laplace2d(10)
    st, ctx = _setup_batched([], 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and not ctx.value and "at least one" in nv.last_error()
    st, ctx = _setup_batched([L, np.eye(40) * 2.0], 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "not batched" in nv.last_error()
    st, ctx = _setup_batched([L, synth.laplace2d(3)], 2, 4, 1e-8)   # n = 9 < 3m for the second
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "3m <= n" in nv.last_error()
    bad = synth.laplace2d(6).copy()
    bad.data[0] = np.inf
    st, ctx = _setup_batched([L, bad], 2, 4, 1e-8)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "non-finite" in nv.last_error()
    assert lib.lobpcg_solve_batched(None, None, 10, None, None, None) == nv.LOBPCG_ERR_INVALID_ARG
    assert lib.lobpcg_batch_count(None) == 0


def test_solve_and_backward_reject_null_context(lib):
    assert lib.lobpcg_solve(None, None, 10, None, None, None) == nv.LOBPCG_ERR_INVALID_ARG
    assert lib.lobpcg_pinvit(None, None, 10, None, None, None, None) == nv.LOBPCG_ERR_INVALID_ARG
    assert lib.lobpcg_backward(None, None, None, None) == nv.LOBPCG_ERR_INVALID_ARG
    assert lib.lobpcg_destroy(None) == nv.LOBPCG_OK


def _exact_fill(Ap):
    """nnz of the lower Cholesky factor of the permuted matrix (structural, via dense LU-free elimination)."""
    n = Ap.shape[0]
    pat = (Ap.toarray() != 0)
    nnz = 0
    for j in range(n):
        rows = np.nonzero(pat[j:, j])[0] + j
        nnz += rows.size
        # eliminating column j connects all its lower neighbours
        pat[np.ix_(rows, rows)] = True
    return nnz


@pytest.mark.parametrize("case", ["grid3d_8", "graph3d_8", "grid2d_20", "graph2d_20", "schrodinger2d_15"])
def test_symbolic_ordering_and_fill(lib, case):
    if case.endswith("3d_8"):
        A = synth.cfg2(N=8).A
        grid = (8, 8, 8) if case.startswith("grid") else (0, 0, 0)
    elif case.endswith("2d_20"):
        A = synth.laplace2d(20)
        grid = (20, 20, 1) if case.startswith("grid") else (0, 0, 0)
    else:
        A = synth.schrodinger((15, 15), np.array([[0.3, 0.4]]), np.array([0.1]), np.array([5.0]))
        grid = (15, 15, 1)
    perm, st = sv.symbolic(A, grid=grid, leaf_size=16)
    n = A.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n))
    Ap = sp.csr_matrix(A)[perm][:, perm]
    exact = _exact_fill(Ap)
    assert st["nnz_factor"] >= exact
    assert sv.exact_fill(A, grid=grid, leaf_size=16) == exact
    assert st["nnz_factor"] <= 2.5 * exact      # relaxed supernodes add a bounded amount of explicit zeros
    assert st["levels"] >= 2


def test_symbolic_dense(lib):
    A, _ = synth.dense_spd(100)
    perm, st = sv.symbolic(A)
    assert np.array_equal(perm, np.arange(100))
    assert st["supernodes"] == 1 and st["nnz_factor"] == 100 * 101 / 2


def test_symbolic_64cube_plan_size(lib):
    A = synth.cfg2(N=64).A
    perm, st = sv.symbolic(A, grid=(64, 64, 64), leaf_size=64)
    # exact geometric nested-dissection fill with 64-node leaves is 1.567e8; the relaxed supernodes stay
    # within 15 % of it
    assert 1.5e8 < st["nnz_factor"] < 1.8e8
    exact = sv.exact_fill(A, grid=(64, 64, 64), leaf_size=64)
    assert 1.5e8 < exact < st["nnz_factor"]
    assert st["levels"] == 13
    # the default for a 3D grid: 256-node leaves, two levels fewer for about 11 % more stored entries
    perm2, st2 = sv.symbolic(A, grid=(64, 64, 64))
    assert st2["levels"] == 11 and st["nnz_factor"] < st2["nnz_factor"] < 1.15 * st["nnz_factor"]
    assert abs(st2["flops"] / st["flops"] - 1.0) < 0.03
    assert sorted(perm2.tolist()) == list(range(64 ** 3))
    # a 2D grid keeps 64-node leaves
    B = synth.laplace2d_rect(40, 50)
    assert np.array_equal(sv.symbolic(B, grid=(40, 50, 1))[0], sv.symbolic(B, grid=(40, 50, 1), leaf_size=64)[0])


def test_mixed_qr_noalloc_rejects_oversized_problems_before_gpu_work(lib):
    # the size check runs on the host before the scratch array or W is touched
    fake = ct.c_void_p(0x1000)
    st = lib.lobpcg_mixed_qr_noalloc(fake, 4_000_000, 64, 64, 0, None, None)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "scratch" in nv.last_error()
    st = lib.lobpcg_mixed_qr_noalloc(fake, 100, 65, 65, 1, None, None)
    assert st == nv.LOBPCG_ERR_INVALID_ARG


def test_hermitian_setup_validates_on_the_host(lib):
    # complex CSR (format 2): a matrix that is not Hermitian, and block sizes beyond the embedding's limit,
    # are rejected before any GPU work
    A = synth.gauge_laplace2d(6, 7).tolil()
    A[0, 1] = A[0, 1] * 1j   # breaks A_10 = conj(A_01)
    M, keep = sv.make_matrix(A.tocsr(), (6, 7, 1))
    assert M.format == 2
    ctx = ct.c_void_p()
    st = lib.lobpcg_setup_hermitian(ct.byref(M), 2, 4, 1e-10, nv.LOBPCG_FP32, None, None, ct.byref(ctx))
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "Hermitian" in nv.last_error()
    M, keep = sv.make_matrix(synth.gauge_laplace2d(6, 7), (6, 7, 1))
    st = lib.lobpcg_setup_hermitian(ct.byref(M), 2, 40, 1e-10, nv.LOBPCG_FP32, None, None, ct.byref(ctx))
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "m must be" in nv.last_error()
    assert lib.lobpcg_solve_hermitian(None, None, 10, None, None, None) == nv.LOBPCG_ERR_INVALID_ARG
