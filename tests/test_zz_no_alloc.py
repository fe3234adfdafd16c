"""lobpcg_mixed_qr_noalloc (Algorithm 2 with its scratch in the library's fixed device array) against
lobpcg_mixed_qr, the entry point that allocates its scratch, through the C-ABI: the same kernels on the
same plans, so Q and R must agree bit for bit; two calls in a row, the second with a smaller input."""
import ctypes as ct

import numpy as np
import pytest

from paper_2302_12528_amd import native as nv

pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _block(n, c, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, c)))
    V, _ = np.linalg.qr(rng.standard_normal((c, c)))
    return (U * np.geomspace(1.0, 1.0 / kappa, c)) @ V.T


def _qr(torch, fn, W, lower):
    n, c = W.shape
    Q = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    R = torch.empty((c, c), dtype=torch.float64, device="cuda")
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    nv.check(fn(ct.c_void_p(Q.data_ptr()), n, c, c, 1 if lower else 0, ct.c_void_p(R.data_ptr()), st))
    return Q.cpu().numpy(), R.cpu().numpy()


@pytest.mark.parametrize("lower", [True, False])
def test_noalloc_matches_allocating_entry_point(torch_cuda, lower):
    lib = nv.load()
    for (n, c, kappa, seed) in [(200_000, 32, 1e3, 1), (5000, 16, 1e6, 2)]:
        print(f"mixed_qr_noalloc n={n} c={c} kappa={kappa} lower={lower}", flush=True)
        W = _block(n, c, kappa, seed)
        Qa, Ra = _qr(torch_cuda, lib.lobpcg_mixed_qr, W, lower)
        Qn, Rn = _qr(torch_cuda, lib.lobpcg_mixed_qr_noalloc, W, lower)
        assert np.array_equal(Qn, Qa) and np.array_equal(Rn, Ra)
        assert np.linalg.norm(Qn.T @ Qn - np.eye(c)) <= 10 * c * U64
        assert np.linalg.norm(W - Qn @ Rn) / np.linalg.norm(W) <= 100 * U64


def test_noalloc_rejects_sizes_beyond_its_array(torch_cuda):
    lib = nv.load()
    W = torch_cuda.zeros((8, 8), dtype=torch_cuda.float64, device="cuda")
    st = lib.lobpcg_mixed_qr_noalloc(ct.c_void_p(W.data_ptr()), 2_000_000, 64, 64, 1, None, None)
    assert st == nv.LOBPCG_ERR_INVALID_ARG and "scratch" in nv.last_error()
