"""Device memory through the caller's allocator (lobpcg_options.allocator): with torch's caching
allocator every device byte of a context is a torch block, the results equal those of a context
that uses hipMalloc, and destroying the context returns the blocks."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_torch_allocator_owns_context_memory(torch_cuda):
    import paper_2302_12528_amd as pk
    torch = torch_cuda
    print("allocator torch vs hip, diffusion3d_16", flush=True)
    p = synth.cfg2(N=16, k=8, m=16)
    X0 = torch.from_numpy(np.ascontiguousarray(p.X0)).cuda()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp32", grid=(16, 16, 16), allocator="torch",
                  stage1_tol=5e-6)
    lam_t, X_t, info_t = s.solve(X0)
    lam_t, X_t = lam_t.cpu().numpy(), X_t.cpu().numpy()
    held = torch.cuda.memory_allocated() - before
    # the factor panels alone are about 4 * nnz_factor bytes
    assert held >= 4 * info_t["nnz_factor"], (held, info_t["nnz_factor"])
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    h = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp32", grid=(16, 16, 16), allocator="hip",
                  stage1_tol=5e-6)
    lam_h, X_h, info_h = h.solve(X0)
    h.close()
    assert info_t["iters"] == info_h["iters"] and info_t["stage1_iters"] == info_h["stage1_iters"]
    assert np.array_equal(lam_t, lam_h.cpu().numpy()) and np.array_equal(X_t, X_h.cpu().numpy())
