"""Graph mode: every steady-state iteration is one replay of a captured HIP graph.

The replays are interleaved with the solve's own eager work (residual, host
convergence test) and synchronisations; the final Ritz pairs must be bitwise
identical to the eager launches, over several solves (so over many replays of
both captured graphs), for one problem and for a batch.
"""
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


@pytest.mark.parametrize("case", ["laplace2d_32", "diffusion3d_16"])
def test_graph_bitwise_equals_eager(torch_cuda, case):
    import paper_2302_12528_amd as pk
    p = synth.cfg1() if case == "laplace2d_32" else synth.cfg2(N=16)
    print(f"graph vs eager {case}", flush=True)
    eager = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision=p.factor_precision, grid=p.grid)
    lam0, X0, info0 = eager.solve(p.X0)
    eager.close()
    g = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision=p.factor_precision, grid=p.grid, graph=True)
    for rep in range(3):
        lam, X, info = g.solve(p.X0)
        assert info["iters"] == info0["iters"]
        assert np.array_equal(lam.cpu().numpy(), lam0.cpu().numpy()), rep
        assert np.array_equal(X.cpu().numpy(), X0.cpu().numpy()), rep
    g.close()


def test_graph_batched(torch_cuda):
    import paper_2302_12528_amd as pk
    probs = synth.cfg4(5, side_override=lambda s: 16 + s // 8)
    kw = dict(grids=[p.grid for p in probs])
    e = pk.BatchedSolver([p.A for p in probs], 8, 16, 1e-10, **kw)
    ev0, ec0, inf0, _ = e.solve([p.X0 for p in probs])
    e.close()
    g = pk.BatchedSolver([p.A for p in probs], 8, 16, 1e-10, graph=True, **kw)
    for rep in range(2):
        ev, ec, inf, _ = g.solve([p.X0 for p in probs])
        for b in range(len(probs)):
            assert inf[b]["iters"] == inf0[b]["iters"]
            assert np.array_equal(ev[b].cpu().numpy(), ev0[b].cpu().numpy()), (rep, b)
            assert np.array_equal(ec[b].cpu().numpy(), ec0[b].cpu().numpy()), (rep, b)
    g.close()
