"""GPU gradients of eigenvalue/eigenvector losses with respect to a diagonal potential.

Checked against the oracle's dense gradient (textbook perturbation theory via a
dense eigensolver), the shift invariant sum_j dlambda_i/dV_j = ||x_i||^2 = 1,
and central finite differences of the GPU forward solve.
"""
import numpy as np
import pytest

import synth
from oracle import grad as ograd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(N, k, m, seed=0, prec="fp32"):
    import paper_2302_12528_amd as pk
    r = np.random.default_rng(seed)
    c = r.uniform(0, 1, (6, 3)); w = r.uniform(0.05, 0.2, 6); a = r.uniform(0, 20, 6)
    L0 = synth.laplace_scaled((N, N, N))
    phi = synth.bump_basis(synth.grid_points((N, N, N)), c, w)
    g = r.standard_normal(N ** 3); g /= np.linalg.norm(g)
    X0 = r.standard_normal((N ** 3, m))
    solver = pk.Solver(L0, k, m, 1e-12, factor_precision=prec, grid=(N, N, N))
    return solver, L0, phi, a, g, X0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grad_diag_vs_dense_oracle(torch_cuda, prec):
    torch = torch_cuda
    N, k, m = 10, 4, 8
    print(f"backward N={N} k={k} prec={prec}", flush=True)
    solver, L0, phi, a, g, X0 = _setup(N, k, m, prec=prec)
    V = phi @ a
    solver.update_values(shift=torch.from_numpy(V).cuda())
    lam, X, info = solver.solve(X0)
    Xn = X.cpu().numpy()
    gx = float(g @ Xn[:, 0])
    dX = np.zeros_like(Xn)
    dX[:, 0] = 2.0 * gx * g
    gv = solver.backward(torch.ones(k, dtype=torch.float64), torch.from_numpy(dX)).cpu().numpy()
    A = (L0 + np.diag(V) if not hasattr(L0, "toarray") else L0.toarray() + np.diag(V))
    loss, gref, lam_ref, _ = ograd.loss_and_grad_diag(A, k, g)
    err = np.max(np.abs(gv - gref)) / np.max(np.abs(gref))
    print(f"backward {prec}: max rel err {err:.2e}", flush=True)
    assert err < 1e-8
    solver.close()


def test_shift_invariant(torch_cuda):
    torch = torch_cuda
    N, k, m = 8, 3, 8
    solver, L0, phi, a, g, X0 = _setup(N, k, m, seed=3)
    solver.update_values(shift=torch.from_numpy(phi @ a).cuda())
    solver.solve(X0)
    for i in range(k):
        e = torch.zeros(k, dtype=torch.float64)
        e[i] = 1.0
        gv = solver.backward(e, None).cpu().numpy()
        assert abs(gv.sum() - 1.0) < 1e-12
        assert np.all(gv >= -1e-15)
    solver.close()


def test_autograd_amplitudes_fd(torch_cuda):
    torch = torch_cuda
    from paper_2302_12528_amd.autograd import eigh_potential
    N, k, m = 8, 3, 8
    solver, L0, phi, a, g, X0 = _setup(N, k, m, seed=5)
    phit = torch.from_numpy(phi).cuda()
    gt = torch.from_numpy(g).cuda()
    X0t = torch.from_numpy(X0).cuda()

    def loss_of(amp):
        lam, X = eigh_potential(phit @ amp, solver, X0t)
        return lam.sum() + (X[:, 0] @ gt) ** 2

    amp = torch.from_numpy(a.copy()).cuda().requires_grad_(True)
    L = loss_of(amp)
    (ga,) = torch.autograd.grad(L, amp)
    ga = ga.cpu().numpy()
    h = 1e-6
    for q in range(3):
        e = torch.zeros_like(amp)
        e[q] = h
        with torch.no_grad():
            fd = (loss_of(amp.detach() + e) - loss_of(amp.detach() - e)).item() / (2 * h)
        assert abs(fd - ga[q]) <= 1e-4 * max(1.0, abs(ga[q])), (q, fd, ga[q])
    solver.close()
