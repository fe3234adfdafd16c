"""torch.autograd.Function over lobpcg_solve / lobpcg_backward for a diagonal potential.

A(V) = A0 + diag(V), with A0 the matrix the Solver was set up with.  forward()
refactors A(V) and solves for the k smallest eigenpairs; backward() returns
dL/dV from the library's adjoint (Hellmann-Feynman term plus projected
preconditioned adjoint solves).  One forward may be in flight per Solver: the
backward uses the eigenpairs the Solver holds from its latest solve.
"""
from __future__ import annotations

import torch


class LobpcgEig(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, solver, X0=None, maxit: int = 1000):
        solver.update_values(shift=V.detach())
        lam, X, info = solver.solve(X0, maxit=maxit)
        ctx.solver = solver
        ctx.info = info
        return lam, X

    @staticmethod
    def backward(ctx, dlam, dX):
        g = ctx.solver.backward(dlam, dX)
        return g, None, None, None


def eigh_potential(V, solver, X0=None, maxit: int = 1000):
    """(evals, evecs) of A0 + diag(V), differentiable with respect to V."""
    return LobpcgEig.apply(V, solver, X0, maxit)
