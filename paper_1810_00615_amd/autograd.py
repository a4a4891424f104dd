"""torch.autograd front end: U = solve(A(kappa) U = b(u0)) with gradients w.r.t.
the initial state u0 and the coefficient kappa by the adjoint (transposed) solve.

Forward: FGMRES on A U = b with C^{-1}.  Backward: FGMRES on A^T lam = dL/dU with
C^{-T} (the conjugated symbol), then dL/du0 = (db/du0)^T lam and
dL/dkappa = lam^T db/dkappa - lam^T (dA/dkappa) U.  With checkpoint_stride c > 1
only every c-th time level of U is kept for the backward pass (memory n ell / c)
and the rest is recomputed by time stepping on the device (heat scheme)."""
from __future__ import annotations

import torch


class AllAtOnceSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, kappa, problem, restart=30, tol=1e-10, maxit=300, checkpoint_stride=1,
                v0=None):
        problem.set_kappa(float(kappa))
        b = problem.rhs(u0.detach().contiguous(), None if v0 is None else v0.detach().contiguous())
        U, info = problem.solve(b, restart=restart, tol=tol, maxit=maxit)
        if not info["converged"]:
            raise RuntimeError(f"forward all-at-once solve did not converge: {info}")
        c = int(checkpoint_stride)
        ctx.problem = problem
        # the Problem is shared: backward re-selects the kappa of this forward pass
        ctx.kappa = float(kappa)
        ctx.opts = (restart, tol, maxit, c)
        ctx.has_v0 = v0 is not None
        if c > 1:
            Uck = U[c - 1::c].contiguous()
            ctx.save_for_backward(u0.detach(), Uck, v0.detach() if v0 is not None else None)
        else:
            ctx.save_for_backward(u0.detach(), U.detach(), v0.detach() if v0 is not None else None)
        return U

    @staticmethod
    def backward(ctx, gU):
        problem = ctx.problem
        restart, tol, maxit, c = ctx.opts
        u0, Usaved, v0 = ctx.saved_tensors
        problem.set_kappa(ctx.kappa)
        lam, info = problem.adjoint(gU.contiguous(), restart=restart, tol=tol, maxit=maxit)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        if c > 1:
            gu, gk = problem.grad_checkpointed(u0, Usaved, c, lam)
            gv = None
        else:
            gu, gv, gk = problem.grad(Usaved, lam, u0, v0, want_v0=ctx.has_v0)
        gkappa = torch.tensor(gk, dtype=torch.float64, device=u0.device)
        return gu, gkappa, None, None, None, None, None, gv


def all_at_once_solve(u0, kappa, problem, restart=30, tol=1e-10, maxit=300, checkpoint_stride=1,
                      v0=None):
    """Differentiable all-at-once solve; kappa may be a float or a 0-dim tensor."""
    if not torch.is_tensor(kappa):
        kappa = torch.tensor(float(kappa), dtype=torch.float64, device=u0.device)
    return AllAtOnceSolve.apply(u0, kappa, problem, restart, tol, maxit, checkpoint_stride, v0)
