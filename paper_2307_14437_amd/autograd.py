"""torch.autograd binding of the GoFD solve: gradients with respect to the grid
right-hand side f and the mesh vertex coordinates X.

Two modes.  ``gofd_solve``: the converged solve, differentiated by the adjoint
of the linear system (below).  ``gofd_solve_unrolled``: a truncated CG solve
(n iterations from x0), differentiated through its iterations in reverse
order by the library (gofd_cg_unrolled_grad), which recomputes the iterates
between checkpoints kept every c iterations.

Forward: build the transfer for the current X (point location and barycentric
weights), then solve eq. GoFD-2.  Backward: the library's adjoint solve
(gofd_solve_adjoint): lambda = K^{-1} dL/du, dL/df = h^{2s} I lambda, and the
weight gradients chained to X through the barycentric coordinates, with the
node-to-element map held fixed (it is locally constant in X almost everywhere).
"""

from __future__ import annotations

import torch

from . import CgTape, Context, FdOp, Precond, Transfer, solve, solve_adjoint


class GoFDProblem:
    """Fixed data of a family of solves: context, element array, grid, order s."""

    def __init__(self, ctx: Context, elems: torch.Tensor, grid, s: float, precond: str = "DIAG", tol: float = 1e-12,
                 M: int = 0):
        self.ctx, self.grid, self.s, self.precond, self.tol = ctx, grid, float(s), precond, float(tol)
        self.elems = elems.to(device="cuda", dtype=torch.int32).contiguous()
        self.op = FdOp(ctx, s, grid, M=M)


class _SolveFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, f, X, prob: GoFDProblem):
        tr = Transfer(prob.ctx, X.detach().contiguous(), prob.elems, prob.grid)
        pc = Precond(prob.ctx, tr, prob.op, prob.precond)
        u, _ = solve(prob.ctx, tr, prob.op, f.detach().contiguous(), tol=prob.tol, pc=pc)
        fctx.prob, fctx.tr, fctx.pc = prob, tr, pc
        fctx.save_for_backward(f, u)
        return u

    @staticmethod
    def backward(fctx, gu):
        f, u = fctx.saved_tensors
        prob = fctx.prob
        gf, gX, _, _ = solve_adjoint(prob.ctx, fctx.tr, prob.op, gu.contiguous(), u, f.contiguous(),
                                     tol=prob.tol, pc=fctx.pc, want_f=fctx.needs_input_grad[0],
                                     want_X=fctx.needs_input_grad[1])
        return (gf.view_as(f) if gf is not None else None), gX, None


def gofd_solve(prob: GoFDProblem, f: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """u(f, X): vertex values of the GoFD-2 solution, differentiable in f and X."""
    return _SolveFn.apply(f, X, prob)


class _UnrolledFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, f, X, x0, prob: GoFDProblem, iters: int, ckpt_every: int, tol: float):
        tr = Transfer(prob.ctx, X.detach().contiguous(), prob.elems, prob.grid)
        tape = CgTape(prob.ctx, tr, prob.op, f.detach(), x0=None if x0 is None else x0.detach(), max_iter=iters,
                      tol=tol, ckpt_every=ckpt_every)
        fctx.tape, fctx.tr, fctx.fshape = tape, tr, f.shape
        return tape.x.clone()

    @staticmethod
    def backward(fctx, gx):
        gf, gX, g0 = fctx.tape.grad(gx.contiguous(), want_f=fctx.needs_input_grad[0],
                                    want_X=fctx.needs_input_grad[1], want_x0=fctx.needs_input_grad[2])
        return (gf.view(fctx.fshape) if gf is not None else None), gX, g0, None, None, None, None


def gofd_solve_unrolled(prob: GoFDProblem, f: torch.Tensor, X: torch.Tensor, x0: torch.Tensor | None = None,
                        iters: int = 50, ckpt_every: int = 8, tol: float = 0.0) -> torch.Tensor:
    """x_n(f, X, x0): n CG iterations on eq. GoFD-2 (stopping early at tol if tol > 0), differentiable in f,
    X and x0 through the iterations (checkpointed every ckpt_every iterations)."""
    return _UnrolledFn.apply(f, X, x0, prob, int(iters), int(ckpt_every), float(tol))
