"""torch.autograd.Function around the solve.

u = L^{-1} (f - N g) (eq. PoissonResidualForm), so for a loss J(u) the
adjoint lambda = L^{-T} dJ/du gives dJ/df = lambda and dJ/dg = -N^T lambda.
Both solves run in the native library on torch's current stream.
"""
import torch


class CutCellSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g, solver):
        nrhs = f.shape[0] if f.dim() == 2 else 1
        f = f.contiguous()
        g = g.contiguous()
        u = torch.zeros_like(f)
        solver.set_boundary(g, nrhs)
        solver.solve(f, u, nrhs)
        ctx.solver = solver
        ctx.nrhs = nrhs
        ctx.gshape = g.shape
        return u

    @staticmethod
    def backward(ctx, grad_u):
        S = ctx.solver
        lam = torch.zeros_like(grad_u)
        S.solve_adjoint(grad_u.contiguous(), lam, ctx.nrhs)
        ng = torch.zeros(ctx.gshape, dtype=grad_u.dtype, device=grad_u.device)
        if ng.numel():
            S.apply_NT(lam, ng, ctx.nrhs)
        return lam, -ng, None


def cutcell_solve(f, g, solver):
    """Differentiable solve: f [ny*nx] or [nrhs, ny*nx], g [n_faces] or [nrhs, n_faces]."""
    return CutCellSolve.apply(f, g, solver)
