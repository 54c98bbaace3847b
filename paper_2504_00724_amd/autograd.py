"""torch.autograd.Function around the solve.

u = L^{-1} (f - N g) (eq. PoissonResidualForm), so for a loss J(u) the
adjoint lambda = L^{-T} dJ/du gives dJ/df = lambda and dJ/dg = -N^T lambda.
Both solves run in the native library on torch's current stream.
"""
import torch


class CutCellSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g, solver):
        n = solver.n_cells
        nf = solver.info["n_bdry_faces"]
        if f.dim() == 1:
            nrhs = 1
        elif f.dim() == 2:
            nrhs = f.shape[0]
        else:
            raise ValueError("f must be [ny*nx] or [nrhs, ny*nx], got shape %s" % (tuple(f.shape),))
        if f.shape[-1] != n:
            raise ValueError("f has %d cells per right-hand side, the grid has %d" % (f.shape[-1], n))
        # one boundary datum per face for every right-hand side; a single
        # [n_faces] vector is shared by all of them (its gradient sums theirs)
        if g.dim() == 1 and g.shape[0] == nf:
            gb = g.unsqueeze(0).expand(nrhs, nf)
        elif g.dim() == 2 and tuple(g.shape) == (nrhs, nf):
            gb = g
        else:
            raise ValueError("g must be [%d] or [%d, %d], got shape %s" % (nf, nrhs, nf, tuple(g.shape)))
        f = f.contiguous()
        gb = gb.contiguous()
        u = torch.zeros_like(f)
        solver.set_boundary(gb, nrhs)
        solver.solve(f, u, nrhs)
        ctx.solver = solver
        ctx.nrhs = nrhs
        ctx.gshape = g.shape
        ctx.shared_g = g.dim() == 1 and nrhs > 1
        return u

    @staticmethod
    def backward(ctx, grad_u):
        S = ctx.solver
        nrhs = ctx.nrhs
        nf = S.info["n_bdry_faces"]
        grad_u = grad_u.contiguous()
        lam = torch.zeros_like(grad_u)
        S.solve_adjoint(grad_u, lam, nrhs)
        ng = torch.zeros((nrhs, nf), dtype=grad_u.dtype, device=grad_u.device)
        if nf:
            S.apply_NT(lam, ng, nrhs)
        dg = -ng.sum(dim=0) if ctx.shared_g else -ng.reshape(ctx.gshape)
        return lam, dg, None


def cutcell_solve(f, g, solver):
    """Differentiable solve: f [ny*nx] or [nrhs, ny*nx]; g [n_faces] (shared
    by every right-hand side) or [nrhs, n_faces]."""
    return CutCellSolve.apply(f, g, solver)
