"""Differentiable SRJ solve: a torch.autograd.Function over the C ABI.

Forward: u = solution of the Poisson problem with source f and Dirichlet ring g
(``srj_solve``).  Backward: one adjoint SRJ solve on the same symmetric operator
(``srj_adjoint``), which returns dL/df and dL/dg directly; no iterate of the forward solve
is stored.  Tensors are float64 CUDA tensors in the full-grid layout with the ring.
"""
import torch

from . import srj


class SRJSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g, plan, tol, max_sweeps):
        u = g.detach().clone()
        inner = tuple(slice(1, -1) for _ in range(u.dim()))
        u[inner] = 0.0
        info = srj.srj_solve(plan, u, f.detach().contiguous(), tol, max_sweeps)
        if info["status"] != "ok":
            raise srj.SrjError(5 if info["status"] == "enoconv" else 6, f"forward solve: {info}")
        ctx.plan, ctx.tol, ctx.max_sweeps = plan, tol, max_sweeps
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, grad_u):
        grad_u = grad_u.contiguous()
        df = torch.empty_like(grad_u)
        dg = torch.empty_like(grad_u)
        info = srj.srj_adjoint(ctx.plan, grad_u, ctx.tol, ctx.max_sweeps, df, dg)
        if info["status"] != "ok":
            raise srj.SrjError(5 if info["status"] == "enoconv" else 6, f"adjoint solve: {info}")
        return df, dg, None, None, None


def srj_solve_diff(f, g, plan, tol=1e-10, max_sweeps=10 ** 9):
    """u(f, g) with gradients to f (interior) and g (ring) by the adjoint SRJ solve."""
    return SRJSolve.apply(f, g, plan, tol, max_sweeps)
