"""Differentiable SRJ solve: a torch.autograd.Function over the C ABI.

Forward: u = solution of the Poisson problem with source f and Dirichlet ring g
(``srj_solve``).  Backward: one adjoint SRJ solve on the same symmetric operator
(``srj_adjoint``), which returns dL/df and dL/dg directly; no iterate of the forward solve
is stored.  Tensors are float64 CUDA tensors in the full-grid layout with the ring.

The backward solve has its own tolerance.  Its right-hand side dL/du is usually smooth, and
then binary64 cannot represent lambda = A^-1 dL/du with a relative residual much below
8 eps / lambda_min (about 2e-10 on a 2048^2 grid), while for such a right-hand side the
relative residual also bounds the relative error of lambda; 1e-9 is the default.
"""
import torch

from . import srj


class SRJSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, g, plan, tol, max_sweeps, tol_backward):
        u = g.detach().clone()
        inner = tuple(slice(1, -1) for _ in range(u.dim()))
        u[inner] = 0.0
        info = srj.srj_solve(plan, u, f.detach().contiguous(), tol, max_sweeps)
        if info["status"] != "ok":
            raise srj.SrjError(5 if info["status"] == "enoconv" else 6, f"forward solve: {info}")
        ctx.plan, ctx.tol, ctx.max_sweeps = plan, tol_backward, max_sweeps
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
        ctx.backward_info = info  # readable as u.grad_fn.backward_info after backward()
        return df, dg, None, None, None, None


def srj_solve_diff(f, g, plan, tol=1e-10, max_sweeps=None, tol_backward=1e-9):
    """u(f, g) with gradients to f (interior) and g (ring) by the adjoint SRJ solve.

    max_sweeps defaults to 200 cycles of the plan's schedule; a solve that does not reach
    tol within it raises instead of running on."""
    if max_sweeps is None:
        max_sweeps = 200 * int(srj.srj_plan_describe(plan)["M"])
    return SRJSolve.apply(f, g, plan, tol, max_sweeps, tol_backward)
