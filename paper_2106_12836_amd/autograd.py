"""Differentiable SAIT-preconditioned solve.

x = A(vals)^-1 b as a torch.autograd.Function.  Forward: restarted FGMRES
on A with the SAIT preconditioner M_U M_L.  Backward (adjoint method):
lambda solves A^T lambda = dl/dx by FGMRES on A^T preconditioned with the
transposed factors, z = M_L^T (M_U^T r); then dl/db = lambda and
dl/dA_ij = -lambda_i x_j on the stored pattern of A.  The preconditioner
is not differentiated: at convergence x does not depend on it.  The
results of the last forward and adjoint solves are kept on the
preconditioner (last_forward_info, last_adjoint_info).
"""

from __future__ import annotations

import torch

from .sait import SaitError, sait_set_values


class SaitSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, pre, restart, maxit, rtol):
        if not pre.opts.build_transpose:
            raise SaitError(-1, "SaitSolve needs a preconditioner built with build_transpose=1")
        vals_c = vals.detach().contiguous()
        sait_set_values(pre.handle, vals_c)
        x, info = pre.solve(b.detach().contiguous(), restart=restart, maxit=maxit, rtol=rtol, flexible=True)
        ctx.pre = pre
        ctx.vals = vals_c
        ctx.opts = (restart, maxit, rtol)
        ctx.info = info
        pre.last_forward_info = info[0]
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        pre = ctx.pre
        restart, maxit, rtol = ctx.opts
        sait_set_values(pre.handle, ctx.vals)
        lam, info = pre.solve(gx.detach().contiguous(), transpose=True, restart=restart, maxit=maxit, rtol=rtol,
                              flexible=True)
        ctx.backward_info = info
        pre.last_adjoint_info = info[0]
        gvals = pre.grad_values(lam, x)
        return gvals, lam, None, None, None, None


def sait_solve_autograd(vals, b, pre, restart=30, maxit=10000, rtol=1e-12):
    """x = A(vals)^-1 b with gradients w.r.t. ``vals`` (A's stored values in
    the CSR order used to build ``pre``) and ``b``."""
    return SaitSolve.apply(vals, b, pre, restart, maxit, rtol)
