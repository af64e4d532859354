"""Differentiable PSLR-FGMRES solve: z = A^{-1} b with gradients for A's nonzeros and b.

Forward: right-preconditioned FGMRES with the PSLR apply (Algorithm 3).
Backward (adjoint): lambda = A^{-T} dL/dz by FGMRES with the transposed apply
M^{-T}, then dL/dA_ij = -lambda_i z_j on the stored pattern of A (SDDMM) and
dL/db = lambda.  All three run in libpslr.so; this module only wires them into
torch.autograd.
"""
from __future__ import annotations

import torch

from . import pslr as P


class PSLRSolve(torch.autograd.Function):
    """Apply with ``PSLRSolve.apply(vals, b, handle, tol, restart, maxit, adj_tol)``.

    ``handle`` must come from ``pslr_setup(..., want_transpose=True)`` on the
    matrix whose CSR values are ``vals`` (original CSR order); ``vals`` is an
    input only so that autograd can return its gradient.  The forward checks
    ``vals`` against the handle's fingerprint of those values (count, sum,
    sum of squares) and raises when they differ: new values need a new handle.  ``b``: (n,) or
    (nrhs, n) float64 device tensor.  ``tol`` / ``adj_tol``: relative residual
    targets of the forward and adjoint solves (the adjoint defaults to ``tol``).
    """

    @staticmethod
    def forward(ctx, vals, b, handle, tol=1e-10, restart=40, maxit=500, adj_tol=None):
        # the handle's factors and A belong to the values it was set up with:
        # a changed vals needs a new handle
        cnt, s1, s2 = handle.vals_fingerprint
        v = vals.detach().to(torch.float64)
        if v.numel() != cnt or not (abs(float(v.sum()) - s1) <= 1e-12 * max(1.0, abs(s1) + s2 ** 0.5 * cnt ** 0.5)
                                    and abs(float((v * v).sum()) - s2) <= 1e-12 * max(1.0, s2)):
            raise ValueError("vals differ from the matrix the handle was set up with: "
                             "rebuild the handle with pslr_setup for new values")
        x = torch.zeros_like(b)
        st, its, rel = P.fgmres_solve(handle, b.contiguous(), x, restart=restart, maxit=maxit, tol=tol)
        if st != P.PSLR_OK:
            raise RuntimeError("forward FGMRES did not converge: its %s relres %s" % (its, rel))
        ctx.iterations = [int(v) for v in its]
        ctx.handle = handle
        ctx.opts = (tol if adj_tol is None else adj_tol, restart, maxit)
        ctx.nnz = vals.numel()
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gz):
        (x,) = ctx.saved_tensors
        tol, restart, maxit = ctx.opts
        lam = torch.zeros_like(gz)
        st, its, rel = P.fgmres_solve(ctx.handle, gz.contiguous(), lam, restart=restart,
                                      maxit=maxit, tol=tol, transpose=True)
        if st != P.PSLR_OK:
            raise RuntimeError("adjoint FGMRES did not converge: its %s relres %s" % (its, rel))
        grad_vals = torch.zeros(ctx.nnz, dtype=torch.float64, device=gz.device)
        P.pslr_sddmm_grad(ctx.handle, lam, x, grad_vals)
        return grad_vals, lam, None, None, None, None, None


def pslr_solve(vals, b, handle, tol=1e-10, restart=40, maxit=500, adj_tol=None):
    return PSLRSolve.apply(vals, b, handle, tol, restart, maxit, adj_tol)
