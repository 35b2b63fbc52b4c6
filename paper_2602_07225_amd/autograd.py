"""Differentiable solve: ``x = A(sigma, Ds)^-1 b`` as a torch autograd node.

Forward: uploads the per-element solid conductivity ``sigma`` and the
particle diffusivities ``Ds`` into the solver context, builds the
preconditioner and solves (p4d_setup + p4d_solve).  Backward: one adjoint
solve ``A^T lambda = dL/dx`` with the transposed operator and transposed
preconditioner (p4d_solve_adjoint), then ``dL/dp = -lambda^T (dA/dp) x``
(p4d_param_gradient) and ``dL/db = lambda``.  All arithmetic runs in the HIP
library.  The electrolyte conductivity, the separate transport coefficients,
the per-element porosity and the Butler-Volmer derivatives are held fixed at
their uploaded values.

The forward pass records the solver's state (coefficients, diffusivities,
preconditioner options) and its version counter.  If anything changed the
context between this forward and its backward (another forward, an upload,
a new setup), the backward first restores the recorded state, so the
adjoint solve and the gradient use the operator of this forward pass."""
from __future__ import annotations

import torch

from . import _lib as L


class P4DSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, sigma, Ds, b, opts=None):
        opts = dict(opts or {})
        dev = solver.device
        sig = sigma.detach().to(dev, torch.float64).contiguous().clone()
        # upload() re-applies the separate transport coefficients and the
        # porosity that the library's upload resets
        solver.upload(sig, solver._kappa, solver._g, solver._s, solver._e)
        Dh = [float(v) for v in Ds.detach().cpu().tolist()]
        solver.set_diffusivity(Dh)
        solver.setup(**opts)
        x, info = solver.solve(b.detach().to(dev, torch.float64))
        if info.status != L.P4D_OK:
            raise L.P4DError(info.status, "forward solve did not converge")
        ctx.solver = solver
        ctx.opts = opts
        ctx.state = solver.state()
        ctx.version = solver.version
        ctx.devs = (sigma.device, Ds.device, b.device)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        s = ctx.solver
        if s.version != ctx.version:
            s.restore(ctx.state, **ctx.opts)
        lam, info = s.solve_adjoint(grad_x.contiguous())
        if info.status != L.P4D_OK:
            raise L.P4DError(info.status, "adjoint solve did not converge")
        dsig, dDs = s.gradient(x, lam)
        ds_dev, dD_dev, db_dev = ctx.devs
        return None, dsig.to(ds_dev), dDs.to(dD_dev), lam.to(db_dev), None


def solve(solver, sigma, Ds, b, **opts):
    """Differentiable ``x = A(sigma, Ds)^-1 b`` (see module docstring)."""
    return P4DSolve.apply(solver, sigma, Ds, b, opts)
