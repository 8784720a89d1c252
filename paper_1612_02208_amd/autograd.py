"""Differentiable Stokes-IB solve: w(kappa) = L_IB(kappa)^+ b as a
``torch.autograd.Function`` of the per-spring stiffnesses.

Backward solves the adjoint system L_IB^T lam = dLoss/dw with the library's
transposed-operator FGMRES path and returns
    dLoss/dkappa_e = -lam^T (dL_IB/dkappa_e) w
                   = -(dt/h^2) sum_c (B_e J lam_c)(B_e J w_c)
from the spring-gradient kernel (dL_IB/dkappa_e is the IB block of spring e
alone, Eq. matrix-impib with K_h of one spring).  Everything runs in libibmg;
this module only sequences the calls.

The handle's operator is the one built for the last ``set_kappa``.  Each
forward keeps its own stiffness field, and backward rebuilds the handle for
that field when another forward (or a ``set_kappa``) has changed it since, so
the adjoint always uses the operator the forward solved with.
"""
import numpy as np
import torch


class StiffnessSolve(torch.autograd.Function):
    """w = StiffnessSolve.apply(kappa, solver, b, rtol)

    kappa: float64 tensor [n_springs] (any device; copied to the host for
    ``set_kappa``), solver: ``StokesIB`` (FP64 handle recommended for
    gradients), b: float64 CUDA right-hand side.  Returns the float64 CUDA
    solution with null-space components removed."""

    @staticmethod
    def forward(ctx, kappa, solver, b, rtol=1e-12):
        k = np.array(kappa.detach().to("cpu", torch.float64).numpy(), copy=True)
        solver.set_kappa(k)
        w, info = solver.solve(b, rtol=rtol, max_it=400)
        if not info["converged"]:
            raise RuntimeError(f"forward solve did not converge: {info['status']}")
        ctx.solver = solver
        ctx.kappa_host = k
        ctx.rtol = rtol
        ctx.kappa_device = kappa.device
        ctx.save_for_backward(w)
        return w

    @staticmethod
    def backward(ctx, grad_w):
        (w,) = ctx.saved_tensors
        solver = ctx.solver
        if not np.array_equal(solver.kappa, ctx.kappa_host):
            solver.set_kappa(ctx.kappa_host)
        g = grad_w.contiguous().to(torch.float64)
        lam, info = solver.solve(g, rtol=ctx.rtol, max_it=400, transpose=True)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info['status']}")
        dk = solver.spring_gradient(w, lam)
        return dk.to(ctx.kappa_device), None, None, None
