"""The converged hyper-reduced RVE map as a differentiable torch operation.

``hrom_pbar(plan, theta, Fbar)`` runs the device micro Newton (``hrom_newton``)
at the macro deformation gradients ``Fbar`` [9, N] and material parameters
``theta`` [4] (mu0, lambda0, mu1, lambda1) and returns the homogenised first
Piola-Kirchhoff stress ``Pbar`` [9, N] and the consistent macro tangent
``Cbar`` [81, N] (the latter not differentiable).  Its backward is the
library's adjoint ``hrom_backward``: dL/dFbar and dL/dtheta of the converged
map, with the amplitudes a eliminated through the implicit function theorem
(the ROM residual r(a, Fbar, theta) = 0 of Sec. 3.2.1 holds at the solution).

All arithmetic runs in the library's kernels; this module sequences calls.
"""
from __future__ import annotations

import torch

from . import binding as B


class _HromPbar(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, Fbar, plan, a0, tol, max_it):
        theta = theta.detach().contiguous()
        Fbar = Fbar.detach().contiguous()
        a = plan.zeros_modes() if a0 is None else a0.detach().clone()
        Pbar = plan.zeros_points(9)
        Cbar = plan.zeros_points(81)
        rnorm = torch.zeros(plan.N, dtype=torch.float64, device=Fbar.device)
        status = plan.status()
        plan.newton(theta, Fbar, a, Pbar, Cbar, rnorm, status, tol=tol, max_it=max_it)
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.save_for_backward(theta, Fbar, a, status)
        ctx.mark_non_differentiable(Cbar, a, status)
        return Pbar, Cbar, a, status

    @staticmethod
    def backward(ctx, gPbar, _gC, _ga, _gs):
        theta, Fbar, a, status = ctx.saved_tensors
        plan = ctx.plan
        if gPbar is None:
            return None, None, None, None, None, None
        st = status.clone()
        if plan.generation != ctx.generation:
            # The plan was used since the forward solve: rebuild the stored
            # factorisation at the converged amplitudes (no update between).
            P = plan.zeros_points(9)
            Cb = plan.zeros_points(81)
            rn = torch.zeros(plan.N, dtype=torch.float64, device=Fbar.device)
            plan.eval(theta, Fbar, a, st)
            plan.condense(P, Cb, rn, st)
            ctx.generation = plan.generation
        gF = plan.zeros_points(9)
        gth = torch.zeros(4, dtype=torch.float64, device=Fbar.device)
        plan.backward(theta, a, gPbar.contiguous().to(torch.float64), gF, gth, st)
        gtheta = gth if ctx.needs_input_grad[0] else None
        gFbar = gF if ctx.needs_input_grad[1] else None
        return gtheta, gFbar, None, None, None, None


def hrom_pbar(plan: B.Plan, theta: torch.Tensor, Fbar: torch.Tensor, a0=None, tol=1e-10,
              max_it=25):
    """Differentiable converged (Pbar, Cbar, a, status) of every macro point.

    theta: [4] float64 CUDA tensor; Fbar: [9, N] float64 CUDA tensor
    (component-major); a0: optional starting amplitudes (mode-indexed 1-D
    layout of the plan).  Gradients flow to theta and Fbar through Pbar only.
    """
    return _HromPbar.apply(theta, Fbar, plan, a0, float(tol), int(max_it))
