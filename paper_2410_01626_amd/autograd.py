"""torch.autograd wrapper of the solver: forward = fmm_eval, backward =
fmm_eval_adjoint, which rebuilds the octree and every expansion from the
saved inputs instead of storing them.

The energy E and the potential phi are differentiable.  F and dV/dlambda are
returned as non-differentiable outputs: an upstream gradient on F would need
a Hessian-vector pass with dipole sources that this library does not provide.
For an upstream weight w on E alone the hand-written adjoint returns
    dE/dx = -w F,  dE/dqA = w (1 - lambda_s) phi,  dE/dqB = w lambda_s phi,
    dE/dlambda = w dV/dlambda
(sites -1: dE/dqA = w phi, dE/dqB = 0); with weights g on phi as well,
fmm_eval_adjoint_phi (three solves) returns the gradient of w E + g . phi.
"""
from __future__ import annotations

import torch


class FmmCoulomb(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, qA, qB, lam, plan, site, box):
        out = plan.eval(x, qA, qB, site, lam, box=box)
        ctx.save_for_backward(x, qA, qB, lam, site)
        ctx.plan = plan
        ctx.box = box
        ctx.mark_non_differentiable(out["F"], out["dVdl"])
        return out["E"], out["F"], out["phi"], out["dVdl"]

    @staticmethod
    def backward(ctx, gE, gF, gphi, gdVdl):
        for g, name in ((gF, "F"), (gdVdl, "dVdl")):
            if g is not None and bool(torch.any(g != 0)):
                raise NotImplementedError(
                    "only the energy and the potential are differentiable; got a gradient on %s"
                    % name)
        x, qA, qB, lam, site = ctx.saved_tensors
        if gphi is not None and bool(torch.any(gphi != 0)):
            w = 0.0 if gE is None else float(gE.reshape(-1)[0].item())
            adj = ctx.plan.eval_adjoint_phi(x, qA, qB, site, lam, w,
                                            gphi.to(x.dtype).contiguous(), box=ctx.box)
        else:
            w = (gE if gE is not None else torch.zeros(1, device=x.device)).to(torch.float64)
            adj = ctx.plan.eval_adjoint(x, qA, qB, site, lam, w.reshape(1).contiguous(), box=ctx.box)
        return (adj["grad_x"] if ctx.needs_input_grad[0] else None,
                adj["grad_qA"] if ctx.needs_input_grad[1] else None,
                adj["grad_qB"] if ctx.needs_input_grad[2] else None,
                adj["grad_lambda"] if ctx.needs_input_grad[3] else None,
                None, None, None)


def fmm_coulomb(plan, x, qA, qB, site, lam, box=None):
    """Differentiable energy and potential (and non-differentiable F, dV/dlambda)."""
    E, F, phi, dVdl = FmmCoulomb.apply(x, qA, qB, lam, plan, site, box)
    return E, F, phi, dVdl
