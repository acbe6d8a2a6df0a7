"""torch.autograd wrapper of the solver: forward = fmm_eval, backward = one of
the library's adjoint calls, which rebuild the octree and every expansion
from the saved inputs instead of storing them.

E, F and phi are differentiable; dV/dlambda is returned as a
non-differentiable output.  For an upstream weight w on E alone,
fmm_eval_adjoint returns
    dE/dx = -w F,  dE/dqA = w (1 - lambda_s) phi,  dE/dqB = w lambda_s phi,
    dE/dlambda = w dV/dlambda
(sites -1: dE/dqA = w phi, dE/dqB = 0); with weights on phi or F as well,
fmm_eval_adjoint_full returns the gradient of w E + gphi . phi + gF . F in one
tree pass (charges and, as second sources, charges gphi with dipoles -q gF).
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
        ctx.mark_non_differentiable(out["dVdl"])
        return out["E"], out["F"], out["phi"], out["dVdl"]

    @staticmethod
    def backward(ctx, gE, gF, gphi, gdVdl):
        if gdVdl is not None and bool(torch.any(gdVdl != 0)):
            raise NotImplementedError("dV/dlambda is not differentiable; got a gradient on it")
        x, qA, qB, lam, site = ctx.saved_tensors
        w = (gE if gE is not None else torch.zeros(1, device=x.device)).to(torch.float64)
        w = w.reshape(1).contiguous()
        use_phi = gphi is not None and bool(torch.any(gphi != 0))
        use_F = gF is not None and bool(torch.any(gF != 0))
        if use_phi or use_F:
            adj = ctx.plan.eval_adjoint_full(
                x, qA, qB, site, lam, gE=w,
                gphi=gphi.to(x.dtype).contiguous() if use_phi else None,
                gF=gF.to(x.dtype).contiguous() if use_F else None, box=ctx.box)
        else:
            adj = ctx.plan.eval_adjoint(x, qA, qB, site, lam, w, box=ctx.box)
        return (adj["grad_x"] if ctx.needs_input_grad[0] else None,
                adj["grad_qA"] if ctx.needs_input_grad[1] else None,
                adj["grad_qB"] if ctx.needs_input_grad[2] else None,
                adj["grad_lambda"] if ctx.needs_input_grad[3] else None,
                None, None, None)


def fmm_coulomb(plan, x, qA, qB, site, lam, box=None):
    """Differentiable energy, forces and potential (and non-differentiable
    dV/dlambda)."""
    E, F, phi, dVdl = FmmCoulomb.apply(x, qA, qB, lam, plan, site, box)
    return E, F, phi, dVdl
