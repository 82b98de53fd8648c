"""torch.autograd.Function over the hand-written adjoint: the period-averaged eddy-current
loss of the periodic steady state as a differentiable function of the element
conductivities and the Brauer constants (k1, k2, k3) of every material.

forward: copy the design with the given parameters to the device (the library copies a
design's materials at creation, so new parameters mean a new problem), solve its periodic
steady state by PP-PC and evaluate the loss; when a gradient will be asked for, the same
ppc_adjoint call runs the adjoint iteration for it, otherwise it stops after the loss;
backward: scale the stored gradient.  All arithmetic runs in the HIP library."""
from __future__ import annotations

import copy

import numpy as np
import torch

from .ppc import Problem


def _design(prob, sigma, brauer):
    q = copy.copy(prob)
    q.sigma = sigma.detach().cpu().numpy().astype(np.float64)
    par = np.array(prob.mat_par, dtype=np.float64, copy=True)
    br = brauer.detach().cpu().numpy().astype(np.float64)
    for mid in range(len(prob.mat_model)):
        if int(prob.mat_model[mid]) == 1:
            par[mid, 1:4] = br[mid]
    q.mat_par = par
    return q


class PeriodicEddyLoss(torch.autograd.Function):
    """loss = PeriodicEddyLoss.apply(sigma [n_tri], brauer [n_mat, 3], prob, params, handle)"""

    @staticmethod
    def forward(ctx, sigma, brauer, prob, prm, handle):
        q = _design(prob, sigma, brauer)
        pr = Problem(handle, q)
        try:
            U, eps, k, st, rc = pr.solve(prm)
            if rc != 0:
                raise RuntimeError(f"periodic solve did not converge (status {rc})")
            grads = bool(ctx.needs_input_grad[0] or ctx.needs_input_grad[1])
            loss, dsig, dk, kadj, _ = pr.adjoint(prm, U, len(prob.mat_model), grads=grads)
        finally:
            pr.close()
        if grads:
            ctx.save_for_backward(torch.as_tensor(dsig, dtype=sigma.dtype, device=sigma.device),
                                  torch.as_tensor(dk, dtype=brauer.dtype, device=brauer.device))
        return torch.as_tensor(loss, dtype=sigma.dtype, device=sigma.device)

    @staticmethod
    def backward(ctx, g):
        dsig, dk = ctx.saved_tensors
        return g * dsig, g * dk, None, None, None


def periodic_eddy_loss(sigma, brauer, prob, prm, handle):
    return PeriodicEddyLoss.apply(sigma, brauer, prob, prm, handle)
