"""torch.autograd.Function over the subcycle: forward se_subcycle, backward
se_subcycle_adjoint (checkpoint-and-recompute every ckpt_every substeps).

Differentiable inputs: eta0, U0, R, H0 (f and W are treated as constants).
Outputs: (eta^M, U^M, <<U>>); <<U>> is float64 in both precisions.
"""
from __future__ import annotations

import torch

from .api import Mesh, Params


class SubcycleFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta0, U0, R, H0, f, mesh: Mesh, params: Params, nsub: int, dt: float,
                ckpt_every: int = 5, W=None):
        eta = eta0.detach().clone()
        U = U0.detach().clone()
        Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device=eta0.device)
        mesh.subcycle(eta, U, R=R.detach(), f=f.detach(), H0=H0.detach(),
                      W=None if W is None else W.detach(), nsub=nsub, dt=dt, params=params,
                      Uavg=Uavg)
        ctx.save_for_backward(eta0.detach(), U0.detach(), R.detach(), H0.detach(), f.detach())
        ctx.W = None if W is None else W.detach()
        ctx.cfg = (mesh, params, nsub, dt, ckpt_every)
        return eta, U, Uavg

    @staticmethod
    def backward(ctx, g_eta, g_U, g_Uavg):
        eta0, U0, R, H0, f = ctx.saved_tensors
        mesh, params, nsub, dt, ckpt_every = ctx.cfg
        dt_ = params.dtype
        lam_eta = None if g_eta is None else g_eta.to(dt_).contiguous()
        lam_U = None if g_U is None else g_U.to(dt_).contiguous()
        lam_Ua = None if g_Uavg is None else g_Uavg.to(torch.float64).contiguous()
        ge, gU, gR, gH = mesh.adjoint(eta0, U0, R=R, f=f, H0=H0, W=ctx.W, nsub=nsub, dt=dt,
                                      params=params, ckpt_every=ckpt_every, lam_eta=lam_eta,
                                      lam_U=lam_U, lam_Uavg=lam_Ua)
        return ge, gU, gR, gH, None, None, None, None, None, None, None


def subcycle(eta0, U0, R, H0, f, mesh: Mesh, params: Params, nsub: int, dt: float,
             ckpt_every: int = 5, W=None):
    """Differentiable one baroclinic step: returns (eta^M, U^M, <<U>>)."""
    return SubcycleFn.apply(eta0, U0, R, H0, f, mesh, params, nsub, dt, ckpt_every, W)
