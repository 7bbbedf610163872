"""Differentiable rollout of the explicit IP+IBM step (FP64 plans).

``rollout(plan, X0, u, kmat, ...)`` runs ``steps`` calls of ``ip_step`` and is
a ``torch.autograd.Function``: its backward walks the steps in reverse with
``ip_step_vjp``, from positions checkpointed before every step (one N x 3
FP64 copy per step, 24 bytes per node per step).  Gradients flow to the
initial positions X0, the MAC velocity u and the per-body constants
kmat[4, B] = (ks, kb, kA, kV), which parametrise the interaction potentials
of Section 2.3.  ``taylor_loss`` is the squared distance of each body's Taylor
deformation (Section 3.1) to a target, with its gradient from ``ip_taylor``.

Every step of both directions runs in the HIP library; this module only
marshals arguments.
"""
from __future__ import annotations

import torch

from . import native as N


def _constants(kmat, mass):
    return N.Constants(kmat[0].contiguous(), kmat[1].contiguous(), kmat[2].contiguous(),
                       kmat[3].contiguous(), mass)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X0, u, kmat, plan, ref, mass, dt, steps):
        if plan.precision != "f64":
            raise N.IpibmError(N.IP_ERR_UNSUPPORTED, "the differentiable rollout needs an f64 plan")
        k = _constants(kmat.detach(), mass)
        X = X0.detach().contiguous().clone()
        u = u.detach().contiguous()
        f = torch.zeros_like(u)          # the spread forcing is not part of the loss here
        checkpoints = []
        for _ in range(steps):
            checkpoints.append(X.clone())
            N.ip_step(plan, X, ref, k, u, f, dt)
        ctx.plan, ctx.ref, ctx.k, ctx.dt = plan, ref, k, dt
        ctx.checkpoints, ctx.u = checkpoints, u
        ctx.B = kmat.shape[1]
        return X

    @staticmethod
    def backward(ctx, gX):
        lam = gX.detach().contiguous().clone()
        gk = torch.zeros(4, ctx.B, dtype=torch.float64, device=lam.device)
        gu = torch.zeros_like(ctx.u)
        for Xn in reversed(ctx.checkpoints):
            N.ip_step_vjp(ctx.plan, Xn, ctx.ref, ctx.k, ctx.u, ctx.dt, lam, lam, gk, gu)
        ctx.checkpoints = None
        return lam, gu, gk, None, None, None, None, None


def rollout(plan, X0, u, kmat, ref, mass, dt, steps):
    """Positions after ``steps`` explicit steps from X0 (differentiable in X0,
    u and kmat)."""
    return _Rollout.apply(X0, u, kmat, plan, ref, mass, dt, steps)


class _TaylorLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, Dstar, plan):
        D, loss, gX = N.ip_taylor(plan, X.detach().contiguous(), Dstar.detach().contiguous())
        ctx.save_for_backward(gX)
        return loss.sum()

    @staticmethod
    def backward(ctx, g):
        (gX,) = ctx.saved_tensors
        return g * gX, None, None


def taylor_loss(plan, X, Dstar):
    """sum_b (D_b(X) - Dstar_b)^2 (differentiable in X)."""
    return _TaylorLoss.apply(X, Dstar, plan)


def taylor(plan, X):
    """Taylor deformation D[B] of every body (no gradient)."""
    return N.ip_taylor(plan, X.detach().contiguous())
