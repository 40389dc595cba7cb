"""Gradient oracle: reverse-mode derivatives of the FP64 step by torch autograd.

Test infrastructure, like the rest of `oracle/`.

The paper differentiates through the solver with PyTorch's automatic
differentiation (Sec. 3.2).  This module does exactly that on the CPU oracle of
`oracle.lbm`, in FP64, keeping the whole graph.  It is the reference for the
hand-written adjoint kernels: `step_vjp` for one adjoint step, `moments_vjp` for
the terminal moments adjoint, `rollout_grad` for a whole differentiated rollout.
"""
from __future__ import annotations

import torch

from . import lbm


def step_vjp(g: torch.Tensor, lam_next: torch.Tensor, tau: float, st: lbm.Stencil,
             force: torch.Tensor | None = None):
    """Vector-Jacobian product of one pull step g' = C(S g; F).

    Returns (lambda, dF): lambda = (dg'/dg)^T lam_next and dF = (dg'/dF)^T lam_next
    (dF is None without a force).
    """
    g = g.detach().to(torch.float64).requires_grad_(True)
    inputs = [g]
    F = None
    if force is not None:
        F = force.detach().to(torch.float64).requires_grad_(True)
        inputs.append(F)
    out = lbm.step(g, tau, st, F)
    grads = torch.autograd.grad(out, inputs, grad_outputs=lam_next.to(torch.float64))
    return grads[0], (grads[1] if force is not None else None)


def moments_vjp(g: torch.Tensor, st: lbm.Stencil, force: torch.Tensor | None,
                dL_drho: torch.Tensor | None, dL_du: torch.Tensor | None):
    """VJP of `lbm.state_moments`: returns (dL/dg, dL/dF or None)."""
    g = g.detach().to(torch.float64).requires_grad_(True)
    inputs = [g]
    F = None
    if force is not None:
        F = force.detach().to(torch.float64).requires_grad_(True)
        inputs.append(F)
    rho, u = lbm.state_moments(g, st, F)
    outs, cots = [], []
    if dL_drho is not None:
        outs.append(rho)
        cots.append(dL_drho.to(torch.float64))
    if dL_du is not None:
        outs.append(u)
        cots.append(dL_du.to(torch.float64))
    grads = torch.autograd.grad(outs, inputs, grad_outputs=cots, allow_unused=True)
    dg = grads[0] if grads[0] is not None else torch.zeros_like(g)
    dF = None
    if force is not None:
        dF = grads[1] if grads[1] is not None else torch.zeros_like(F)
    return dg, dF


def rollout_grad(g0: torch.Tensor, force: torch.Tensor | None, tau: float, st: lbm.Stencil,
                 n_steps: int, loss_fn):
    """Loss L = loss_fn(rho(T), u(T)) after n_steps pull steps from g0 with a constant
    force field, and its gradients (L, dL/dg0, dL/dF or None), by autograd through
    every step."""
    g0 = g0.detach().to(torch.float64).requires_grad_(True)
    inputs = [g0]
    F = None
    if force is not None:
        F = force.detach().to(torch.float64).requires_grad_(True)
        inputs.append(F)
    g = g0
    for _ in range(n_steps):
        g = lbm.step(g, tau, st, F)
    rho, u = lbm.state_moments(g, st, F)
    L = loss_fn(rho, u)
    grads = torch.autograd.grad(L, inputs)
    return L.detach(), grads[0], (grads[1] if force is not None else None)
