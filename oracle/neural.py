"""Neural collision model of Sec. 3.1 (oracle side): the MRT collision of Eq. 5 whose
ghost-moment relaxation times tau_6, tau_7, tau_8 come from a shallow network
evaluated per cell and step.

Test infrastructure, like the rest of `oracle/`.

What the paper fixes: D2Q9 with Dellar's moment basis; tau_0..2 have no effect,
tau_3..5 = nu/c_s^2 + 1/2 (the shear times); a network with one hidden layer and 530
parameters maps local moments to outputs t_n, and tau_n = exp(t_n) + 1/2 for
n = 6, 7, 8 (so every ghost time exceeds 1/2).

Readings (the paper names neither the inputs nor the activation, and prints no
weights):
  * inputs: the six non-conserved moments of the cell's non-equilibrium part,
    x = M[3:9] (h - f^eq(rho, u)), i.e. (Pi_xx, Pi_xy, Pi_yy, N, J_x, J_y) of
    h - f^eq with the rows c_x^2, c_x c_y, c_y^2, g, g c_x, g c_y of `dellar_matrix`;
    they vanish at equilibrium and do not see the conserved moments;
  * layout: 6 inputs, 53 hidden units with a bias, 3 outputs without a bias:
    6*53 + 53 + 53*3 = 530 parameters, the paper's count;
  * activation: ReLU or tanh (both are provided).
Parameter vector order: W1 [53][6] row-major, b1 [53], W2 [3][53] row-major.
"""
from __future__ import annotations

import torch

from . import lbm

N_IN = 6
N_HIDDEN = 53
N_OUT = 3
N_PARAMS = N_IN * N_HIDDEN + N_HIDDEN + N_OUT * N_HIDDEN  # 530
ACTIVATIONS = ("relu", "tanh")

F64 = torch.float64


def split(params: torch.Tensor):
    """The parameter vector as (W1 [53, 6], b1 [53], W2 [3, 53]), float64."""
    p = params.to(F64).reshape(-1)
    if p.numel() != N_PARAMS:
        raise ValueError(f"the network has {N_PARAMS} parameters, got {p.numel()}")
    a = N_IN * N_HIDDEN
    W1 = p[:a].reshape(N_HIDDEN, N_IN)
    b1 = p[a:a + N_HIDDEN]
    W2 = p[a + N_HIDDEN:].reshape(N_OUT, N_HIDDEN)
    return W1, b1, W2


def inputs(h: torch.Tensor, st: lbm.Stencil) -> torch.Tensor:
    """The six non-conserved Dellar moments of h - f^eq(rho, u): [6, *spatial]."""
    rho = lbm.density(h)
    feq = lbm.equilibrium(rho, lbm.momentum(h, st) / rho, st)
    M = lbm.dellar_matrix(st)
    return torch.einsum("kq,q...->k...", M[3:], h - feq)


def _act(z: torch.Tensor, activation: str) -> torch.Tensor:
    if activation == "relu":
        return torch.clamp(z, min=0.0)
    if activation == "tanh":
        return torch.tanh(z)
    raise ValueError(f"unknown activation {activation!r}")


def ghost_taus(h: torch.Tensor, params: torch.Tensor, activation: str, st: lbm.Stencil) -> torch.Tensor:
    """tau_6, tau_7, tau_8 of every cell: exp(W2 act(W1 x + b1)) + 1/2, [3, *spatial]."""
    W1, b1, W2 = split(params)
    x = inputs(h, st)
    nd = x.dim() - 1
    hidden = _act(torch.einsum("jk,k...->j...", W1, x) + b1.reshape((N_HIDDEN,) + (1,) * nd), activation)
    t = torch.einsum("nj,j...->n...", W2, hidden)
    return torch.exp(t) + 0.5


def collide(h: torch.Tensor, tau_shear: float, params: torch.Tensor, activation: str,
            st: lbm.Stencil) -> torch.Tensor:
    """Eq. 5 with S = diag(1, 1, 1, tau_s, tau_s, tau_s, tau_6, tau_7, tau_8), the ghost
    times from the network."""
    tg = ghost_taus(h, params, activation, st)
    taus = [1.0, 1.0, 1.0, tau_shear, tau_shear, tau_shear, tg[0], tg[1], tg[2]]
    return lbm.mrt_collide(h, taus, st)


def step(g: torch.Tensor, tau_shear: float, params: torch.Tensor, activation: str,
         st: lbm.Stencil) -> torch.Tensor:
    """Pull-convention step with the neural collision: C(S g)."""
    return collide(lbm.stream(g, st), tau_shear, params, activation, st)
