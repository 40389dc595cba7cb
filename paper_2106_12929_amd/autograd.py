"""torch.autograd wrappers of the hand-written adjoint kernels.

The paper differentiates its solver by PyTorch autograd through every tensor
operation (Sec. 3.2).  Here the derivative of a whole rollout comes from the
library's adjoint kernels instead:

  LBMRollout.apply(g0, force, grid, tau, n_steps, checkpoint_every[, pair_adjoint]) -> g_T
      forward: per segment of K steps, its first step, then the steps between in one
      lbm_step call (several steps per launch where the library can), then the K-th
      step, which writes into a fresh buffer kept as a checkpoint (no copies);
      backward: for each K-step segment, last to first, replay the segment from
      its checkpoint (keeping its K states), then run K adjoint steps backwards in
      the collision-local form (lbm_adjoint_step_local, aligned stores only; after
      the rollout's last step, two steps per lbm_adjoint_step2_local launch where the
      library takes the grid and pair_adjoint is set, bitwise the same) and finish
      with one lbm_adjoint_unstream; the force gradient accumulates in place in the
      kernels.
      Memory: ceil(n/K) checkpoints + K segment states + 2 adjoint buffers.
      Forward and adjoint kernels are deterministic (no atomics), so the gradient
      is bitwise independent of K.

  LBMMoments.apply(g, force, grid) -> (rho, u)
      forward: lbm_moments; backward: lbm_moments_adjoint.

The derivative is that of the exact-arithmetic step at the stored state: rounding
to a reduced-precision storage format is not differentiated.
"""
from __future__ import annotations

import torch

from . import binding as B


def _real(grid: B.Grid, t: torch.Tensor | None) -> torch.Tensor | None:
    if t is None:
        return None
    return t.detach().to(grid.real_dtype).contiguous()


class LBMRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g0, force, grid: B.Grid, tau: float, n_steps: int, checkpoint_every: int,
                pair_adjoint: bool = True):
        if n_steps < 1 or checkpoint_every < 1:
            raise ValueError("n_steps and checkpoint_every must be >= 1")
        F = _real(grid, force)
        cur = g0.detach().contiguous().clone()  # checkpoint 0 (the caller may change g0)
        ckpts = [cur]
        spare = [torch.empty_like(cur), torch.empty_like(cur)]
        K = checkpoint_every
        t = 0
        while t < n_steps:
            steps = min(K, n_steps - t)
            last_ckpt = t + steps < n_steps  # this segment ends in a new checkpoint
            # the segment's first step leaves the checkpoint it starts from untouched;
            # the steps between run in one lbm_step call on the two spare buffers (the
            # library takes several steps per launch there); the last step writes the
            # next checkpoint itself
            mid = steps - 1 - (1 if last_ckpt else 0)
            if steps - (1 if last_ckpt else 0) >= 1:
                B.lbm_step(grid, cur, spare[0], tau, F, 1)
                cur = spare[0]
            if mid >= 1:
                where = B.lbm_step(grid, spare[0], spare[1], tau, F, mid)
                cur = spare[1] if where == 0 else spare[0]
            if last_ckpt:
                dst = torch.empty_like(cur)
                ckpts.append(dst)
                B.lbm_step(grid, cur, dst, tau, F, 1)
                cur = dst
            t += steps
        a = cur
        ctx.grid, ctx.tau, ctx.n, ctx.K = grid, tau, n_steps, checkpoint_every
        ctx.pair = bool(pair_adjoint) and B.lbm_adjoint_step2_available(grid)
        ctx.ckpts = ckpts
        ctx.force = F
        ctx.force_needs_grad = force is not None and ctx.needs_input_grad[1]
        return a

    @staticmethod
    def backward(ctx, lam_T):
        grid, tau, n, K, F = ctx.grid, ctx.tau, ctx.n, ctx.K, ctx.force
        # Adjoint in collision-local form: chi_t = J_C(h_t)^T lam_{t+1} with
        # lam_{t+1} = S^T chi_{t+1}; every kernel store is aligned, and
        # lam_0 = S^T chi_0 at the end (bitwise what the scatter form gives).
        cur = lam_T.detach().to(grid.real_dtype).contiguous()
        # a pitched layout has pad words that the kernels never write and whose gradient
        # is zero: its adjoint buffers start zero-filled
        alloc = torch.zeros_like if grid.row_pitch != grid.nx else torch.empty_like
        bufs = [alloc(cur), alloc(cur)]
        is_chi = False
        dF = torch.zeros_like(F) if ctx.force_needs_grad else None
        n_seg = len(ctx.ckpts)
        # states[0] of a segment is its checkpoint itself (read only); the replay writes
        # the other K - 1 states
        states = [None] + [torch.empty_like(ctx.ckpts[0]) for _ in range(min(K, n) - 1)]
        k = 0
        for seg in reversed(range(n_seg)):
            t0 = seg * K
            t1 = min(t0 + K, n)
            states[0] = ctx.ckpts[seg]
            for t in range(t0 + 1, t1):
                B.lbm_step(grid, states[t - 1 - t0], states[t - t0], tau, F, 1)
            t = t1 - 1
            while t >= t0:
                out = bufs[k & 1]
                if ctx.pair and is_chi and t - 1 >= t0:
                    # steps t and t - 1 in one launch, chi_t kept on chip
                    B.lbm_adjoint_step2_local(grid, states[t - t0], states[t - 1 - t0], cur, out, tau, F, dF)
                    t -= 2
                else:
                    B.lbm_adjoint_step_local(grid, states[t - t0], cur, is_chi, out, tau, F, dF)
                    t -= 1
                cur, is_chi, k = out, True, k + 1
            ctx.ckpts[seg] = None  # released once the next segment replaces states[0]
        states = None
        lam0 = bufs[k & 1]
        B.lbm_adjoint_unstream(grid, cur, lam0)
        return lam0, dF, None, None, None, None, None


class LBMMoments(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, force, grid: B.Grid):
        F = _real(grid, force)
        gc = g.detach().contiguous()
        rho = grid.empty_real(0, g.device)
        u = grid.empty_real(grid.D, g.device)
        B.lbm_moments(grid, gc, F, rho, u)
        ctx.save_for_backward(gc)
        ctx.grid, ctx.force = grid, F
        ctx.force_needs_grad = force is not None and ctx.needs_input_grad[1]
        return rho, u

    @staticmethod
    def backward(ctx, drho, du):
        (g,) = ctx.saved_tensors
        grid, F = ctx.grid, ctx.force
        lam = torch.zeros(grid.population_shape(), dtype=grid.real_dtype, device=g.device)
        dF = torch.zeros_like(F) if ctx.force_needs_grad else None
        B.lbm_moments_adjoint(grid, g, F, _real(grid, drho), _real(grid, du), lam, dF)
        return lam, dF, None


def rollout(grid: B.Grid, g0: torch.Tensor, force: torch.Tensor | None, tau: float, n_steps: int,
            checkpoint_every: int = 10, pair_adjoint: bool = True) -> torch.Tensor:
    """Differentiable n-step rollout from g0 under a constant force field."""
    return LBMRollout.apply(g0, force, grid, tau, n_steps, checkpoint_every, pair_adjoint)


def moments(grid: B.Grid, g: torch.Tensor, force: torch.Tensor | None = None):
    """Differentiable (rho, u) of a state."""
    return LBMMoments.apply(g, force, grid)
