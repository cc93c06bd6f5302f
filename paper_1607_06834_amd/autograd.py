"""Reverse-mode differentiation of ROK trajectories through librok.

`rok_trajectory(rok, y0, h, tableau, M, nsteps)` advances y0 by nsteps ROK
steps with exact (tangent) Jacobian-vector products and returns y_K as a
tensor that torch can differentiate: the backward pass runs the discrete
adjoint of every step (rok_step_vjp) in reverse order.

Checkpointing (default): the forward keeps the states y_n with n a multiple of
`checkpoint_every` (all of them by default).  The backward walks the
segments from last to first; each segment's intermediate states are
recomputed from its checkpoint with rok_step, and every rok_step_vjp call
recomputes the step's Krylov basis and stages from y_n itself.  Memory is
therefore about (nsteps / checkpoint_every + checkpoint_every) state vectors
plus one step's workspace.  With store_forward=True every step keeps its
state and forward workspace instead, and the backward runs only the reverse
sweeps (rok_step_vjp_stored): the HBM of one GPU holds hundreds of steps at
512^2.
"""
from __future__ import annotations

import torch

from .rok import Rok


class _RokTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, rok: Rok, h: float, tableau: dict, M: int, nsteps: int, every: int):
        y = y0.detach().contiguous()
        checkpoints = {0: y.clone()}
        if nsteps == 0:
            y = y.clone()   # the identity map: a tensor of its own, not a view of the input
        for n in range(nsteps):
            y = rok.step(y, h, tableau, M, mode="tangent")
            if (n + 1) % every == 0 and n + 1 < nsteps:
                checkpoints[n + 1] = y.clone()
        ctx.rok, ctx.h, ctx.tableau, ctx.M, ctx.nsteps, ctx.every = rok, h, tableau, M, nsteps, every
        ctx.checkpoints = checkpoints
        return y

    @staticmethod
    def backward(ctx, gout):
        rok, h, tab, M, every = ctx.rok, ctx.h, ctx.tableau, ctx.M, ctx.every
        g = gout.detach().contiguous().clone()
        nxt = torch.empty_like(g)
        starts = sorted(ctx.checkpoints, reverse=True)
        end = ctx.nsteps
        for s0 in starts:
            if s0 >= end:   # no step in this segment (nsteps = 0): the identity
                continue
            states = [ctx.checkpoints[s0]]
            for _ in range(s0, end - 1):   # recompute y_{s0+1} .. y_{end-1}
                states.append(rok.step(states[-1], h, tab, M, mode="tangent"))
            for y in reversed(states):
                rok.step_vjp(y, g, h, tab, M, out=nxt)
                g, nxt = nxt, g
            end = s0
        ctx.checkpoints = None
        return g, None, None, None, None, None, None


class _RokTrajectoryStored(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, rok: Rok, h: float, tableau: dict, M: int, nsteps: int):
        y = y0.detach().contiguous().clone()
        recs = []
        for _ in range(nsteps):
            y1, rec = rok.step_keep(y, h, tableau, M)
            recs.append(rec)
            y = y1
        ctx.rok, ctx.recs = rok, recs
        return y

    @staticmethod
    def backward(ctx, gout):
        g = gout.detach().contiguous().clone()
        nxt = torch.empty_like(g)
        for rec in reversed(ctx.recs):
            ctx.rok.step_vjp_stored(rec, g, out=nxt)
            g, nxt = nxt, g
        ctx.recs = None
        return g, None, None, None, None, None


def rok_trajectory(rok: Rok, y0: torch.Tensor, h: float, tableau: dict, M: int, nsteps: int,
                   checkpoint_every: int | None = None, store_forward: bool = False) -> torch.Tensor:
    """y_K after nsteps exact-product ROK steps, differentiable with respect to y0.

    store_forward=True keeps every step's state and forward workspace (about
    M + 2 s + 1 state vectors per step) and reverses the steps from them
    (Rok.step_vjp_stored) instead of recomputing: same bits, less time, more
    memory.  Otherwise states are checkpointed every `checkpoint_every` steps.
    """
    if int(nsteps) < 0:
        raise ValueError("nsteps must be >= 0")
    if store_forward:
        return _RokTrajectoryStored.apply(y0, rok, float(h), tableau, int(M), int(nsteps))
    every = 1 if checkpoint_every is None else int(checkpoint_every)
    if every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    return _RokTrajectory.apply(y0, rok, float(h), tableau, int(M), int(nsteps), every)


def rok_step_fn(rok: Rok, y: torch.Tensor, h: float, tableau: dict, M: int) -> torch.Tensor:
    """One exact-product ROK step, differentiable with respect to y."""
    return _RokTrajectory.apply(y, rok, float(h), tableau, int(M), 1, 1)
