"""Differentiable SSP-RK3 rollout with binomial (revolve-type) checkpointing.

``rollout(plan, U0, dt, nsteps, snapshots)`` advances ``U0`` by ``nsteps``
SSP-RK3 steps of fixed size ``dt`` through the HIP library and returns the
final state as a tensor that autograd can differentiate: the backward pass
runs the library's discrete adjoint of one step (``wcns_rk3_step_adjoint``)
from the last step to the first.  The adjoint step needs the state at the
start of its step; those states come from at most ``snapshots`` stored
checkpoints plus recomputation, scheduled so that the number of recomputed
steps is the smallest possible for that many checkpoints (binomial
checkpointing, Griewank 1992; Griewank and Walther, ACM TOMS 26 (2000),
"Algorithm 799: revolve").

The schedule is computed by dynamic programming over

    cost(m, s) = min over 1 <= j < m of  j + cost(m - j, s - 1) + cost(j, s),
    cost(1, s) = 0,   cost(m, 0) = m (m - 1) / 2,

the number of forward steps needed to reverse m steps when the state at
their start is held and s further checkpoints are free: advance j steps,
keep that state in a free checkpoint, reverse the last m - j steps with one
checkpoint fewer, release it, then reverse the first j steps.  The first
chain of "advance and keep" moves is exactly the forward pass, so the
forward pass stores those states and the backward pass starts from them.

With ``stages=True`` the forward pass keeps every step's start state and
both stage states (``wcns_rk3_step_stages``, three states per step) and the
backward pass reverses each step from them (``wcns_rk3_step_adjoint_stages``)
without any recomputation: memory traded for the two residual evaluations
per step that the adjoint step otherwise repeats.

dt is held fixed (a CFL-limited dt depends on the state, and its derivative
is not part of the step adjoint).  Every step runs on the GPU; this module
only orders the calls.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
import torch

from .solver import Plan


@lru_cache(maxsize=64)
def _tables(m_max: int, s_max: int):
    """cost[s][m] and split[s][m] for 1 <= m <= m_max, 0 <= s <= s_max."""
    cost = np.zeros((s_max + 1, m_max + 1), dtype=np.int64)
    split = np.zeros((s_max + 1, m_max + 1), dtype=np.int64)
    m = np.arange(m_max + 1, dtype=np.int64)
    cost[0] = m * (m - 1) // 2
    cost[0, 0] = 0
    split[0, 2:] = m[2:] - 1
    for s in range(1, s_max + 1):
        for mm in range(2, m_max + 1):
            j = np.arange(1, mm)
            c = j + cost[s - 1, mm - j] + cost[s, j]
            k = int(np.argmin(c))
            cost[s, mm] = c[k]
            split[s, mm] = j[k]
    return cost, split


def schedule_cost(nsteps: int, snapshots: int) -> int:
    """Forward steps recomputed by the backward pass (the forward pass itself,
    nsteps steps, not included) when ``snapshots`` checkpoints besides the
    initial state are available."""
    if nsteps <= 1:
        return 0
    s = min(snapshots, nsteps - 1)
    cost, split = _tables(nsteps, s)
    # the first chain of advances is done by the forward pass
    first = 0
    lo, m, ss = 0, nsteps, s
    while m > 1 and ss > 0:
        j = int(split[ss, m])
        first += j
        lo, m, ss = lo + j, m - j, ss - 1
    return int(cost[s, nsteps]) - first


def checkpoint_positions(nsteps: int, snapshots: int):
    """Step indices whose states the forward pass keeps (0 always)."""
    pos = [0]
    if nsteps <= 1:
        return pos
    s = min(snapshots, nsteps - 1)
    _, split = _tables(nsteps, s)
    lo, m, ss = 0, nsteps, s
    while m > 1 and ss > 0:
        j = int(split[ss, m])
        lo, m, ss = lo + j, m - j, ss - 1
        pos.append(lo)
    return pos


class _StagedRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, plan, dt, nsteps):
        U = U0.detach().clone()
        saved = []
        for _ in range(nsteps):
            Un = U.clone()
            U1, U2 = torch.empty_like(U), torch.empty_like(U)
            plan.rk3_step_stages(U, U1, U2, dt=dt)
            saved.append((Un, U1, U2))
        ctx.plan, ctx.dt, ctx.saved = plan, dt, saved
        return U

    @staticmethod
    def backward(ctx, gU):
        lam = gU.detach().clone().contiguous()
        for Un, U1, U2 in reversed(ctx.saved):
            ctx.plan.rk3_step_adjoint(Un, lam, ctx.dt, stages=(U1, U2))
        ctx.saved = None
        return lam, None, None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, plan, dt, nsteps, snapshots):
        s = max(0, min(int(snapshots), max(nsteps - 1, 0)))
        keep = set(checkpoint_positions(nsteps, s))
        snaps = {0: U0.detach().clone()}
        U = U0.detach().clone()
        for k in range(nsteps):
            plan.rk3_step(U, dt=dt)
            if k + 1 in keep and k + 1 < nsteps:
                snaps[k + 1] = U.clone()
        ctx.plan, ctx.dt, ctx.nsteps, ctx.s = plan, dt, nsteps, s
        ctx.snaps = snaps
        return U

    @staticmethod
    def backward(ctx, gU):
        plan, dt, n, s = ctx.plan, ctx.dt, ctx.nsteps, ctx.s
        snaps = ctx.snaps
        lam = gU.detach().clone().contiguous()
        if n == 0:
            return lam, None, None, None, None
        _, split = _tables(n, s)

        def advance(U, j):
            U = U.clone()
            for _ in range(j):
                plan.rk3_step(U, dt=dt)
            return U

        def reverse(lo, hi, ss, first):
            m = hi - lo
            if m == 1:
                plan.rk3_step_adjoint(snaps[lo], lam, dt)
                return
            if ss == 0:
                for k in range(hi - 1, lo, -1):
                    plan.rk3_step_adjoint(advance(snaps[lo], k - lo), lam, dt)
                plan.rk3_step_adjoint(snaps[lo], lam, dt)
                return
            j = int(split[ss, m])
            mid = lo + j
            if not first:
                snaps[mid] = advance(snaps[lo], j)
            reverse(mid, hi, ss - 1, first)
            del snaps[mid]
            reverse(lo, mid, ss, False)

        reverse(0, n, s, True)
        ctx.snaps = None
        return lam, None, None, None, None


def rollout(plan, U0: torch.Tensor, dt: torch.Tensor, nsteps: int, snapshots: int = 8,
            stages: bool = False):
    """U(T) after ``nsteps`` SSP-RK3 steps of size ``dt`` (a (1,) device
    tensor); differentiable with respect to ``U0``.  ``snapshots`` bounds
    the number of stored states besides ``U0``; snapshots >= nsteps - 1
    stores every state, and the backward pass then recomputes no step but
    still each step's two stage states.  ``stages=True`` stores those too
    (3 nsteps states; ``snapshots`` is then ignored)."""
    if nsteps < 0:
        raise ValueError("nsteps must be >= 0")
    if isinstance(plan, Plan):  # the library's plans check what reaches the kernels
        plan._check_state(U0)
        plan._dt(dt, optional=False)
    if stages:
        return _StagedRollout.apply(U0, plan, dt, int(nsteps))
    return _Rollout.apply(U0, plan, dt, int(nsteps), int(snapshots))
