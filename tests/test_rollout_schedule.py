"""The checkpointing schedule of the differentiable rollout, on the CPU.

The dynamic programme is pinned to Griewank's closed form for binomial
checkpointing (Griewank 1992; Griewank and Walther 2000): with c checkpoints
(the initial state's included) and m steps to reverse, the fewest forward
steps is  r m - C(c + r, r - 1),  r being the smallest integer with
C(c + r, r) >= m.  The reversal itself is checked on a stand-in plan (a small
nonlinear map with a hand-written adjoint), against torch autograd through
the same map, for every checkpoint count; the stand-in also counts the
forward steps the backward pass recomputes."""
from math import comb

import numpy as np
import pytest
import torch

from paper_2306_09760_amd import rollout as R


def griewank_min_steps(m, c):
    r = 0
    while comb(c + r, r) < m:
        r += 1
    return r * m - comb(c + r, r - 1) if r > 0 else 0


@pytest.mark.parametrize("s", [0, 1, 2, 3, 5, 8])
def test_dp_cost_equals_binomial_closed_form(s):
    nmax = 120
    cost, _ = R._tables(nmax, s)
    for m in range(1, nmax + 1):
        assert cost[s, m] == griewank_min_steps(m, s + 1), (m, s)


def test_split_realises_cost():
    cost, split = R._tables(60, 4)

    def walk(m, s):
        if m == 1:
            return 0
        if s == 0:
            return m * (m - 1) // 2
        j = int(split[s, m])
        assert 1 <= j < m
        return j + walk(m - j, s - 1) + walk(j, s)

    for s in range(5):
        for m in range(1, 61):
            assert walk(m, s) == cost[s, m]


def test_checkpoint_positions():
    assert R.checkpoint_positions(1, 5) == [0]
    assert R.checkpoint_positions(10, 9) == list(range(10))   # every state kept
    assert R.checkpoint_positions(10, 0) == [0]
    pos = R.checkpoint_positions(100, 4)
    assert len(pos) == 5 and pos == sorted(set(pos)) and pos[-1] < 100


class ToyPlan:
    """U <- U + dt tanh(M U) applied in place; its exact adjoint."""

    def __init__(self, n, seed=0):
        g = np.random.default_rng(seed)
        self.M = torch.from_numpy(g.standard_normal((n, n)) / np.sqrt(n))
        self.forward_steps = 0
        self.adjoint_states = []

    def rk3_step(self, U, dt=None):
        U += dt * torch.tanh(self.M @ U)
        self.forward_steps += 1
        return U

    def rk3_step_adjoint(self, Un, lam, dt):
        self.adjoint_states.append(Un.clone())
        t = torch.tanh(self.M @ Un)
        lam += dt * (self.M.T @ ((1 - t * t) * lam))
        return lam


@pytest.mark.parametrize("nsteps", [1, 2, 7, 30])
@pytest.mark.parametrize("snapshots", [0, 1, 2, 4, 100])
def test_rollout_gradient_and_recompute_count(nsteps, snapshots):
    n = 12
    P = ToyPlan(n)
    dt = torch.tensor([0.1], dtype=torch.float64)
    g = np.random.default_rng(1)
    U0 = torch.from_numpy(g.standard_normal(n)).requires_grad_(True)
    w = torch.from_numpy(g.standard_normal(n))
    UT = R.rollout(P, U0, dt, nsteps, snapshots)
    assert P.forward_steps == nsteps
    (UT * w).sum().backward()
    recomputed = P.forward_steps - nsteps
    assert recomputed == R.schedule_cost(nsteps, snapshots)
    # the adjoint steps saw U_{n-1}, ..., U_0 in that order
    states = [U0.detach().clone()]
    for _ in range(nsteps):
        states.append(states[-1] + 0.1 * torch.tanh(P.M @ states[-1]))
    assert len(P.adjoint_states) == nsteps
    for k, S in enumerate(P.adjoint_states):
        assert torch.equal(S, states[nsteps - 1 - k])
    # gradient against autograd through the same map
    V = U0.detach().clone().requires_grad_(True)
    X = V
    for _ in range(nsteps):
        X = X + 0.1 * torch.tanh(P.M @ X)
    (X * w).sum().backward()
    assert torch.allclose(U0.grad, V.grad, rtol=1e-13, atol=1e-14)


def test_rollout_recompute_budget():
    # 100 steps: storing 9 states besides U0 costs at most two recomputed
    # steps per step; storing all costs none
    assert R.schedule_cost(100, 99) == 0
    assert R.schedule_cost(100, 9) <= 2 * 100
    assert R.schedule_cost(100, 0) == 100 * 99 // 2
