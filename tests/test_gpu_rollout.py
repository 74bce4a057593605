"""Gradient of a tracking loss through an SSP-RK3 rollout on the GPU.

J(rho0) = 1/2 || rho(T) - rho_target ||^2 on the 2D periodic Euler problem
with a smooth initial density rho0 (fixed dt from the initial state); the
control is the initial density, u, v and p held at their initial fields, so
a direction d rho changes the state by dU = (1, u, v, (u^2 + v^2) / 2) d rho.

The flow fields u, v, p carry a small smooth variation (amplitude 0.05).
With u = v = 0.5 and p = 1 exactly, the acoustic and shear characteristic
fields are uniform: their smoothness indicators are rounding noise (~1e-32,
far above eps = 1e-40), the exact derivative of the weights there is set by
that noise, and the tangent of the rollout grows about threefold per step in
those fields (the oracle's own JVP shows it), so no derivative check can pass
after a few dozen steps.  Resolving every field keeps the linearisation
meaningful.

The gradient from the checkpointed adjoint rollout is checked
  * against the oracle's exact dual-number JVPs of the same run (64^2,
    20 steps, and the reduced config-5 run at 128^2 and 100 steps, white-noise
    directions): <grad J, d> = sum (rho(T) - rho_target) d rho(T), to 1e-9
    or twice the spread between the two oracle builds (with and without FMA
    contraction), which must stay below 1e-7;
  * element by element: the whole gradient at 16^2 and 3 steps against 256
    oracle JVPs along the unit directions of the initial density;
  * at full size (1024^2, 100 steps) against central differences of the GPU
    forward along 32 seeded smooth Gaussian directions (random Fourier
    coefficients, |k| <= 4);
  * for independence from the checkpoint count (bitwise: recomputed states
    are the same kernels on the same inputs)."""
import numpy as np
import pytest
import torch

from gpu_util import SPREAD_CAP, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2306_09760_amd import rollout, solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return solver, rollout


GAMMA = 1.4
FLOW_AMP = 0.05


class Control:
    """U0(rho) = (rho, rho u, rho v, p / (gamma - 1) + rho (u^2 + v^2) / 2)
    with the workload's u, v, p fields; differentiable in rho."""

    def __init__(self, U0):
        rho = U0[0]
        self.u = U0[1] / rho
        self.v = U0[2] / rho
        self.p = (GAMMA - 1.0) * (U0[3] - 0.5 * rho * (self.u ** 2 + self.v ** 2))
        self.ke = 0.5 * (self.u ** 2 + self.v ** 2)

    def __call__(self, rho):
        return torch.stack([rho, rho * self.u, rho * self.v,
                            self.p / (GAMMA - 1.0) + rho * self.ke]).contiguous()

    def direction(self, drho):
        return torch.stack([drho, drho * self.u, drho * self.v, drho * self.ke])


def _setup(solver, W, n, seed=0):
    prob, U0, extra = W.adjoint2d(seed=seed, n=n, flow_amp=FLOW_AMP)
    G = solver.Plan(**prob, weights="fe", xi=100.0)
    ctl = Control(to_dev(U0))
    rho0 = to_dev(U0[0])
    dt = G.cfl_dt(ctl(rho0), 0.5).clone()
    target = to_dev(extra["target_init"])
    return prob, ctl, rho0, target, G, dt


def _loss_grad(G, roll, ctl, rho0, target_T, dt, nsteps, snapshots, stages=False):
    r = rho0.clone().requires_grad_(True)
    UT = roll.rollout(G, ctl(r), dt, nsteps, snapshots, stages=stages)
    J = 0.5 * ((UT[0] - target_T[0]) ** 2).sum()
    J.backward()
    return float(J.detach()), r.grad.detach()


def _jvp_check(mods, ora, W, n, nsteps, ndir, snapshots):
    """<grad J, d> from the checkpointed adjoint rollout against the
    oracle's dual-number JVP of the same run, on ndir white-noise
    directions."""
    solver, roll = mods
    prob, ctl, rho0, target0, G, dt = _setup(solver, W, n)
    say("rollout vs oracle jvp", n, nsteps)
    target = target0.clone()
    for _ in range(nsteps):
        G.rk3_step(target, dt=dt)
    _, grad = _loss_grad(G, roll, ctl, rho0, target, dt, nsteps, snapshots=snapshots)
    grad = to_host(grad)
    dth = float(to_host(dt)[0])
    U0 = to_host(ctl(rho0))
    O = ora.Problem(**prob, weights="fe", xi=100.0)
    Of = ora.Problem(**prob, weights="fe", xi=100.0, variant="fma")
    tgt, bad = O.run_steps(to_host(target0), nsteps, dt=dth)
    assert bad == 0
    rng = np.random.default_rng(11)
    for k in range(ndir):
        drho = rng.standard_normal(U0.shape[1:])
        V = to_host(ctl.direction(to_dev(drho)))
        dJ = []
        for P in (O, Of):
            U, dU = U0.copy(), V.copy()
            for _ in range(nsteps):
                U, dU, bad = P.rk3_step_jvp(U, dU, dth)
                assert bad == 0
            dJ.append(float(np.sum((U[0] - tgt[0]) * dU[0])))
        rhs = dJ[0]
        spread = abs(dJ[1] - dJ[0]) / abs(rhs)
        lhs = float(np.sum(grad * drho))
        say("  direction", k, lhs, rhs, "rel diff %.2e" % (abs(lhs - rhs) / abs(rhs)),
            "oracle fma spread %.2e" % spread)
        assert spread <= SPREAD_CAP, spread
        assert abs(lhs - rhs) <= max(1e-9, 2 * spread) * abs(rhs), (lhs, rhs, spread)


def test_rollout_gradient_matches_oracle_jvp(mods, ora, W):
    _jvp_check(mods, ora, W, 64, 20, 3, snapshots=3)


@pytest.mark.timeout(300)
def test_config5_reduced_gradient_matches_oracle_jvp(mods, ora, W):
    """The reduced config-5 run: 128^2, 100 steps, 9 checkpoints."""
    _jvp_check(mods, ora, W, 128, 100, 3, snapshots=9)


def test_full_gradient_by_oracle_jvps(mods, ora, W):
    """16^2, 3 steps: every component of the gradient with respect to the
    initial density against the oracle's JVP along that unit direction."""
    solver, roll = mods
    n, nsteps = 16, 3
    prob, ctl, rho0, target0, G, dt = _setup(solver, W, n)
    say("full gradient by 256 oracle jvps")
    target = target0.clone()
    for _ in range(nsteps):
        G.rk3_step(target, dt=dt)
    _, grad = _loss_grad(G, roll, ctl, rho0, target, dt, nsteps, snapshots=1)
    grad = to_host(grad).ravel()
    dth = float(to_host(dt)[0])
    U0 = to_host(ctl(rho0))
    O = ora.Problem(**prob, weights="fe", xi=100.0)
    tgt, bad = O.run_steps(to_host(target0), nsteps, dt=dth)
    ref = np.empty(n * n)
    for i in range(n * n):
        drho = np.zeros(n * n)
        drho[i] = 1.0
        V = to_host(ctl.direction(to_dev(drho.reshape(n, n))))
        U, dU = U0.copy(), V.copy()
        for _ in range(nsteps):
            U, dU, bad = O.rk3_step_jvp(U, dU, dth)
            assert bad == 0
        ref[i] = float(np.sum((U[0] - tgt[0]) * dU[0]))
    err = np.abs(grad - ref).max() / np.abs(ref).max()
    say("  max componentwise difference / max |grad|", err)
    assert err <= 1e-10, err


def test_rollout_gradient_independent_of_checkpoints(mods, W):
    solver, roll = mods
    prob, ctl, rho0, target, G, dt = _setup(solver, W, 128)
    say("rollout checkpoint counts")
    grads = []
    for s in (0, 2, 5, 23):
        say("  snapshots", s)
        _, g = _loss_grad(G, roll, ctl, rho0, target, dt, 24, s)
        grads.append(g)
    for g in grads[1:]:
        assert torch.equal(g, grads[0])


def test_staged_rollout_gradient_equals_checkpointed(mods, W):
    """Stored stage states (no recomputation in the backward pass) give the
    gradient of the checkpointed rollout bit for bit: the adjoint step
    recomputes its stage states with the forward step's own launches."""
    solver, roll = mods
    prob, ctl, rho0, target, G, dt = _setup(solver, W, 128)
    say("staged rollout")
    J0, g0 = _loss_grad(G, roll, ctl, rho0, target, dt, 24, 5)
    J1, g1 = _loss_grad(G, roll, ctl, rho0, target, dt, 24, 5, stages=True)
    assert J1 == J0
    assert torch.equal(g1, g0)


def _smooth_direction(gen, n, kmax=4):
    x = torch.arange(n, dtype=torch.float64, device="cuda") / n
    Y, X = torch.meshgrid(x, x, indexing="ij")
    d = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            a, b = torch.randn(2, dtype=torch.float64, device="cuda", generator=gen)
            ph = 2 * np.pi * (kx * X + ky * Y)
            d += a * torch.cos(ph) + b * torch.sin(ph)
    return d


def test_rollout_gradient_full_size_central_differences(mods, W):
    """1024^2, 100 steps, 9 checkpoints besides U0."""
    solver, roll = mods
    n, nsteps = 1024, 100
    prob, ctl, rho0, target, G, dt = _setup(solver, W, n)
    say("rollout full size", n, nsteps)
    for _ in range(nsteps):
        G.rk3_step(target, dt=dt)
    _, grad = _loss_grad(G, roll, ctl, rho0, target, dt, nsteps, snapshots=9)

    def rho_T(r):
        X = ctl(r)
        for _ in range(nsteps):
            G.rk3_step(X, dt=dt)
        return X[0]

    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    worst = 0.0
    for k in range(32):
        d = _smooth_direction(gen, n)
        lhs = float((grad * d).sum())
        errs = []
        for eps in (1e-6, 1e-7, 1e-8):
            rp, rm = rho_T(rho0 + eps * d), rho_T(rho0 - eps * d)
            # J+ - J- = 1/2 sum (r+ - r-) (r+ + r- - 2 target), free of cancellation in J
            fd = float((0.5 * (rp - rm) * (rp + rm - 2 * target[0])).sum()) / (2 * eps)
            errs.append(abs(fd - lhs) / abs(fd))
        say("  direction", k, lhs, ["%.1e" % e for e in errs])
        worst = max(worst, min(errs))
        assert min(errs) < 1e-7, (k, lhs, errs)
    say("  worst relative difference", worst)
