"""Helpers shared by the GPU tests: host/device copies, the parity norms and
the multi-step parity checks.

Multi-step runs are held to two bars:
  * a shadow check of the step map: at every step (or at sampled steps) the
    GPU's step from its own state equals the oracle's one step from that same
    state with the same dt, to STEP_TOL normwise and STEP_PTOL pointwise.
    This pins every step without the amplification of rounding differences
    that a long run of a nonlinear scheme brings;
  * the end state against the free-running oracle, to RUN_TOL, or where the
    method itself is more sensitive to rounding order on that run, to twice
    the spread of valid roundings of the same run around the oracle's,
    scaled by r, the ratio of the GPU's per-step difference from the oracle
    to the FMA build's (both measured at the shadowed steps, from the same
    states; rounding differences grow along a run in proportion to their
    per-step size).  The spread is the largest of three samples: the
    oracle's FMA build (another valid rounding of the same arithmetic), and
    the plain and FMA builds started from the initial state perturbed by one
    ulp per value; one sample alone understates how far a fourth valid
    rounding (the GPU's) may land once rounding differences are amplified.
    A bar above SPREAD_CAP means valid roundings of the run disagree too much
    for the end state to pin anything; such runs are checked against an
    exact solution, or compared at a horizon where the bar is still below
    the cap."""
import sys
from types import SimpleNamespace

import numpy as np
import torch

DEV = "cuda"

STEP_TOL = 1e-12
STEP_PTOL = 1e-10
RUN_TOL = 1e-9
SPREAD_CAP = 1e-7


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(gpu, ref):
    """Per-variable normwise relative error, max over variables, and the
    largest pointwise difference relative to max |ref|."""
    gpu = np.asarray(gpu).reshape(gpu.shape[0], -1)
    ref = np.asarray(ref).reshape(ref.shape[0], -1)
    norm = 0.0
    for v in range(ref.shape[0]):
        den = np.linalg.norm(ref[v])
        num = np.linalg.norm(gpu[v] - ref[v])
        norm = max(norm, num / den if den > 0 else num)
    point = np.abs(gpu - ref).max() / max(np.abs(ref).max(), 1e-300)
    return norm, point


def say(*a):
    """Names the case on stdout before GPU work (flushed)."""
    print(*a, flush=True)
    sys.stdout.flush()


def end_bar(ref, alt, ratio=1.0):
    """Bar for the end state of a run: (normwise bar, pointwise bar, spread,
    informative).  ``alt`` is one other valid rounding of the same run (or a
    list of them: the spread is the largest); the bar is RUN_TOL, or 2
    max(1, ratio) times the spread where that is larger; ``informative`` is
    False when the normwise bar exceeds SPREAD_CAP."""
    alts = alt if isinstance(alt, (list, tuple)) else [alt]
    errs = [rel_err(a, ref) for a in alts]
    n = max(e[0] for e in errs)
    p = max(e[1] for e in errs)
    r = 2.0 * max(1.0, ratio)
    tol = max(RUN_TOL, r * n)
    return tol, max(RUN_TOL, r * p), (n, p), tol <= SPREAD_CAP


def ulp_perturbed(U, seed=0):
    """U with every value moved by one unit in the last place, up or down at
    random (a valid initial state for a second rounding of a run)."""
    g = np.random.default_rng(seed)
    up = g.random(np.shape(U)) < 0.5
    return np.where(up, np.nextafter(U, np.inf), np.nextafter(U, -np.inf))


def other_roundings(ref, run_plain, run_fma, U0, gpu=None, ratio=1.0):
    """Valid other roundings of an oracle run, as few as decide: the FMA
    build's run, then (if the GPU end state `gpu` is outside the bar that
    one gives) the plain and FMA builds from the one-ulp-perturbed U0."""
    alts = [run_fma(U0)]
    if gpu is not None:
        tol, ptol, _, _ = end_bar(ref, alts, ratio)
        n, p = rel_err(gpu, ref)
        if n <= tol and p <= ptol:
            return alts
    U1 = ulp_perturbed(U0)
    alts += [run_plain(U1), run_fma(U1)]
    return alts


class StepRatio:
    """Accumulates, over shadowed steps, the GPU's and the FMA build's
    normwise differences from the oracle's step from the same state."""

    def __init__(self):
        self.gpu = 0.0
        self.fma = 0.0

    def add(self, e_gpu, e_fma):
        self.gpu += e_gpu
        self.fma += e_fma

    @property
    def value(self):
        return self.gpu / self.fma if self.fma > 0 else 1.0


def check_step(gpu_after, ref_after, what=""):
    n, p = rel_err(gpu_after, ref_after)
    assert n <= STEP_TOL and p <= STEP_PTOL, f"{what}: step map {n:.3e} / {p:.3e}"
    return n, p


def shadowed_run(G, O, U0, nsteps, cfl=0.5, dt_fixed=None, every=1, method="rk3", Of=None,
                 keep=()):
    """Runs nsteps steps of plan G from U0 (CFL-limited, or dt_fixed), and
    at every `every`-th step (and the last) checks the step against the
    oracle O's one step from the GPU's own state with the GPU's dt; with Of
    (the FMA build) the same step of Of is taken too, for the step ratio.
    The host states after the steps listed in `keep` are returned as well.
    Returns a namespace: U (final device state), worst (step errors),
    checked, ratio (StepRatio), kept ({step count: state})."""
    Ud = to_dev(U0)
    dt = torch.zeros(1, dtype=torch.float64, device=DEV)
    if dt_fixed is not None:
        dt.fill_(dt_fixed)
    step = {"rk3": G.rk3_step, "rk4": G.rk4_step}[method]
    ostep = {"rk3": O.rk3_step, "rk4": O.rk4_step}[method]
    worst = (0.0, 0.0)
    checked = 0
    ratio = StepRatio()
    kept = {}
    for k in range(nsteps):
        if dt_fixed is None:
            G.cfl_dt(Ud, cfl, out=dt)
        shadow = (k % every == 0) or k == nsteps - 1
        if shadow:
            Ub = to_host(Ud).copy()
            dth = float(dt.item())
        step(Ud, dt=dt)
        if shadow:
            Uo, bad = ostep(Ub, dth)
            assert bad == 0, f"oracle step {k} non-physical"
            Ua = to_host(Ud)
            e = check_step(Ua, Uo, what=f"step {k}")
            worst = (max(worst[0], e[0]), max(worst[1], e[1]))
            checked += 1
            if Of is not None:
                Uf, _ = {"rk3": Of.rk3_step, "rk4": Of.rk4_step}[method](Ub, dth)
                ratio.add(e[0], rel_err(Uf, Uo)[0])
        if k + 1 in keep:
            kept[k + 1] = to_host(Ud).copy()
    return SimpleNamespace(U=Ud, worst=worst, checked=checked, ratio=ratio, kept=kept)


def shadowed_run_to_time(G, O, U0, t_end, cfl=0.5, method="rk3", every=1, Of=None):
    """March plan G from U0 to t_end as Plan.run_to_time does (CFL-limited
    steps, the last one clipped), shadowing every `every`-th step by the
    oracle O's step from the GPU's state with the GPU's dt (and by the FMA
    build Of's, for the step ratio).  Returns (final device state, steps, t,
    worst step errors, StepRatio)."""
    Ud = to_dev(U0)
    dt = torch.zeros(1, dtype=torch.float64, device=DEV)
    step = {"rk3": G.rk3_step, "rk4": G.rk4_step}[method]
    ostep = {"rk3": O.rk3_step, "rk4": O.rk4_step}[method]
    t, k = 0.0, 0
    worst = (0.0, 0.0)
    ratio = StepRatio()
    while t < t_end:
        G.cfl_dt(Ud, cfl, out=dt)
        h = float(dt.item())
        if t + h > t_end:
            h = t_end - t
            dt.fill_(h)
        shadow = k % every == 0
        if shadow:
            Ub = to_host(Ud).copy()
        step(Ud, dt=dt)
        if shadow:
            Uo, bad = ostep(Ub, h)
            assert bad == 0, f"oracle step {k} non-physical"
            e = check_step(to_host(Ud), Uo, what=f"step {k}")
            worst = (max(worst[0], e[0]), max(worst[1], e[1]))
            if Of is not None:
                Uf, _ = {"rk3": Of.rk3_step, "rk4": Of.rk4_step}[method](Ub, h)
                ratio.add(e[0], rel_err(Uf, Uo)[0])
        t += h
        k += 1
    return Ud, k, t, worst, ratio
