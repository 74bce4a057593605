"""Parity of the HIP residual, CFL step and SSP-RK3 step with the CPU oracle,
element by element on the same seeded inputs (sizes that span several tiles
and a ragged tail).  Tolerances: normwise relative error per variable
<= 1e-12 for one residual / one stage; multi-step runs are shadowed step by
step at that bar and compared with the free-running oracle at the end
(gpu_util: 1e-9, or twice the oracle's own rounding-order spread)."""
import numpy as np
import pytest
import torch

from gpu_util import end_bar, other_roundings, rel_err, say, shadowed_run, to_dev, to_host

pytestmark = pytest.mark.gpu

STAGE_TOL = 1e-12
# Isolated points may legitimately differ more where a weight sits within
# ~1/xi of a mapping null point (the map amplifies a 1-ulp difference by
# up to xi * amplitude); bounded relative to the largest value.
POINT_TOL = 1e-10
RUN_TOL = 1e-9

WEIGHTS = [("js", 100.0), ("z", 100.0), ("fe", 100.0), ("fe", 1e6), ("pfe", 100.0), ("linear", 100.0)]
# The unlimited linear scheme (ideal weights) is not defined on shock data:
# its interpolated states reach negative pressure (NaN on both sides).
SHOCK_WEIGHTS = [w for w in WEIGHTS if w[0] != "linear"]


@pytest.fixture(scope="module")
def lib():
    from paper_2306_09760_amd import solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return solver


def _pair(lib, ora, prob, **kw):
    return lib.Plan(**prob, **kw), ora.Problem(**prob, **kw)


def _check(gpu, ref, tol=STAGE_TOL, ptol=POINT_TOL, what=""):
    n, p = rel_err(gpu, ref)
    assert n <= tol and p <= ptol, f"{what}: normwise {n:.3e}, pointwise {p:.3e}"


# ------------------------------------------------------------------------ 1D --
@pytest.mark.parametrize("weights,xi", WEIGHTS)
@pytest.mark.parametrize("diff", ["mnd6", "md6"])
def test_residual_advection_config1(lib, ora, W, weights, xi, diff):
    prob, U, _ = W.advection_sine(seed=0)
    say("advection residual", weights, xi, diff)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi, diff=diff)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="advection")


@pytest.mark.parametrize("weights,xi", SHOCK_WEIGHTS)
@pytest.mark.parametrize("bc", ["transmissive", "periodic"])
@pytest.mark.parametrize("charproj", [True, False])
def test_residual_euler1d(lib, ora, W, weights, xi, bc, charproj):
    prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, -0.3, 0.1, 517)
    prob["bc"] = bc
    say("euler1d residual", weights, xi, bc, charproj)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi, charproj=charproj)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="euler1d")


@pytest.mark.parametrize("tm", [128, 256])
@pytest.mark.parametrize("diff", ["mnd6", "md6"])
def test_xsweep_tile_shape_invariance(lib, W, tm, diff):
    """Every tile shape gives bitwise the same residual (halo / LDS checks)."""
    prob, U, _ = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1000)
    say("tile invariance", tm, diff)
    G = lib.Plan(**prob, weights="fe", diff=diff)
    Ud = to_dev(U)
    G.tiles = (128, 32, 4)
    ref = to_host(G.residual(Ud))
    G.tiles = (tm, 32, 4)
    assert np.array_equal(to_host(G.residual(Ud)), ref)


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("diff", ["mnd6", "md6"])
def test_xsweep_packed_lines_2d(lib, ora, W, bc, diff):
    """x-lines of 300 nodes packed end to end: a tile holds the end of one
    line, the ghosts of both and the start of the next.  Both x tile sizes
    match the oracle and each other bitwise."""
    prob, U = W.random_smooth_state(7, 2, (300, 24), amp=0.3)
    U = U.copy()
    U[0, :, 290:] *= 1.8  # a jump next to the line ends
    prob["bc"] = (bc, "transmissive")
    say("packed x-lines", bc, diff)
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0, diff=diff)
    Ud = to_dev(U)
    G.tiles = (128, 32, 4)
    r128 = to_host(G.residual(Ud))
    G.tiles = (256, 32, 4)
    r256 = to_host(G.residual(Ud))
    assert np.array_equal(r128, r256)
    _check(r256, O.residual(U), what="packed x-lines")


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("diff", ["mnd6", "md6"])
def test_residual_minimum_grids(lib, ora, W, ndim, bc, diff):
    """The smallest accepted grid, 9 nodes per axis: fewer nodes than ghost
    slots plus a tile, so every x tile spans several packed lines and every
    y/z tile is mostly ghosts."""
    n = (9,) * ndim
    prob, U = W.random_smooth_state(8, ndim, n, amp=0.3)
    U = U.copy()
    U[0].flat[::4] *= 1.5  # jumps between neighbours
    prob["bc"] = bc
    say("minimum grid", ndim, bc, diff)
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0, diff=diff)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="minimum grid")


# ------------------------------------------------------------------------ 2D --
@pytest.mark.parametrize("weights,xi", SHOCK_WEIGHTS)
@pytest.mark.parametrize("diff", ["mnd6", "md6"])
def test_residual_riemann2d(lib, ora, W, weights, xi, diff):
    prob, U, _ = W.riemann2d(seed=0, n=70)
    prob["n"] = (70, 70)
    say("riemann2d residual", weights, xi, diff)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi, diff=diff)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="riemann2d")


@pytest.mark.parametrize("seg,bw", [(16, 8), (32, 4), (32, 8), (64, 4), (128, 2), (256, 1)])
def test_residual_2d_rectangular_and_march_shapes(lib, ora, W, seg, bw):
    """Non-square grid, periodic in x and transmissive in y, several march
    segment / lane shapes."""
    prob, U = W.random_smooth_state(4, 2, (77, 45), amp=0.3)
    U = U.copy()
    U[0, 10:30, 20:50] *= 2.0  # a density block with sharp edges
    prob["bc"] = ("periodic", "transmissive")
    say("2d rect", seg, bw)
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    G.tiles = (128, seg, bw)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="2d rect")


def test_residual_advection_2d(lib, ora):
    n = (40, 33)
    x = np.arange(n[0]) / n[0]
    y = np.arange(n[1]) / n[1]
    X, Y = np.meshgrid(x, y)
    U = np.where((X - 0.5) ** 2 + (Y - 0.5) ** 2 < 0.05, 1.0, 0.0)[None] + 0.1 * np.sin(2 * np.pi * X)[None]
    prob = dict(system="advection", ndim=2, n=n, adv=(1.0, -0.7), bc="periodic")
    say("advection 2d")
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="advection2d")


# ------------------------------------------------------------------------ 3D --
@pytest.mark.parametrize("weights,xi", [("fe", 100.0), ("z", 100.0), ("fe", 1e6), ("js", 100.0)])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_residual_turbulence3d(lib, ora, W, weights, xi, bc):
    prob, U, _ = W.turbulence3d(seed=0, n=20)
    prob["bc"] = bc
    say("turbulence3d residual", weights, xi, bc)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="turbulence3d")


def test_residual_3d_rectangular_md6(lib, ora, W):
    prob, U = W.random_smooth_state(6, 3, (23, 17, 19), amp=0.3)
    U = U.copy()
    U[0, :, 5:9, :] *= 1.7
    prob["bc"] = ("transmissive", "periodic", "transmissive")
    say("3d rect md6")
    G, O = _pair(lib, ora, prob, weights="pfe", xi=100.0, diff="md6")
    G.tiles = (256, 16, 8)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what="3d md6")


# ------------------------------------------------------------ CFL and RK3 ----
@pytest.mark.parametrize("case", ["adv1d", "tube", "riemann2d", "turb3d"])
def test_cfl_dt_and_one_rk3_step(lib, ora, W, case):
    if case == "adv1d":
        prob, U, _ = W.advection_sine(seed=3)
    elif case == "tube":
        prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, 300)
    elif case == "riemann2d":
        prob, U, _ = W.riemann2d(seed=2, n=48)
    else:
        prob, U, _ = W.turbulence3d(seed=1, n=16)
    say("cfl + rk3 step", case)
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    Ud = to_dev(U)
    dt = to_host(G.cfl_dt(Ud, 0.5))[0]
    dt_ref = O.cfl_dt(U, 0.5)
    assert dt == pytest.approx(dt_ref, rel=1e-14)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    G.rk3_step(Ud, dt=None, cfl=0.5, status=status)
    U1, bad = O.rk3_step(U, dt_ref)
    assert bad == 0 and int(status.item()) == 0
    _check(to_host(Ud), U1, what=f"rk3 {case}")


def _end_check(ora, prob, kw, U0, Ug, Uo, run, ratio=1.0):
    """End state of a run against the free-running oracle: 1e-9, else the
    spread of other valid roundings of the run (run(P, U) runs oracle P
    from U; gpu_util.other_roundings) times 2 max(1, ratio), which must
    itself stay informative."""
    n, p = rel_err(Ug, Uo)
    if n <= RUN_TOL and p <= RUN_TOL:
        say("  end state vs oracle", n, p)
        return
    Op = ora.Problem(**prob, **kw)
    Of = ora.Problem(**prob, **kw, variant="fma")
    alts = other_roundings(Uo, lambda X: run(Op, X), lambda X: run(Of, X), U0, Ug, ratio)
    tol, ptol, spread, informative = end_bar(Uo, alts, ratio)
    say("  end state vs oracle", n, p, "oracle rounding-order spread", spread, "step ratio", ratio)
    assert informative, f"spread {spread} too large to pin the end state"
    assert n <= tol and p <= ptol, (n, p, spread, ratio)


def test_config1_full_run(lib, ora, W):
    """Config 1 to t = 2 (400 steps of dt = 0.005) with FE at the paper's
    xi = 100: every step shadowed by the oracle's step from the GPU state,
    and the end state vs the oracle's run to 1e-9."""
    prob, U, meta = W.advection_sine(seed=0)
    say("config1 full run")
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    r = shadowed_run(G, O, U, 400, dt_fixed=0.005)
    say("  steps shadowed", r.checked, "worst step", r.worst)
    Uo, bad = O.run_steps(U, 400, dt=0.005)
    _check(to_host(r.U), Uo, tol=RUN_TOL, ptol=RUN_TOL, what="config1 run")


def test_riemann2d_multi_step_run(lib, ora, W):
    prob, U, _ = W.riemann2d(seed=0, n=64)
    say("riemann2d 20 steps")
    kw = dict(weights="fe", xi=100.0)
    G, O = _pair(lib, ora, prob, **kw)
    r = shadowed_run(G, O, U, 20, cfl=0.5, Of=ora.Problem(**prob, **kw, variant="fma"))
    say("  steps shadowed", r.checked, "worst step", r.worst, "step ratio", r.ratio.value)
    Uo, bad = O.run_steps(U, 20, cfl=0.5)
    assert bad == 0
    _end_check(ora, prob, kw, U, to_host(r.U), Uo, lambda P, X: P.run_steps(X, 20, cfl=0.5)[0],
               r.ratio.value)


def test_config3_reduced_full_run(lib, ora, W):
    """The 2D four-quadrant Riemann problem (seeded quadrant states) at
    256^2 for 200 CFL-limited steps, the reduced form of the 2048^2 run:
    every second step shadowed by the oracle's step from the GPU's state,
    and the state after 10 steps against the oracle's run.  Later states
    pin nothing element by element: two valid roundings of the oracle's own
    run (with and without FMA contraction) differ by 1.7e-13 after 10 steps,
    2e-10 after 20, 3.5e-9 after 30, 2.5e-7 after 50 and 1e-5 from 75 steps
    on."""
    n, nsteps, horizon = 256, 200, 10
    prob, U, _ = W.riemann2d(seed=0, n=n)
    say("config3 reduced run", n, nsteps)
    kw = dict(weights="fe", xi=100.0)
    G, O = _pair(lib, ora, prob, **kw)
    r = shadowed_run(G, O, U, nsteps, cfl=0.5, every=2, Of=ora.Problem(**prob, **kw, variant="fma"),
                     keep=(horizon,))
    say("  steps shadowed", r.checked, "worst step", r.worst, "step ratio", r.ratio.value)
    Uo, bad = O.run_steps(U, horizon, cfl=0.5)
    assert bad == 0
    _end_check(ora, prob, kw, U, r.kept[horizon], Uo,
               lambda P, X: P.run_steps(X, horizon, cfl=0.5)[0], r.ratio.value)


def test_config4_reduced_run_shadowed(lib, ora, W):
    """The 3D decaying-turbulence field at 64^3 for 100 CFL-limited steps,
    the reduced form of the 256^3 run: every fourth step shadowed by the
    oracle's step from the GPU's state."""
    n, nsteps = 64, 100
    prob, U, _ = W.turbulence3d(seed=0, n=n)
    say("config4 reduced run, shadowed", n, nsteps)
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    r = shadowed_run(G, O, U, nsteps, cfl=0.5, every=4)
    say("  steps shadowed", r.checked, "worst step", r.worst)


@pytest.mark.timeout(400)
def test_config4_reduced_run_end_state(lib, ora, W):
    """The same 64^3 x 100-step run: end state vs the oracle's own run."""
    n, nsteps = 64, 100
    prob, U, _ = W.turbulence3d(seed=0, n=n)
    say("config4 reduced run, end state", n, nsteps)
    kw = dict(weights="fe", xi=100.0)
    G, O = _pair(lib, ora, prob, **kw)
    Ud = to_dev(U)
    for _ in range(nsteps):
        G.rk3_step(Ud, cfl=0.5)
    Ug = to_host(Ud)
    Uo, bad = O.run_steps(U, nsteps, cfl=0.5)
    assert bad == 0
    _end_check(ora, prob, kw, U, Ug, Uo, lambda P, X: P.run_steps(X, nsteps, cfl=0.5)[0])


@pytest.mark.parametrize("case", ["tube", "riemann2d"])
def test_multi_step_run_fe_large_xi(lib, ora, W, case):
    """FE at xi = 1e6 (every map term through its own saturating tanh) over
    30 CFL-limited steps: GPU vs oracle to the run bar."""
    if case == "tube":
        prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, -0.3, 0.1, 400)
    else:
        prob, U, _ = W.riemann2d(seed=1, n=48)
    say("multi-step run, FE xi = 1e6,", case)
    kw = dict(weights="fe", xi=1e6)
    G, O = _pair(lib, ora, prob, **kw)
    r = shadowed_run(G, O, U, 30, cfl=0.5, Of=ora.Problem(**prob, **kw, variant="fma"))
    say("  steps shadowed", r.checked, "worst step", r.worst, "step ratio", r.ratio.value)
    Uo, bad = O.run_steps(U, 30, cfl=0.5)
    assert bad == 0
    _end_check(ora, prob, kw, U, to_host(r.U), Uo, lambda P, X: P.run_steps(X, 30, cfl=0.5)[0],
               r.ratio.value)


def test_status_word_flags_nonphysical_state(lib, W):
    prob, U, _ = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 64)
    U = U.copy()
    U[2, 30] = -1.0  # negative energy -> negative pressure
    say("status word")
    G = lib.Plan(**prob, weights="fe")
    Ud = to_dev(U)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    dt = torch.full((1,), 1e-4, dtype=torch.float64, device="cuda")
    G.rk3_step(Ud, dt=dt, status=status)
    assert int(status.item()) & 1


def test_autotune_keeps_results_and_picks_a_candidate(lib, ora, W):
    prob, U, _ = W.riemann2d(seed=0, n=96)
    say("autotune")
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    Ud = to_dev(U)
    tiles = G.autotune(Ud)
    assert tiles[0] in (128, 256)
    assert (tiles[1], tiles[2]) in ((16, 8), (32, 4), (32, 8), (64, 4), (128, 2), (256, 1))
    _check(to_host(G.residual(Ud)), O.residual(U), what="after autotune")


@pytest.mark.parametrize("scheme", ["wcns", "weno"])
@pytest.mark.parametrize("xi", [10.0, 120.0, 200.0, 1000.0])
def test_fe_residual_across_xi(lib, ora, W, xi, scheme):
    """FE weights at steepnesses that select each device evaluation of the
    map: one exponential per map with unclamped products (xi = 10, 120),
    one per map with a reciprocal per term (xi = 200), one per term
    (xi = 1000), for the WCNS and the WENO (App. B) family.  An evolved
    shock tube spreads the weights over [0, 1]."""
    kw = dict(weights="fe", xi=xi)
    okw = dict(kw, family=scheme)
    prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, -0.3, 0.1, 301)
    O = ora.Problem(**prob, **okw)
    U1, bad = O.run_steps(U, 30, cfl=0.5)
    assert bad == 0
    say("fe residual across xi", xi, scheme)
    G = lib.Plan(**prob, **kw, scheme=scheme)
    _check(to_host(G.residual(to_dev(U1))), O.residual(U1), what=f"fe xi={xi} {scheme}")
    prob, U = W.random_smooth_state(4, 2, (48, 40), amp=0.3)
    G, O = lib.Plan(**prob, **kw, scheme=scheme), ora.Problem(**prob, **okw)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), what=f"fe 2d xi={xi} {scheme}")
