"""The filtered embedded WENO scheme of App. B on the GPU (scheme="weno")
against the oracle's (family="weno"): residuals element by element, one
SSP-RK3 and one eq. 16 step, a shock-tube run; unsupported calls refuse."""
import numpy as np
import pytest
import torch

from gpu_util import end_bar, rel_err, say, shadowed_run_to_time, to_dev, to_host

pytestmark = pytest.mark.gpu

WEIGHTS = [("js", 100.0), ("z", 100.0), ("fe", 100.0), ("fe", 1e6), ("pfe", 100.0)]


@pytest.fixture(scope="module")
def lib():
    from paper_2306_09760_amd import solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return solver


def _pair(lib, ora, prob, **kw):
    return lib.Plan(**prob, scheme="weno", **kw), ora.Problem(**prob, family="weno", **kw)


def _check(gpu, ref, what, tol=1e-12, ptol=1e-10):
    n, p = rel_err(gpu, ref)
    assert n <= tol and p <= ptol, f"{what}: normwise {n:.3e}, pointwise {p:.3e}"


@pytest.mark.parametrize("weights,xi", WEIGHTS + [("linear", 100.0)])
def test_weno_residual_advection(lib, ora, W, weights, xi):
    prob, U, _ = W.advection_sine(seed=1, n=150)
    if weights != "linear":
        U = U.copy()
        U[0, 40:70] += 1.0     # a square pulse on the sine
    say("weno advection", weights, xi)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), "weno advection")


@pytest.mark.parametrize("weights,xi", WEIGHTS)
@pytest.mark.parametrize("bc", ["transmissive", "periodic"])
@pytest.mark.parametrize("charproj", [True, False])
def test_weno_residual_euler1d(lib, ora, W, weights, xi, bc, charproj):
    prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, 301)
    prob["bc"] = bc
    say("weno tube", weights, xi, bc, charproj)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi, charproj=charproj)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), "weno tube")


@pytest.mark.parametrize("weights,xi", [("fe", 100.0), ("z", 100.0), ("pfe", 100.0)])
def test_weno_residual_2d_3d(lib, ora, W, weights, xi):
    prob, U, _ = W.riemann2d(seed=0, n=70)
    say("weno riemann2d", weights)
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), "weno riemann2d")
    prob, U, _ = W.turbulence3d(seed=0, n=20)
    prob["bc"] = "transmissive"
    G, O = _pair(lib, ora, prob, weights=weights, xi=xi)
    _check(to_host(G.residual(to_dev(U))), O.residual(U), "weno turbulence3d")


def test_weno_steps_and_run(lib, ora, W):
    prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, 201)
    G, O = _pair(lib, ora, prob, weights="fe", xi=100.0)
    dt = O.cfl_dt(U, 0.5)
    dtd = torch.full((1,), dt, dtype=torch.float64, device="cuda")
    for method in ("rk3", "rk4"):
        Ud = to_dev(U)
        (G.rk3_step if method == "rk3" else G.rk4_step)(Ud, dt=dtd)
        U1, bad = (O.rk3_step if method == "rk3" else O.rk4_step)(U, dt)
        assert bad == 0
        _check(to_host(Ud), U1, f"weno {method} step")
    say("weno sod run")
    Of = ora.Problem(**prob, family="weno", weights="fe", xi=100.0, variant="fma")
    Ud, steps, t, worst, ratio = shadowed_run_to_time(G, O, U, 0.15, cfl=0.5, Of=Of)
    Uo, _, _, bad = O.run_to_time(U, 0.15, cfl=0.5)
    Uf, _, _, _ = Of.run_to_time(U, 0.15, cfl=0.5)
    tol, ptol, spread, informative = end_bar(Uo, Uf, ratio.value)
    n, p = rel_err(to_host(Ud), Uo)
    say("  steps", steps, "worst step", worst, "spread", spread, "gpu vs oracle", n, p)
    assert bad == 0 and informative and n <= tol and p <= ptol


def test_weno_unsupported_calls_refuse(lib, W):
    from paper_2306_09760_amd._lib import WCNSError
    prob, U, meta = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 64)
    G = lib.Plan(**prob, scheme="weno", weights="fe")
    Ud = to_dev(U)
    with pytest.raises(WCNSError):
        G.residual_adjoint(Ud, torch.ones_like(Ud))
    with pytest.raises(WCNSError):
        G.weight_histogram(Ud)
    assert G.autotune(Ud) == G.tiles
    prob, U, meta = W.shock_tube_batch(seed=0, nprob=4)
    with pytest.raises(WCNSError):
        lib.BatchPlan(meta["offsets"], meta["h"], scheme="weno")
