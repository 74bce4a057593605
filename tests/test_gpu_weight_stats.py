"""Weight histograms (App. A statistics) from the GPU against histograms of
the oracle's per-interpolation weights on the same states.  Both sides bin
FP64 weights that agree to rounding, so a bin may differ only for a weight
within rounding of a bin edge; totals agree exactly."""
import numpy as np
import pytest
import torch

from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu
NB = 10000


@pytest.fixture(scope="module")
def lib():
    from paper_2306_09760_amd import solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return solver


def _oracle_hist(w, nbins=NB):
    h = np.zeros((3, 3, nbins), dtype=np.int64)
    b = np.minimum((w * nbins).astype(np.int64), nbins - 1)
    for kind in range(3):
        for k in range(3):
            h[kind, k] = np.bincount(b[:, kind, k], minlength=nbins)
    return h


def _compare(G, O, U, what):
    hg = to_host(G.weight_histogram(to_dev(U), nbins=NB))
    ho = _oracle_hist(O.interpolation_weights(U))
    total = ho[0, 0].sum()
    assert (hg.sum(axis=2) == total).all(), (what, hg.sum(axis=2), total)
    diff = np.abs(hg - ho).sum()
    say(what, "interpolations", total, "bin differences", diff)
    assert diff <= max(4, 1e-5 * total * 9), (what, diff)


@pytest.mark.parametrize("name,weights", [("sod", "pfe"), ("shu_osher", "fe"), ("lax", "z"),
                                          ("titarev_toro", "pfe")])
def test_weight_histogram_1d_paper_problems(lib, ora, W, name, weights):
    """Initial states: flat stretches give IS = 0 exactly on both sides."""
    prob, U, meta = W.paper_problem(name)
    _compare(lib.Plan(**prob, weights=weights, xi=100.0),
             ora.Problem(**prob, weights=weights, xi=100.0), U, f"{name} t=0")


@pytest.mark.parametrize("weights", ["pfe", "z", "js"])
def test_weight_histogram_evolved_smooth_state(lib, ora, W, weights):
    """An evolved state whose every field varies: no stencil is flat to
    rounding.  (Near-flat stencils of evolved shock problems, whose
    smoothness indicators are rounding noise, give implementation-defined
    weights on any two codes and are not compared bin by bin.)"""
    prob, U = W.random_smooth_state(7, 1, (300,), amp=0.3)
    O = ora.Problem(**prob, weights=weights, xi=100.0)
    U1, bad = O.run_steps(U, 20, cfl=0.3)
    assert bad == 0
    _compare(lib.Plan(**prob, weights=weights, xi=100.0), O, U1, f"smooth evolved {weights}")


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_weight_histogram_2d_3d(lib, ora, W, bc):
    prob, U, _ = W.riemann2d(seed=3, n=40)   # flat quadrants: IS = 0 exactly
    prob["bc"] = bc
    _compare(lib.Plan(**prob, weights="pfe", xi=100.0), ora.Problem(**prob, weights="pfe", xi=100.0),
             U, f"riemann2d {bc}")
    prob, U = W.random_smooth_state(2, 3, (12, 11, 10), amp=0.3)
    prob["bc"] = bc
    _compare(lib.Plan(**prob, weights="z", xi=100.0, diff="md6"),
             ora.Problem(**prob, weights="z", xi=100.0, diff="md6"), U, f"turbulence3d {bc}")


@pytest.mark.parametrize("xi", [100.0, 1e6])
def test_weight_statistics_runner_sod(lib, xi):
    """App. A on Sod: the FE images put more of the interpolations in the
    ideal region than the Z weights (the paper reports about twice as
    many), and at xi = 1e6 the PFE run's used weights stay close to the FE
    run's.  At xi = 100 the ideal-region fractions are decided by which
    stencils stay bit-exactly flat (IS = 0, weights exactly d_k): a
    rounding-level property of the whole run (the oracle's own run gives
    P(Z) = 0.28 on Sod, and reordering the FE arithmetic moves the GPU
    figure between 0.22 and 0.45), so only the ordering is asserted there."""
    from paper_2306_09760_amd import paper_problems as pp
    s0 = pp.weight_statistics("sod", 0.0, xi=xi)
    s3 = pp.weight_statistics("sod", 1e-3, xi=xi)
    say("sod stats xi", xi, s0["p_ideal"], s0["ideal_bins"], s3["p_ideal"]["used"])
    for k in range(3):
        assert 0.0 < s0["p_ideal"]["z"][k] < s0["p_ideal"]["fe_mapped"][k] <= 1.0
        if xi == 1e6:
            assert abs(1 - s3["p_ideal"]["used"][k] / s0["p_ideal"]["used"][k]) < 0.2
