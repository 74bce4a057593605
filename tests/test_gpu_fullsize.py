"""Parity at the full benchmark sizes, in the launch configuration the bench
uses (autotuned tiles): the 2D four-quadrant Riemann problem at 2048^2 and
the 3D turbulence box at 256^3.

The oracle cannot evaluate those grids in test time, so the residual is
checked on sampled points: the residual of a dimension-by-dimension scheme is
the sum of one line contribution per direction, and the oracle computes each
from that line alone, as a grid whose other axes hold nine periodic copies of
the line (their differences vanish exactly, so only the line's direction
contributes).  The CFL time step is checked on the whole grid."""
import numpy as np
import pytest
import torch

from gpu_util import say, to_dev, to_host
from line_parity import line_contribution

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2306_09760_amd import solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return solver


def _samples(shape, rng, special, count):
    pts = set(special)
    while len(pts) < count:
        pts.add(tuple(int(rng.integers(0, s)) for s in shape))
    return sorted(pts)


def _check_sampled(lib, ora, prob, U, special, count, kw, what):
    G = lib.Plan(**prob, **kw)
    Ud = to_dev(U)
    tiles = G.autotune(Ud)
    say(what, "tiles", tiles)
    R = to_host(G.residual(Ud))
    scale = np.abs(R).reshape(R.shape[0], -1).max(axis=1)
    rng = np.random.default_rng(17)
    pts = _samples(U.shape[1:], rng, special, count)
    worst = 0.0
    for idx in pts:
        ref = sum(line_contribution(ora, prob, U, axis, idx, kw) for axis in range(prob["ndim"]))
        got = R[(slice(None),) + idx]
        err = np.max(np.abs(got - ref) / scale)
        worst = max(worst, err)
        assert err <= 1e-10, (what, idx, got, ref, err)
    say(what, "sampled points", len(pts), "worst pointwise error / max|R|", worst)
    # CFL step on the whole grid
    O = ora.Problem(**prob, **kw)
    dt = to_host(G.cfl_dt(Ud, 0.5))[0]
    assert dt == pytest.approx(O.cfl_dt(U, 0.5), rel=1e-14)


def test_riemann2d_2048_sampled(lib, ora, W):
    prob, U, _ = W.riemann2d(seed=0, n=2048)
    n = 2048
    q = int(round(0.8 * (n - 1)))  # node index of the quadrant lines
    special = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (q, q), (q - 1, q + 1),
               (q + 2, q - 3), (q, 5), (7, q), (n - 2, q), (q, n - 3), (1, 2)]
    _check_sampled(lib, ora, prob, U, special, 48, dict(weights="fe", xi=100.0),
                   "riemann2d 2048^2")


def test_turbulence3d_256_sampled(lib, ora, W):
    prob, U, _ = W.turbulence3d(seed=0, n=256)
    special = [(0, 0, 0), (255, 255, 255), (0, 128, 255), (255, 0, 7), (100, 200, 3)]
    _check_sampled(lib, ora, prob, U, special, 24, dict(weights="fe", xi=100.0),
                   "turbulence3d 256^3")
