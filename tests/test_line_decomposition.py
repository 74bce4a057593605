"""The line decomposition used by the full-size GPU parity tests, checked on
the oracle alone: at small sizes the oracle's residual at a point equals the
sum of its line contributions (to rounding)."""
import numpy as np

from line_parity import line_contribution


def _check(ora, prob, U, pts, kw):
    R = ora.Problem(**prob, **kw).residual(U)
    scale = np.abs(R).reshape(R.shape[0], -1).max(axis=1)
    for idx in pts:
        ref = sum(line_contribution(ora, prob, U, ax, idx, kw) for ax in range(prob["ndim"]))
        assert np.max(np.abs(R[(slice(None),) + idx] - ref) / scale) <= 1e-13, idx


def test_line_decomposition_2d_riemann(ora, W):
    prob, U, _ = W.riemann2d(seed=1, n=40)
    _check(ora, prob, U, [(0, 0), (31, 31), (30, 33), (39, 12), (5, 39), (20, 20)],
           dict(weights="fe", xi=100.0))


def test_line_decomposition_3d_box(ora, W):
    prob, U, _ = W.turbulence3d(seed=1, n=12)
    _check(ora, prob, U, [(0, 0, 0), (11, 5, 3), (6, 11, 0)], dict(weights="z", xi=100.0))
    prob["bc"] = "transmissive"
    _check(ora, prob, U, [(0, 0, 0), (11, 11, 11), (3, 0, 7)], dict(weights="fe", xi=100.0))
