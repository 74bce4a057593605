"""The oracle's per-interpolation weights (App. A statistics): how many
interpolations one residual performs, and what the three recorded weight
sets are on data where they are known exactly."""
import numpy as np
import pytest

D = np.array([1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0])


@pytest.mark.parametrize("bc,diff", [("periodic", "mnd6"), ("transmissive", "mnd6"),
                                     ("transmissive", "md6")])
def test_interpolation_count(ora, W, bc, diff):
    prob, U = W.random_smooth_state(3, 2, (12, 10))
    prob["bc"] = bc
    P = ora.Problem(**prob, weights="z", xi=100.0, diff=diff)
    G = 5 if diff == "md6" else 4
    mids = lambda n: n if bc == "periodic" else n + 2 * G - 5
    expect = (10 * mids(12) + 12 * mids(10)) * 4 * 2   # lines x midpoints x fields x sides
    assert P.interpolation_weights(U).shape == (expect, 3, 3)


@pytest.mark.parametrize("weights", ["z", "js", "fe", "pfe"])
def test_flat_state_weights(ora, W, weights):
    prob, U, _ = W.shock_tube(1.0, 0.0, 1.0, 1.0, 0.0, 1.0, 40)   # uniform state
    w = ora.Problem(**prob, weights=weights, xi=100.0).interpolation_weights(U)
    if weights == "js":   # d_k / eps^2 normalised: d_k up to rounding
        assert np.allclose(w[:, 0, :], D, rtol=1e-15, atol=0)
    else:                 # Z: tau = 0 gives alpha = d exactly, and sum d = 1
        assert np.array_equal(w[:, 0, :], np.broadcast_to(D, w[:, 0, :].shape))
    g = np.array([ora.fe_map(k, D[k], 100.0) for k in range(3)])
    assert np.allclose(w[:, 1, :], g / g.sum(), rtol=0, atol=1e-16)
    used = {"z": w[:, 0, :], "js": w[:, 0, :], "fe": w[:, 1, :], "pfe": w[:, 0, :]}[weights]
    assert np.array_equal(w[:, 2, :], used)


def test_pfe_switch_rule(ora, W):
    prob, U, _ = W.paper_problem("shu_osher")
    cv = 1e-3
    w = ora.Problem(**prob, weights="pfe", xi=100.0, cv=cv).interpolation_weights(U)
    inside = np.all(np.abs(w[:, 0, :] - D) <= cv, axis=1)
    assert inside.any() and (~inside).any()
    assert np.array_equal(w[inside, 2, :], w[inside, 0, :])
    assert np.array_equal(w[~inside, 2, :], w[~inside, 1, :])
    assert np.allclose(w.sum(axis=2), 1.0, atol=1e-14)
