"""Pins of the oracle's filtered embedded WENO scheme (App. B): the
finite-difference WENO5 reconstruction with the ideal weights of Table B.1,
the FE map with the coefficients of Table B.2, Lax-Friedrichs flux splitting
and a conservative difference."""
import numpy as np
import pytest

D_WENO = np.array([0.1, 0.6, 0.3])


def _rec(ora, weights, f, xi=100.0):
    P = ora.Problem(system="advection", ndim=1, n=(16,), weights=weights, xi=xi, family="weno")
    return P.reconstruct_weno(np.asarray(f, dtype=np.float64))


def test_linear_reconstruction_is_the_fifth_order_upwind_flux(ora):
    """f_j are cell averages of the primitive H; the flux at x_{i+1/2} is H
    there: solve the 5x5 moment system for the coefficients."""
    A = np.empty((5, 5))
    for p in range(5):
        for k, j in enumerate(range(-2, 3)):
            A[p, k] = ((j + 0.5) ** (p + 1) - (j - 0.5) ** (p + 1)) / (p + 1)
    c = np.linalg.solve(A, 0.5 ** np.arange(5))
    assert np.allclose(c, np.array([2, -13, 47, 27, -3]) / 60, atol=1e-14)
    rng = np.random.default_rng(0)
    for _ in range(5):
        f = rng.standard_normal(5)
        v, wb, wo = _rec(ora, "linear", f)
        assert v == pytest.approx(float(c @ f), abs=1e-14)
        assert np.allclose(wo, D_WENO, atol=0)


CONTROL_B1 = [(0, 0.1, 0.1), (1, 0.6, 0.6), (2, 0.3, 0.3),        # Case_0
              (1, 2 / 3, 0.5), (2, 1 / 3, 0.5),                   # Case_1
              (2, 1.0, 1.0), (0, 1.0, 1.0),                       # Case_2, Case_3
              (0, 1 / 7, 0.25), (1, 6 / 7, 0.75)]                 # Case_4


@pytest.mark.parametrize("i,w,g", CONTROL_B1)
def test_weno_fe_map_hits_table_b1_at_large_xi(ora, i, w, g):
    assert ora.fe_map(i, w, 1e6, 0.5, family="weno") == pytest.approx(g, abs=2e-16)


@pytest.mark.parametrize("weights", ["js", "z"])
@pytest.mark.parametrize("case,limit", [("case1", (0.0, 2 / 3, 1 / 3)), ("case2", (0.0, 0.0, 1.0)),
                                        ("case3", (1.0, 0.0, 0.0)), ("case4", (1 / 7, 6 / 7, 0.0))])
def test_base_weights_reach_table_b1_original_values(ora, weights, case, limit):
    f = np.array([0.10, 0.20, 0.30, 0.40, 0.50])
    shift = {"case1": [0], "case2": [0, 1], "case3": [3, 4], "case4": [4]}[case]
    f[shift] += 1e4
    _, wb, _ = _rec(ora, weights, f)
    assert np.allclose(wb, limit, atol=1e-9), (case, wb)


@pytest.mark.parametrize("weights,xi,order", [("linear", 1e6, 5), ("js", 1e6, 5), ("fe", 1e6, 5),
                                              ("z", 1e6, 5)])
def test_weno_smooth_advection_residual_order(ora, weights, xi, order):
    errs = []
    Ns = (80, 160, 320)
    for N in Ns:
        h = 2.0 / N
        x = -1 + h * np.arange(N)
        P = ora.Problem(system="advection", ndim=1, n=(N,), h=h, weights=weights, xi=xi,
                        family="weno")
        R = P.residual(np.sin(np.pi * x + 0.3))
        errs.append(np.abs(R + np.pi * np.cos(np.pi * x + 0.3)).max())
    rate = np.log(errs[0] / errs[-1]) / np.log(Ns[-1] / Ns[0])
    assert rate == pytest.approx(order, abs=0.35), errs


@pytest.mark.parametrize("weights", ["z", "fe", "pfe"])
def test_weno_periodic_residual_is_conservative(ora, W, weights):
    prob, U = W.random_smooth_state(5, 2, (16, 12))
    U = U.copy()
    U[0].flat[: U[0].size // 3] *= 1.5
    R = ora.Problem(weights=weights, xi=100.0, family="weno", **prob).residual(U)
    for v in range(U.shape[0]):
        assert abs(R[v].sum()) < 1e-11 * np.abs(R[v]).sum()


def test_weno_sod_converges_to_exact_riemann_solution(ora, W):
    from oracle import exact_riemann as er
    errs = []
    for N in (101, 201, 401):
        prob, U, meta = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, N)
        P = ora.Problem(weights="fe", xi=100.0, family="weno", **prob)
        U2, steps, t, bad = P.run_to_time(U, 0.2, cfl=0.5)
        assert bad == 0 and t == pytest.approx(0.2)
        rho_ex, _, _ = er.sample(meta["x"], 0.2, 0.5, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
        errs.append(np.mean(np.abs(U2[0] - rho_ex)))
    assert errs[0] > errs[1] > errs[2] and errs[-1] < 5e-3, errs
