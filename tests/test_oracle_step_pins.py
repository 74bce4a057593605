"""Pins of the oracle's time-step restriction, state check and operation
counter against values written out by hand.

* cfl_dt: dt = CFL / max_i sum_d (|u_d| + c) / h_d (Sec. 4 runs at a fixed
  CFL number; the sum over directions is the reading of the multi-dimensional
  restriction), c = sqrt(gamma p / rho), and sum_d |a_d| / h_d for scalar
  advection.  The cases below are built so that replacing the sum by a
  maximum over directions, dropping a 1/h, or taking another sound speed
  changes the result.
* check_state: a state is physical when every value is finite and (Euler)
  rho > 0 and p > 0; the edges rho = 0 and p = 0 are non-physical.
* op counter: one interpolation (eq. 5-6 with eq. 9-11, 14-15, 20-21) and
  one midpoint flux, tallied term by term from the formulas as written.
"""
import numpy as np
import pytest

GAMMA = 1.4


def cons(rho, vel, p, g=GAMMA):
    vel = np.asarray(vel, dtype=float)
    return np.concatenate([[rho], rho * vel, [p / (g - 1) + 0.5 * rho * vel @ vel]])


def grid_state(prims, n):
    """Variable-major state of len(prims) nodes along x of an (n) grid,
    filled cyclically with the given (rho, vel, p) triples."""
    nd = len(n)
    npts = int(np.prod(n))
    U = np.empty((nd + 2, npts))
    for i in range(npts):
        rho, vel, p = prims[i % len(prims)]
        U[:, i] = cons(rho, vel, p)
    return U.reshape((nd + 2,) + tuple(reversed(n)))


# ------------------------------------------------------------------ cfl_dt --
@pytest.mark.parametrize("nd", [1, 2, 3])
def test_cfl_dt_uniform_state_unequal_spacing(ora, nd):
    """A uniform state: dt = CFL / sum_d (|u_d| + c) / h_d by hand."""
    rho, p = 1.3, 0.7
    vel = [0.4, -0.9, 0.25][:nd]
    h = [0.01, 0.037, 0.0023][:nd]
    n = (11, 10, 9)[:nd]
    c = np.sqrt(GAMMA * p / rho)
    expect = 0.5 / sum((abs(v) + c) / hd for v, hd in zip(vel, h))
    P = ora.Problem(system="euler", ndim=nd, n=n, h=h)
    dt = P.cfl_dt(grid_state([(rho, vel, p)], n), 0.5)
    assert dt == pytest.approx(expect, rel=1e-14)


def test_cfl_dt_sums_over_directions_at_the_worst_node(ora):
    """Two states in 2D with h = (1, 1): node A has u = (1, 0), c = 1, node B
    u = (0.8, 0.8), c = 1.  Summed rates: A 3.0, B 3.6 -> dt = CFL / 3.6.
    The maximum over directions would pick A (2.0 > 1.8) and give CFL / 2."""
    rho = 1.0
    p = rho / GAMMA  # c = 1
    n = (9, 9)
    A = (rho, [1.0, 0.0], p)
    B = (rho, [0.8, 0.8], p)
    U = grid_state([A] * 40 + [B] + [A] * 40, n)  # B at node 40, inside the grid
    P = ora.Problem(system="euler", ndim=2, n=n, h=(1.0, 1.0))
    assert P.cfl_dt(U, 0.5) == pytest.approx(0.5 / 3.6, rel=1e-14)
    # and with h_y = 0.5 the y term of B doubles: 1.8 + 2 * 1.8 = 5.4
    P = ora.Problem(system="euler", ndim=2, n=n, h=(1.0, 0.5))
    assert P.cfl_dt(U, 0.5) == pytest.approx(0.5 / 5.4, rel=1e-14)


def test_cfl_dt_sound_speed_from_pressure_and_density(ora):
    """1D two-state tube: the faster node decides, c = sqrt(gamma p / rho)."""
    n = (20,)
    L = (1.0, [0.0], 1.0)      # |u| + c = sqrt(1.4)
    R = (0.125, [0.3], 0.1)    # |u| + c = 0.3 + sqrt(1.12)
    U = grid_state([L] * 10 + [R] * 10, n)
    P = ora.Problem(system="euler", ndim=1, n=n, h=(0.05,))
    expect = 0.5 / (max(np.sqrt(1.4), 0.3 + np.sqrt(1.4 * 0.1 / 0.125)) / 0.05)
    assert P.cfl_dt(U, 0.5) == pytest.approx(expect, rel=1e-14)


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_cfl_dt_advection(ora, nd):
    adv = (1.5, -2.0, 0.5)[:nd]
    h = (0.1, 0.02, 0.05)[:nd]
    n = (9, 10, 11)[:nd]
    P = ora.Problem(system="advection", ndim=nd, n=n, h=h, adv=adv + (0.0,) * (3 - nd))
    U = np.random.default_rng(0).standard_normal((1,) + tuple(reversed(n)))
    expect = 0.3 / sum(abs(a) / hd for a, hd in zip(adv, h))
    assert P.cfl_dt(U, 0.3) == pytest.approx(expect, rel=1e-14)


# ------------------------------------------------------------- check_state --
@pytest.mark.parametrize("nd", [1, 2, 3])
def test_check_state_edges(ora, nd):
    n = (9,) * nd
    P = ora.Problem(system="euler", ndim=nd, n=n)
    good = grid_state([(1.0, [0.1] * nd, 1.0)], n)
    assert P.check_state(good) == 0

    def with_node(vals):
        U = good.copy().reshape(nd + 2, -1)
        U[:, 5] = vals
        return U.reshape(good.shape)

    m = np.zeros(nd)
    m[0] = 2.0
    # rho = 0, rho < 0
    assert P.check_state(with_node(np.r_[0.0, m, 3.0])) == 1
    assert P.check_state(with_node(np.r_[-1.0, m, 3.0])) == 1
    # p = 0 exactly: E = |m|^2 / (2 rho) = 2 (the inclusive edge)
    assert P.check_state(with_node(np.r_[1.0, m, 2.0])) == 1
    # p < 0
    assert P.check_state(with_node(np.r_[1.0, m, 1.5])) == 1
    # a nearly degenerate but valid state: p = (gamma - 1) 2^-40 > 0
    assert P.check_state(with_node(np.r_[1.0, m, 2.0 + 2.0 ** -40])) == 0
    # a tiny density with a valid pressure
    assert P.check_state(with_node(np.r_[1e-300, np.zeros(nd), 1.0])) == 0
    # non-finite values anywhere
    for k in range(nd + 2):
        v = np.r_[1.0, np.zeros(nd), 3.0]
        v[k] = np.nan
        assert P.check_state(with_node(v)) == 1
        v[k] = np.inf
        assert P.check_state(with_node(v)) == 1


def test_check_state_uses_every_momentum_component(ora):
    """rho = 1, m = (1, 1), E = 0.75: |m|^2 / 2 = 1 > E, so p < 0; a check
    that read only the first component would see p = 0.4 * 0.25 > 0."""
    n = (9, 9)
    P = ora.Problem(system="euler", ndim=2, n=n)
    U = grid_state([(1.0, [0.1, 0.1], 1.0)], n).reshape(4, -1)
    U[:, 5] = [1.0, 1.0, 1.0, 0.75]
    assert P.check_state(U.reshape(4, 9, 9)) == 1
    U[:, 5] = [1.0, 1.0, 0.0, 0.75]
    assert P.check_state(U.reshape(4, 9, 9)) == 0


def test_check_state_advection_only_needs_finite_values(ora):
    P = ora.Problem(system="advection", ndim=1, n=(12,))
    U = -np.ones((1, 12))
    assert P.check_state(U) == 0
    U[0, 3] = np.nan
    assert P.check_state(U) == 1


# --------------------------------------------------------------- op counter --
def _ops(add=0, mul=0, div=0, sqrt=0, tanh=0):
    return dict(add=add, mul=mul, div=div, sqrt=sqrt, tanh=tanh)


def _plus(*parts, times=None):
    out = _ops()
    for k, part in enumerate(parts):
        f = 1 if times is None else times[k]
        for key in out:
            out[key] += f * part[key]
    return out


# One interpolation, term by term:
#   four first differences of the stencil                      4 add
#   eq. 10 through them: h f_0 = (3 du_1 - du_0)/2             2 mul 1 add
#                        h s_0 = du_1 - du_0                          1 add
#                        h f_1 = (du_1 + du_2)/2               1 mul 1 add
#                        h s_1 = du_2 - du_1                          1 add
#                        h f_2 = (3 du_2 - du_3)/2             2 mul 1 add
#                        h s_2 = du_3 - du_2                          1 add
#   eq. 9: IS_k = (h f_k)^2 + (h^2 s_k)^2, three of them       6 mul 3 add
IS = _ops(add=13, mul=11)
# eq. 11 (JS): (IS_k + eps) 3 add, alpha_k = d_k / den^2 3 mul 3 div, the sum
# of the alphas 3 add, omega_k = alpha_k / sum 3 div
JS = _ops(add=6, mul=3, div=6)
# eq. 14-15 (Z, p = 2): tau = |IS_0 - IS_2| 1 add; per k: ratio = tau / (IS_k
# + eps) 1 add 1 div, ratio^2 as two products 2 mul, d_k (1 + r^2) 1 add 1 mul,
# the sum 1 add; omega_k = alpha_k / sum 3 div
Z = _ops(add=1 + 3 * 3, mul=3 * 3, div=3 + 3)
# eq. 20 per term: (omega_{i,j} - omega_{i,j-1}) 1 add, times phi 1 mul, / 2
# 1 div, (omega - null point) 1 add, times xi phi 1 mul, tanh, amplitude x tanh
# 1 mul, accumulated 1 add; 3 + 4 + 3 = 10 terms; renormalisation: the sum of
# the three g 3 add, g_k / sum 3 div
FE = _plus(_ops(add=3, mul=3, div=1, tanh=1), _ops(add=3, div=3), times=[10, 1])
# eq. 5: three candidates of 3, 3, 2 scaled values, 2 add each, / 8 each
CAND = _ops(add=6, mul=8, div=3)
# eq. 6: sum_k omega_k u_k
COMB = _ops(add=2, mul=3)


@pytest.mark.parametrize("weights,expect", [
    ("linear", _plus(IS, CAND, COMB)),
    ("js", _plus(IS, JS, CAND, COMB)),
    ("z", _plus(IS, Z, CAND, COMB)),
    ("fe", _plus(IS, Z, FE, CAND, COMB)),
])
def test_op_count_of_one_interpolation(ora, weights, expect):
    P = ora.Problem(system="euler", ndim=1, n=(16,), weights=weights, xi=100.0)
    got = P.count_interpolate_ops(np.array([1.0, 2.0, 0.5, 3.0, 1.0]))
    assert got == expect


# Roe average and eigenvectors of the 1D Euler Jacobian (nd = 1):
#   sqrt(rho_A), sqrt(rho_B)                                          2 sqrt
#   |u|^2 of each node: m * m / (rho * rho), summed                   4 mul 2 div 2 add
#   p of each node: (gamma - 1)(E - 0.5 rho |u|^2)                    6 mul 2 add
#   Roe velocity (sA u_A + sB u_B)/(sA + sB), u_X = m/rho             3 div 2 mul 2 add
#   q^2 = u u (accumulated)                                           1 mul 1 add
#   H_X = (E + p)/rho for both nodes                                  2 add 2 div
#   Roe H                                                             2 mul 2 add 1 div
#   c = sqrt((gamma - 1)(H - 0.5 q^2))                                2 mul 1 add 1 sqrt
#   b1 = (gamma - 1)/c^2, b2 = 0.5 q^2 b1                             3 mul 1 div
#   right eigenvectors: u - c, u + c, H - u c, 0.5 q^2, H + u c       3 mul 4 add
#   left eigenvectors: 0.5 (b2 +- u/c) (2 div 2 add 2 mul), 1 - b2 (1 add),
#     1/c (1 div), 0.5 (-b1 u -+ 1/c) (6 mul 2 add), b1 u (1 mul),
#     0.5 b1, -b1, 0.5 b1 (3 mul)                                     3 div 5 add 12 mul
EIG1 = _ops(add=21, mul=35, div=12, sqrt=3)
# projection of six nodes and back-projection of two states, nv = 3
PROJ1 = _ops(add=6 * 9, mul=6 * 9)
BACK1 = _ops(add=2 * 9, mul=2 * 9)
# eq. 32: u = m/rho, q^2 (1 mul 1 add), p (3 mul 1 add), F_1 = m u + p
# (1 mul 1 add), F_2 = (E + p) u (1 add 1 mul)
FLUX1 = _ops(add=4, mul=6, div=1)
# |u| + c: q^2 from (m/rho)^2 (2 div 1 mul 1 add), p (3 mul 1 add),
# c = sqrt(gamma p / rho) (1 mul 1 div 1 sqrt), |m/rho| + c (1 div 1 add)
SPEED1 = _ops(add=3, mul=5, div=4, sqrt=1)
# local Lax-Friedrichs: 0.5 (FL + FR) - 0.5 alpha (UR - UL) per variable
LLF1 = _ops(add=9, mul=9)


def test_op_count_of_one_midpoint_flux(ora):
    P = ora.Problem(system="euler", ndim=1, n=(16,), weights="fe", xi=100.0)
    nodes = np.array([[1.0, 0.1, 2.5]] * 3 + [[0.2, 0.0, 0.3]] * 3)
    interp = _plus(IS, Z, FE, CAND, COMB)
    expect = _plus(EIG1, PROJ1, interp, BACK1, FLUX1, SPEED1, LLF1, times=[1, 1, 6, 1, 2, 2, 1])
    assert P.count_midpoint_flux_ops(nodes) == expect


@pytest.mark.parametrize("bc,diff", [("transmissive", "mnd6"), ("periodic", "md6")])
def test_op_count_of_a_residual_is_the_sum_of_its_parts(ora, W, bc, diff):
    """One 1D residual of N nodes: N + 2G - 5 midpoint fluxes per line, N + 2
    node fluxes, and per node and variable the difference (MND6: three
    differences, three products, two sums, / h and the accumulation into R;
    MD6 the same count)."""
    N = 40
    G = 5 if diff == "md6" else 4
    _, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, N)
    P = ora.Problem(system="euler", ndim=1, n=(N,), h=(1.0 / (N - 1),), weights="fe", xi=100.0,
                    bc=bc, diff=diff)
    mid = P.count_midpoint_flux_ops(np.array([[1.0, 0.1, 2.5]] * 3 + [[0.2, 0.0, 0.3]] * 3))
    diffop = _ops(add=6, mul=3, div=1)
    expect = _plus(mid, FLUX1, diffop, times=[N + 2 * G - 5, N + 2, 3 * N])
    assert P.count_residual_ops(U) == expect


def test_run_dt_sequence_is_the_steps_it_lists(ora, W):
    """The oracle driven by a given step sequence (zeros skipped) is the
    same as its single steps of those sizes."""
    prob, U, _ = W.shock_tube(1.0, 0.75, 1.0, 0.125, 0.0, 0.1, 100)
    O = ora.Problem(**prob, weights="fe", xi=100.0)
    dts = [1e-3, 0.0, 7e-4, 1.2e-3]
    ref = U.copy()
    for dt in dts:
        if dt > 0:
            ref, _ = O.rk3_step(ref, dt)
    got, bad = O.run_dt_sequence(U, dts)
    assert bad == 0 and np.array_equal(got, ref)
