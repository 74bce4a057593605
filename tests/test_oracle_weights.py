"""Pins of the oracle's interpolation, weights and FE mapping against what the
paper fixes (Sec. 2 eq. 5-15, Sec. 3.1 eq. 17-21 and Table 1)."""
import numpy as np
import pytest
import sympy as sp

D_IDEAL = np.array([1 / 16, 10 / 16, 5 / 16])


def _interp(ora, weights, u, **kw):
    P = ora.Problem(system="advection", ndim=1, n=(16,), weights=weights, **kw)
    return P.interpolate(np.asarray(u, dtype=np.float64))


def test_linear_weights_reproduce_lagrange_midpoint(ora):
    """Ideal weights combine the eq. 5 candidates into the unique quartic
    through the five nodes, evaluated at the midpoint (exact for quartics)."""
    x = np.arange(-2, 3, dtype=np.float64)
    # Lagrange weights at x = 1/2, computed from the Vandermonde system.
    V = np.vander(x, 5, increasing=True).T
    lag = np.linalg.solve(V, 0.5 ** np.arange(5))
    assert np.allclose(lag * 128, [3, -20, 90, 60, -5], atol=1e-12)
    rng = np.random.default_rng(1)
    for _ in range(5):
        c = rng.standard_normal(5)
        u = np.polyval(c[::-1], x)
        exact = np.polyval(c[::-1], 0.5)
        v, _, w = _interp(ora, "linear", u)
        assert abs(v - exact) < 1e-12 * (1 + abs(exact))
        assert np.allclose(w, D_IDEAL, rtol=0, atol=0)


@pytest.mark.parametrize("weights", ["js", "z"])
@pytest.mark.parametrize("case,jump_at,limit", [
    # Table 1 "original" values: a jump inside a sub-stencil zeroes its weight
    # and the others keep their ideal ratio (eq. 17).
    ("case1", 0, (0.0, 2 / 3, 1 / 3)),
    ("case2", 1, (0.0, 0.0, 1.0)),
    ("case3", 3, (1.0, 0.0, 0.0)),
    ("case4", 4, (1 / 11, 10 / 11, 0.0)),
])
def test_base_weights_reach_table1_original_values(ora, weights, case, jump_at, limit):
    # Case_1: jump in [x_{i-2}, x_{i-1}] -> shift u_{i-2}; Case_2: [x_{i-1}, x_i]
    # -> shift u_{i-2}, u_{i-1}; Case_3: [x_i, x_{i+1}] -> shift u_{i+1}, u_{i+2};
    # Case_4: [x_{i+1}, x_{i+2}] -> shift u_{i+2}.
    u = np.array([0.10, 0.20, 0.30, 0.40, 0.50])
    if case == "case1":
        u[0] += 1e4
    elif case == "case2":
        u[:2] += 1e4
    elif case == "case3":
        u[3:] += 1e4
    else:
        u[4] += 1e4
    _, wb, _ = _interp(ora, weights, u)
    assert np.allclose(wb, limit, atol=1e-9), (case, wb)


@pytest.mark.parametrize("weights", ["js", "z", "fe"])
def test_smooth_linear_data_gives_ideal_weights(ora, weights):
    # On linear data all three IS are equal, so JS and Z return d exactly
    # and FE maps d to itself (Table 1, Case_0).
    u = 0.3 + 0.7 * np.arange(5.0)
    _, wb, wo = _interp(ora, weights, u, xi=1e6)
    assert np.allclose(wb, D_IDEAL, atol=1e-15)
    assert np.allclose(wo, D_IDEAL, atol=1e-15)


# ---- eq. 20 mapping: control points and values (Table 1) ----------------------
CONTROL = [
    (0, 1 / 16, 1 / 16), (1, 10 / 16, 10 / 16), (2, 5 / 16, 5 / 16),   # Case_0
    (1, 2 / 3, 1 / 2), (2, 1 / 3, 1 / 2),                                # Case_1
    (0, 1 / 11, 1 / 6), (1, 10 / 11, 5 / 6),                             # Case_4
    (0, 0.0, 0.0), (1, 0.0, 0.0), (2, 0.0, 0.0),                         # zeroed weights
    (0, 1.0, 1.0), (2, 1.0, 1.0),                                        # Case_3 / Case_2
]


@pytest.mark.parametrize("i,w,g", CONTROL)
def test_fe_map_hits_control_values_at_large_xi(ora, i, w, g):
    assert ora.fe_map(i, w, 1e6, 0.5) == pytest.approx(g, abs=2e-16)


def _sharp_limit(i, w):
    """Piecewise limit of eq. 20 as xi -> infinity: between two adjacent null
    points kappa*(psi_j + psi_{j-1}) (kappa = 1/2) the map is flat at the
    control value; outside the band it is the identity (Sec. 3.1)."""
    bands = {
        0: [(1 / 32, 27 / 352, 1 / 16), (27 / 352, 6 / 11, 1 / 6)],
        1: [(5 / 16, 31 / 48, 5 / 8), (31 / 48, 26 / 33, 1 / 2), (26 / 33, 21 / 22, 5 / 6)],
        2: [(5 / 32, 31 / 96, 5 / 16), (31 / 96, 2 / 3, 1 / 2)],
    }[i]
    for lo, hi, v in bands:
        if lo < w < hi:
            return v
    return w


@pytest.mark.parametrize("i", [0, 1, 2])
def test_fe_map_sharp_limit_shape(ora, i):
    ws = np.linspace(0.0, 1.0, 2001)
    for w in ws:
        lim = _sharp_limit(i, w)
        # stay away from the null points where the step is resolved at width 1/xi
        nulls = {0: [1 / 32, 27 / 352, 6 / 11], 1: [5 / 16, 31 / 48, 26 / 33, 21 / 22],
                 2: [5 / 32, 31 / 96, 2 / 3]}[i]
        if min(abs(w - n) for n in nulls) < 1e-4:
            continue
        assert ora.fe_map(i, w, 1e6, 0.5) == pytest.approx(lim, abs=1e-13), (i, w)


def test_fe_map_xi100_misses_control_values(ora):
    """At the paper's xi = 100 the map does not reach its control values;
    checked against the same map evaluated in 40-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 40
    tab = {0: ([None, "1/16", "1/6", None], ["0", "1/16", "1/11", "1"]),
           1: ([None, "10/16", "1/2", "5/6", None], ["0", "10/16", "2/3", "10/11", "1"]),
           2: ([None, "5/16", "1/2", None], ["0", "5/16", "1/3", "1"])}

    def g_mp(i, w):
        om, ps = tab[i]
        w = mp.mpf(w)
        tot = w
        for j in range(1, len(om)):
            wj = w if om[j] is None else mp.mpf(sp.Rational(om[j]))
            wjm = w if om[j - 1] is None else mp.mpf(sp.Rational(om[j - 1]))
            nu = mp.mpf("0.5") * (mp.mpf(sp.Rational(ps[j])) + mp.mpf(sp.Rational(ps[j - 1])))
            tot += (wj - wjm) / 2 * mp.tanh(100 * (w - nu))
        return tot

    for i, w in [(0, 1 / 16), (0, 0.0), (1, 2 / 3), (2, 1 / 3), (0, 1 / 11), (1, 10 / 11)]:
        ref = float(g_mp(i, w))
        assert ora.fe_map(i, w, 100.0, 0.5) == pytest.approx(ref, abs=1e-15)
    assert abs(ora.fe_map(0, 1 / 16, 100.0, 0.5) - 1 / 16) > 5e-3


# ---- eq. 18: truncation error of the embedded transition cases ---------------
def _eq18(case, h, x0):
    """Leading terms of eq. 18 as f(x_{i+1/2}) - u_hat, f = sin(x + 0.3)."""
    d = {k: sp.diff(sp.sin(sp.Symbol("x") + sp.Rational(3, 10)), sp.Symbol("x"), k)
         for k in (3, 4, 5, 6)}
    f = {k: float(d[k].subs(sp.Symbol("x"), x0)) for k in d}
    return {
        "case0": 3 * h ** 5 * f[5] / 256 + h ** 6 * f[6] / 1024,
        "case1": 3 * h ** 4 * f[4] / 128 + 3 * h ** 5 * f[5] / 256,
        "case4": -5 * h ** 4 * f[4] / 128 + 3 * h ** 5 * f[5] / 256,
    }[case]


@pytest.mark.parametrize("case", ["case0", "case1", "case4"])
def test_eq18_truncation_error_of_fe_at_transition_points(ora, case):
    """FE (xi = 1e6, p = 2) on sin data with a large jump in the sub-stencil
    the case names reproduces the case's truncation error of eq. 18: the
    mapped weights (0, 1/2, 1/2) and (1/6, 5/6, 0) make it fourth order."""
    x0 = 0.0
    errs = []
    for h in (0.04, 0.02, 0.01):
        xs = x0 + h * np.arange(-2, 3)
        u = np.sin(xs + 0.3)
        if case == "case1":
            u[0] += 1e3
        elif case == "case4":
            u[4] += 1e3
        v, _, w = _interp(ora, "fe", u, xi=1e6)
        err = np.sin(x0 + 0.5 * h + 0.3) - v
        lead = _eq18(case, h, x0)
        errs.append((h, err, lead))
        # agreement up to the next order (h^6 or h^7 terms)
        tol = 3 * h ** (6 if case != "case0" else 7)
        assert abs(err - lead) < tol, (case, h, err, lead)
    # and the order itself
    (h1, e1, _), (h2, e2, _) = errs[0], errs[-1]
    order = np.log(abs(e1) / abs(e2)) / np.log(h1 / h2)
    assert order == pytest.approx(5.0 if case == "case0" else 4.0, abs=0.15)


def test_z_weights_are_third_order_at_case1(ora):
    """Unmapped Z weights (0, 2/3, 1/3) at Case_1 lose an order (h^3)."""
    errs = []
    for h in (0.02, 0.01, 0.005):
        xs = h * np.arange(-2, 3)
        u = np.sin(xs + 0.3)
        u[0] += 1e3
        v, _, _ = _interp(ora, "z", u)
        errs.append(abs(np.sin(0.5 * h + 0.3) - v))
    order = np.log(errs[0] / errs[-1]) / np.log(4.0)
    assert order == pytest.approx(3.0, abs=0.15)


@pytest.mark.parametrize("weights", ["js", "z", "fe", "pfe"])
def test_weights_sum_to_one_and_lie_in_unit_interval(ora, weights):
    rng = np.random.default_rng(7)
    for _ in range(200):
        u = rng.standard_normal(5) * 10 ** rng.uniform(-3, 3)
        _, wb, wo = _interp(ora, weights, u, xi=100.0)
        assert abs(wo.sum() - 1.0) < 1e-14
        assert (wo >= -1e-15).all() and (wo <= 1 + 1e-15).all()


def test_pfe_keeps_z_weights_inside_band_and_maps_outside(ora):
    # smooth data: Z weights within c_v of d -> kept (equal to base)
    u = np.sin(0.01 * np.arange(5.0))
    _, wb, wo = _interp(ora, "pfe", u, xi=100.0, cv=1e-3)
    assert np.all(np.abs(wb - D_IDEAL) <= 1e-3)
    assert np.array_equal(wb, wo)
    # a jump: outside the band -> FE weights
    u2 = np.array([0.0, 0.0, 0.0, 0.0, 1.0])
    _, wb2, wo2 = _interp(ora, "pfe", u2, xi=100.0, cv=1e-3)
    _, _, wfe = _interp(ora, "fe", u2, xi=100.0)
    assert np.array_equal(wo2, wfe)
    assert not np.array_equal(wb2, wo2)
