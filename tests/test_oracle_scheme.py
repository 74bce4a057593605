"""Pins of the oracle's residual, eigenvectors, flux difference and SSP-RK3
step against what the paper and the mathematics fix."""
import numpy as np
import pytest

GAMMA = 1.4


# ---------------------------------------------------------------- Euler flux --
def test_flux_satisfies_rankine_hugoniot_for_stationary_shock(ora):
    """A stationary normal shock (textbook Mach relations) has equal fluxes
    on both sides, which pins eq. 32."""
    g = GAMMA
    for M in (1.5, 3.0):
        rho1, p1 = 1.0, 1.0
        u1 = M * np.sqrt(g * p1 / rho1)
        rho2 = rho1 * (g + 1) * M ** 2 / ((g - 1) * M ** 2 + 2)
        p2 = p1 * (1 + 2 * g / (g + 1) * (M ** 2 - 1))
        u2 = rho1 * u1 / rho2

        def cons(r, u, p):
            return np.array([r, r * u, p / (g - 1) + 0.5 * r * u * u])

        F1 = ora.euler_flux(1, 0, g, cons(rho1, u1, p1))
        F2 = ora.euler_flux(1, 0, g, cons(rho2, u2, p2))
        assert np.allclose(F1, F2, rtol=1e-13)
        # and the momentum flux is rho u^2 + p on one side
        assert F1[1] == pytest.approx(rho1 * u1 ** 2 + p1, rel=1e-14)


def _rand_state(rng, nd):
    rho = rng.uniform(0.5, 2.0)
    vel = rng.uniform(-1, 1, nd)
    p = rng.uniform(0.5, 2.0)
    return np.concatenate([[rho], rho * vel, [p / (GAMMA - 1) + 0.5 * rho * vel @ vel]])


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_eigenvectors_diagonalise_the_flux_jacobian(ora, nd):
    """With both states equal, L R = I and L A R = diag(u_d - c, u_d..., u_d + c)
    where A is the flux Jacobian by central differences of the oracle flux."""
    rng = np.random.default_rng(nd)
    for d in range(nd):
        U = _rand_state(rng, nd)
        L, R = ora.eigenvectors(nd, d, GAMMA, U, U)
        nv = nd + 2
        assert np.allclose(L @ R, np.eye(nv), atol=1e-13)
        A = np.zeros((nv, nv))
        for k in range(nv):
            e = np.zeros(nv)
            e[k] = 1e-6 * max(1.0, abs(U[k]))
            A[:, k] = (ora.euler_flux(nd, d, GAMMA, U + e) - ora.euler_flux(nd, d, GAMMA, U - e)) / (2 * e[k])
        rho = U[0]
        u = U[1 + d] / rho
        q2 = np.sum((U[1:1 + nd] / rho) ** 2)
        p = (GAMMA - 1) * (U[-1] - 0.5 * rho * q2)
        c = np.sqrt(GAMMA * p / rho)
        lam = np.array([u - c] + [u] * nd + [u + c])
        assert np.allclose(L @ A @ R, np.diag(lam), atol=1e-7)


def test_roe_average_satisfies_property_u(ora):
    """Roe's average makes A(U_roe) (Ub - Ua) = F(Ub) - F(Ua) (1D), so
    R diag(lam) L (Ub - Ua) equals the flux jump."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        Ua, Ub = _rand_state(rng, 1), _rand_state(rng, 1)
        L, R = ora.eigenvectors(1, 0, GAMMA, Ua, Ub)
        # eigenvalues of the Roe matrix from its eigenvectors: A = R diag L
        sa, sb = np.sqrt(Ua[0]), np.sqrt(Ub[0])
        u = (sa * Ua[1] / Ua[0] + sb * Ub[1] / Ub[0]) / (sa + sb)
        pa = (GAMMA - 1) * (Ua[2] - 0.5 * Ua[1] ** 2 / Ua[0])
        pb = (GAMMA - 1) * (Ub[2] - 0.5 * Ub[1] ** 2 / Ub[0])
        H = (sa * (Ua[2] + pa) / Ua[0] + sb * (Ub[2] + pb) / Ub[0]) / (sa + sb)
        c = np.sqrt((GAMMA - 1) * (H - 0.5 * u * u))
        A = R @ np.diag([u - c, u, u + c]) @ L
        dF = ora.euler_flux(1, 0, GAMMA, Ub) - ora.euler_flux(1, 0, GAMMA, Ua)
        assert np.allclose(A @ (Ub - Ua), dF, rtol=1e-11, atol=1e-12)


# -------------------------------------------------------- difference operator --
def _mnd6_coefficients():
    """(a, b, c) of a(F~_{i+1/2}-F~_{i-1/2}) + b(F_{i+1}-F_{i-1}) +
    c(F~_{i+3/2}-F~_{i-3/2}) from the odd Taylor moments (orders 1, 3, 5)."""
    offs = np.array([0.5, 1.0, 1.5])
    M = np.array([[2 * o ** k for o in offs] for k in (1, 3, 5)])
    return np.linalg.solve(M, [1.0, 0.0, 0.0])


def test_mnd6_coefficients_are_the_unique_sixth_order_choice():
    assert np.allclose(_mnd6_coefficients(), [1.5, -0.3, 1.0 / 30.0], atol=1e-14)


def _symbol(theta, diff="mnd6"):
    """h * (numerical d/dx) / (ik-wave) of the linear upwind scheme: ideal
    weights on the upwind stencil, then the flux difference."""
    x = np.arange(-2, 3, dtype=np.float64)
    lag = np.linalg.solve(np.vander(x, 5, increasing=True).T, 0.5 ** np.arange(5))
    C = sum(lag[k] * np.exp(1j * (k - 2) * theta) for k in range(5))  # F~_{j+1/2} / u_j
    if diff == "mnd6":
        a, b, c = _mnd6_coefficients()
        return (a * C * (1 - np.exp(-1j * theta)) + b * (np.exp(1j * theta) - np.exp(-1j * theta))
                + c * C * (np.exp(1j * theta) - np.exp(-2j * theta)))
    d1, d2, d3 = 75 / 64, -25 / 384, 3 / 640
    return (d1 * C * (1 - np.exp(-1j * theta)) + d2 * C * (np.exp(1j * theta) - np.exp(-2j * theta))
            + d3 * C * (np.exp(2j * theta) - np.exp(-3j * theta)))


@pytest.mark.parametrize("diff", ["mnd6", "md6"])
def test_linear_residual_matches_the_scheme_symbol(ora, diff):
    """On a Fourier mode the residual with ideal weights is -a S(theta)/h u."""
    N, a = 64, 1.0
    h = 2.0 / N
    x = -1 + h * np.arange(N)
    for kw in (1, 3, 7):
        theta = np.pi * kw * h
        u = np.cos(np.pi * kw * x + 0.4)
        P = ora.Problem(system="advection", ndim=1, n=(N,), h=h, adv=(a,), weights="linear", diff=diff)
        R = P.residual(u)
        expect = np.real(-a * _symbol(theta, diff) / h * np.exp(1j * (np.pi * kw * x + 0.4)))
        assert np.allclose(R, expect, atol=1e-11)


# ----------------------------------------------------------- order of accuracy --
@pytest.mark.parametrize("weights,xi,order", [
    ("linear", 1e6, 5.0), ("fe", 1e6, 5.0), ("js", 1e6, 5.0), ("z", 1e6, 5.0), ("fe", 100.0, 3.0)])
def test_smooth_advection_residual_order(ora, weights, xi, order):
    errs = []
    Ns = (80, 160, 320)
    for N in Ns:
        h = 2.0 / N
        x = -1 + h * np.arange(N)
        P = ora.Problem(system="advection", ndim=1, n=(N,), h=h, weights=weights, xi=xi)
        R = P.residual(np.sin(np.pi * x + 0.3))
        errs.append(np.abs(R + np.pi * np.cos(np.pi * x + 0.3)).max())
    rate = np.log(errs[0] / errs[-1]) / np.log(Ns[-1] / Ns[0])
    assert rate == pytest.approx(order, abs=0.3), errs


def test_fe_large_xi_equals_linear_scheme_on_smooth_data(ora):
    N = 200
    h = 0.01
    x = -1 + h * np.arange(N)
    u = np.sin(np.pi * x + 0.3)
    Rl = ora.Problem(system="advection", ndim=1, n=(N,), h=h, weights="linear").residual(u)
    Rf = ora.Problem(system="advection", ndim=1, n=(N,), h=h, weights="fe", xi=1e6).residual(u)
    # the mapped weights equal d up to rounding of the tanh sums
    assert np.abs(Rl - Rf).max() < 1e-12 * np.abs(Rl).max()


# --------------------------------------------------- config 1 closed form (RK3) --
def test_config1_rk3_matches_discrete_closed_form(ora, W):
    """With FE at xi = 1e6 the weights are the ideal ones on this data, so
    400 SSP-RK3 steps give u_j^n = a Im(G^n e^{i(pi x_j + phi)}),
    G = 1 + z + z^2/2 + z^3/6, z = -nu S(pi h)."""
    prob, U0, meta = W.advection_sine(seed=0)
    P = ora.Problem(weights="fe", xi=1e6, **prob)
    U, bad = P.run_steps(U0, 400, dt=0.005)
    assert bad == 0
    h = 0.01
    z = -0.5 * _symbol(np.pi * h)
    G = 1 + z + z * z / 2 + z ** 3 / 6
    x = meta["x"]
    closed = meta["a"] * np.imag(G ** 400 * np.exp(1j * (np.pi * x + meta["phi"])))
    assert np.abs(U[0] - closed).max() < 1e-12
    assert abs(abs(G ** 400) - 1) == pytest.approx(1.018e-6, rel=2e-3)


def test_rk3_step_is_the_ssp_rk3_polynomial(ora):
    """For the linear scheme on one Fourier mode, one step multiplies by
    1 + z + z^2/2 + z^3/6 exactly."""
    N, h = 40, 0.05
    x = h * np.arange(N)
    theta = 2 * np.pi * 3 / N
    u0 = np.cos(2 * np.pi * 3 * x / (N * h))
    P = ora.Problem(system="advection", ndim=1, n=(N,), h=h, weights="linear")
    dt = 0.02
    u1, _ = P.rk3_step(u0, dt)
    z = -(dt / h) * _symbol(theta)
    G = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.allclose(u1, np.real(G * np.exp(1j * 2 * np.pi * 3 * x / (N * h))), atol=1e-13)


def test_rk4_step_is_the_fourth_order_taylor_polynomial(ora):
    """eq. 16 on the linear scheme and one Fourier mode multiplies it by
    1 + z + z^2/2 + z^3/6 + z^4/24 (the stage coefficients of eq. 16 give
    classical RK4)."""
    N, h = 40, 0.05
    x = h * np.arange(N)
    theta = 2 * np.pi * 3 / N
    u0 = np.cos(2 * np.pi * 3 * x / (N * h))
    P = ora.Problem(system="advection", ndim=1, n=(N,), h=h, weights="linear")
    dt = 0.02
    u1, bad = P.rk4_step(u0, dt)
    assert bad == 0
    z = -(dt / h) * _symbol(theta)
    G = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.allclose(u1, np.real(G * np.exp(1j * 2 * np.pi * 3 * x / (N * h))), atol=1e-13)


def test_config1_rk4_matches_discrete_closed_form(ora, W):
    """The config-1 sine with FE at xi = 1e6 (ideal weights on this data) and
    400 steps of eq. 16: u_j^n = a Im(G^n e^{i(pi x_j + phi)}) with the RK4
    amplification factor."""
    prob, U0, meta = W.advection_sine(seed=0)
    P = ora.Problem(weights="fe", xi=1e6, **prob)
    U = U0
    for _ in range(400):
        U, bad = P.rk4_step(U, 0.005)
        assert bad == 0
    z = -0.5 * _symbol(np.pi * 0.01)
    G = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    closed = meta["a"] * np.imag(G ** 400 * np.exp(1j * (np.pi * meta["x"] + meta["phi"])))
    assert np.abs(U[0] - closed).max() < 1e-12


def test_rk4_run_to_time_lands_on_t_end(ora, W):
    prob, U, _ = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 101)
    P = ora.Problem(weights="fe", xi=100.0, **prob)
    U1, steps, t, bad = P.run_to_time(U, 0.05, cfl=0.3, method="rk4")
    assert bad == 0 and t == 0.05 and steps > 10
    # mass is conserved up to the boundary flux of the undisturbed ends
    assert abs(U1[0].sum() - U[0].sum()) < 1e-12 * U[0].sum()


# ------------------------------------------------------------------ invariants --
@pytest.mark.parametrize("weights", ["js", "z", "fe", "pfe"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_periodic_residual_is_conservative(ora, W, weights, ndim):
    n = {1: (48,), 2: (16, 12), 3: (10, 9, 11)}[ndim]
    prob, U = W.random_smooth_state(5, ndim, n)
    U = U.copy()
    # add a density jump so the nonlinear weights are active
    U[0].flat[: U[0].size // 3] *= 1.5
    P = ora.Problem(weights=weights, xi=100.0, **prob)
    R = P.residual(U)
    for v in range(U.shape[0]):
        assert abs(R[v].sum()) < 1e-11 * np.abs(R[v]).sum()


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_constant_state_has_zero_residual(ora, ndim):
    n = {1: (20,), 2: (12, 10), 3: (9, 10, 9)}[ndim]
    nv = ndim + 2
    U = np.empty((nv,) + tuple(reversed(n)))
    rho, p = 1.3, 0.8
    vel = [0.3, -0.2, 0.1][:ndim]
    U[0] = rho
    for k in range(ndim):
        U[1 + k] = rho * vel[k]
    U[-1] = p / (GAMMA - 1) + 0.5 * rho * sum(v * v for v in vel)
    for bc in ("periodic", "transmissive"):
        P = ora.Problem(system="euler", ndim=ndim, n=n, bc=bc, weights="fe", xi=100.0)
        assert np.abs(P.residual(U)).max() < 1e-12


def test_moving_contact_keeps_velocity_and_pressure_uniform(ora, W):
    prob, U, _ = W.shock_tube(2.0, 0.5, 1.0, 1.0, 0.5, 1.0, 101)
    P = ora.Problem(weights="fe", xi=100.0, **prob)
    U1, bad = P.rk3_step(U, 0.002)
    assert bad == 0
    u = U1[1] / U1[0]
    p = (GAMMA - 1) * (U1[2] - 0.5 * U1[1] ** 2 / U1[0])
    assert np.abs(u - 0.5).max() < 1e-13
    assert np.abs(p - 1.0).max() < 1e-13


@pytest.mark.parametrize("weights", ["js", "z", "fe"])
def test_mirror_symmetry(ora, W, weights):
    """Reflecting x -> -x (and u -> -u) reflects the residual; this checks
    that the right-biased state is the mirrored left-biased one."""
    prob, U, _ = W.shock_tube(1.0, 0.3, 1.0, 0.2, -0.4, 0.15, 64)
    rng = np.random.default_rng(0)
    U = U * (1 + 0.05 * rng.standard_normal(U.shape[1]))
    P = ora.Problem(weights=weights, xi=100.0, **prob)
    R = P.residual(U)
    Um = U[:, ::-1].copy()
    Um[1] *= -1
    Rm = P.residual(Um)
    Rm = Rm[:, ::-1]
    Rm[1] *= -1
    assert np.allclose(R, Rm, atol=1e-12 * np.abs(R).max())


def test_2d_rows_match_1d_and_axes_are_interchangeable(ora, W):
    """A 2D state uniform in y gives the 1D residual on every row (and no
    y-momentum residual); transposing x and y transposes the residual."""
    prob1, U1, _ = W.shock_tube(1.0, 0.2, 1.0, 0.3, -0.1, 0.4, 24)
    R1 = ora.Problem(weights="fe", xi=100.0, **prob1).residual(U1)
    ny = 10
    U2 = np.zeros((4, ny, 24))
    U2[0] = U1[0]
    U2[1] = U1[1]
    U2[3] = U1[2]
    P2 = ora.Problem(system="euler", ndim=2, n=(24, ny), h=(prob1["h"][0], 0.1),
                     bc=("transmissive", "periodic"), weights="fe", xi=100.0)
    R2 = P2.residual(U2)
    for j in range(ny):
        assert np.allclose(R2[[0, 1, 3], j], R1, atol=1e-13)
    assert np.abs(R2[2]).max() < 1e-13
    # axis interchange on a genuinely 2D state
    prob, U = W.random_smooth_state(9, 2, (14, 14))
    P = ora.Problem(weights="z", **prob)
    R = P.residual(U)
    Ut = U.transpose(0, 2, 1)[[0, 2, 1, 3]].copy()
    Rt = P.residual(Ut).transpose(0, 2, 1)[[0, 2, 1, 3]]
    assert np.allclose(R, Rt, atol=1e-12 * np.abs(R).max())


# ------------------------------------------------------------ exact Riemann ---
@pytest.mark.slow
def test_sod_converges_to_exact_riemann_solution(ora, W):
    from oracle import exact_riemann as er
    errs = []
    for N in (101, 201, 401):
        prob, U, meta = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, N)
        P = ora.Problem(weights="fe", xi=100.0, **prob)
        U2, steps, t, bad = P.run_to_time(U, 0.2, cfl=0.5)
        assert bad == 0 and t == 0.2
        rho_ex, _, _ = er.sample(meta["x"], 0.2, 0.5, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
        errs.append(np.mean(np.abs(U2[0] - rho_ex)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[-1] < 4e-3


# ------------------------------------------------ dual-number JVP vs differences --
@pytest.mark.parametrize("weights", ["js", "z", "fe", "pfe", "linear"])
@pytest.mark.parametrize("ndim", [1, 2])
def test_dual_jvp_matches_central_differences(ora, W, weights, ndim):
    n = (24,) if ndim == 1 else (12, 10)
    prob, U = W.random_smooth_state(11, ndim, n, amp=0.2)
    P = ora.Problem(weights=weights, xi=100.0, **prob)
    rng = np.random.default_rng(2)
    V = rng.standard_normal(U.shape)
    R, JV = P.residual_jvp(U, V)
    assert np.array_equal(R, P.residual(U))
    # Central differences must converge to the exact JVP for some step; the
    # JS/Z weights are strongly curved where an indicator is tiny (critical
    # points of a characteristic field), so no single step suits every node.
    def cd(eps):
        return (P.residual(U + eps * V) - P.residual(U - eps * V)) / (2 * eps)
    best = min(np.abs(JV - cd(eps)).max() for eps in (1e-5, 1e-6, 1e-7, 1e-8))
    assert best < 1e-7 * np.abs(JV).max()


@pytest.mark.parametrize("ndim", [2, 3])
def test_threaded_residual_equals_one_thread(ora, W, ndim):
    """The lines of a residual may run on several threads: the values (and
    the dual-number tangents) are bitwise those of one thread."""
    n = (24, 20) if ndim == 2 else (12, 10, 9)
    prob, U = W.random_smooth_state(3, ndim, n, amp=0.3)
    U = U.copy()
    U[0].flat[::7] *= 1.4
    V = np.random.default_rng(1).standard_normal(U.shape)
    P = ora.Problem(**prob, weights="fe", xi=100.0)
    try:
        ora.set_threads(1)
        R1 = P.residual(U)
        _, J1 = P.residual_jvp(U, V)
        ora.set_threads(4)
        R4 = P.residual(U)
        _, J4 = P.residual_jvp(U, V)
    finally:
        ora.set_threads(0)
    assert np.array_equal(R1, R4) and np.array_equal(J1, J4)
