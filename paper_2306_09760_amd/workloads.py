"""Seeded synthetic inputs for the WCNS-FE residual workloads.

This module only draws initial data (numpy ``Generator(PCG64(seed))``) and
converts primitive to conservative variables; it holds none of the scheme's
arithmetic.  Both the GPU path and the CPU oracle take their inputs from here.

All states are float64, variable-major and C-contiguous:
``(nv, nx)`` in 1D, ``(nv, ny, nx)`` in 2D, ``(nv, nz, ny, nx)`` in 3D, with
Euler variables ``(rho, rho*u, rho*v, rho*w, E)`` truncated to ``ndim + 2``.

Grid convention: a periodic axis of length L with N nodes has h = L/N and
nodes x_j = x0 + j*h; a transmissive axis has N nodes including both ends,
h = L/(N-1).
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def prim_to_cons(rho, vel, p, gamma=GAMMA):
    """(rho, [u, v, w], p) -> (rho, rho*u.., E); arrays broadcast together."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.asarray(v, dtype=np.float64) for v in vel]
    ke = 0.5 * rho * sum(v * v for v in vel)
    E = np.asarray(p, dtype=np.float64) / (gamma - 1.0) + ke
    return np.stack([rho * np.ones_like(E)] + [rho * v for v in vel] + [E]).astype(np.float64)


def node_coords(n, length, x0, periodic):
    h = length / n if periodic else length / (n - 1)
    return x0 + h * np.arange(n), h


# ---------------------------------------------------------------- config 1 --
def advection_sine(seed=0, n=200):
    """u0 = a sin(pi x + phi) on periodic [-1, 1], a ~ U[0.5, 1.5],
    phi ~ U[0, 2 pi); advection speed 1."""
    g = rng(seed)
    a = g.uniform(0.5, 1.5)
    phi = g.uniform(0.0, 2.0 * np.pi)
    x, h = node_coords(n, 2.0, -1.0, True)
    U = (a * np.sin(np.pi * x + phi))[None, :].copy()
    prob = dict(system="advection", ndim=1, n=(n,), h=(h,), adv=(1.0,), bc="periodic")
    return prob, U, dict(a=a, phi=phi, x=x)


# ---------------------------------------------------------------- config 2 --
def _draw_tube_states(g, gamma):
    """Left/right (rho, u, p): rho, p log-uniform in [0.1, 10], u ~ U[-1, 1].
    Draws whose rarefactions come within a factor two of forming vacuum
    (u_R - u_L > (a_L + a_R) / (gamma - 1)) are drawn again."""
    while True:
        rho = np.exp(g.uniform(np.log(0.1), np.log(10.0), size=2))
        p = np.exp(g.uniform(np.log(0.1), np.log(10.0), size=2))
        u = g.uniform(-1.0, 1.0, size=2)
        a = np.sqrt(gamma * p / rho)
        if u[1] - u[0] <= (a[0] + a[1]) / (gamma - 1.0):
            return rho, u, p


def shock_tube_batch(seed=0, nprob=4096, nmin=256, nmax=4096, gamma=GAMMA):
    """Ragged batch of independent 1D Euler shock tubes on [0, 1], jump at
    x = 0.5 (x <= 0.5 takes the left state), transmissive ends.

    Returns (prob, U, meta): ``U`` is (3, total) with problem p occupying
    columns offsets[p]:offsets[p+1]; meta has lengths, offsets, h, states."""
    g = rng(seed)
    lengths = g.integers(nmin, nmax + 1, size=nprob)
    offsets = np.zeros(nprob + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    total = int(offsets[-1])
    U = np.empty((3, total), dtype=np.float64)
    hs = np.empty(nprob)
    states = np.empty((nprob, 2, 3))
    for p in range(nprob):
        rho, u, pr = _draw_tube_states(g, gamma)
        N = int(lengths[p])
        x, h = node_coords(N, 1.0, 0.0, False)
        left = x <= 0.5
        U[:, offsets[p]:offsets[p + 1]] = prim_to_cons(
            np.where(left, rho[0], rho[1]), [np.where(left, u[0], u[1])],
            np.where(left, pr[0], pr[1]), gamma)
        hs[p] = h
        states[p, 0] = (rho[0], u[0], pr[0])
        states[p, 1] = (rho[1], u[1], pr[1])
    prob = dict(system="euler", ndim=1, bc="transmissive", gamma=gamma)
    return prob, U, dict(lengths=lengths, offsets=offsets, h=hs, states=states)


def shock_tube(rhoL, uL, pL, rhoR, uR, pR, n, length=1.0, x_jump=0.5, gamma=GAMMA):
    """A single 1D shock tube (x <= x_jump takes the left state)."""
    x, h = node_coords(n, length, 0.0, False)
    left = x <= x_jump
    U = prim_to_cons(np.where(left, rhoL, rhoR), [np.where(left, uL, uR)],
                     np.where(left, pL, pR), gamma)
    prob = dict(system="euler", ndim=1, n=(n,), h=(h,), bc="transmissive", gamma=gamma)
    return prob, U, dict(x=x)


# ------------------------------------------------- the paper's 1D problems --
# Sec. 4.2: initial states as printed (eq. 33-36), transmissive ends, end
# times and point counts of the text (201 points; 2001 for Titarev-Toro).
PAPER_1D = {
    "sod": dict(domain=(0.0, 10.0), x_jump=5.0, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
                t_end=2.0, n=201),
    "lax": dict(domain=(0.0, 1.0), x_jump=0.5, left=(0.445, 0.698, 3.528),
                right=(0.5, 0.0, 0.571), t_end=0.15, n=201),
    "shu_osher": dict(domain=(0.0, 10.0), x_jump=1.0, left=(3.857143, 2.629369, 10.3333),
                      right="shu_osher", t_end=1.8, n=201),
    "titarev_toro": dict(domain=(0.0, 10.0), x_jump=3.5, left=(1.515695, 0.523346, 1.805),
                         right="titarev_toro", t_end=4.0, n=2001),
}


def paper_problem(name, n=None, gamma=GAMMA):
    """One of the paper's 1D Euler problems (Sec. 4.2, eq. 33-36) on n points
    (default: the paper's).  x <= x_jump takes the left state.  Returns
    (prob, U, meta) with meta = {x, t_end}."""
    c = PAPER_1D[name]
    n = c["n"] if n is None else n
    x0, x1 = c["domain"]
    x, h = node_coords(n, x1 - x0, x0, False)
    left = x <= c["x_jump"]
    rl, ul, pl = c["left"]
    if c["right"] == "shu_osher":
        rr, ur, pr = 1.0 + 0.2 * np.sin(5.0 * x), 0.0, 1.0
    elif c["right"] == "titarev_toro":
        rr, ur, pr = 1.0 + 0.1 * np.sin(20.0 * np.pi * x), 0.0, 1.0
    else:
        rr, ur, pr = c["right"]
    rho = np.where(left, rl, rr)
    u = np.where(left, ul, ur)
    p = np.where(left, pl, pr)
    U = prim_to_cons(rho, [u], p, gamma)
    prob = dict(system="euler", ndim=1, n=(n,), h=(h,), bc="transmissive", gamma=gamma)
    return prob, np.ascontiguousarray(U), dict(x=x, t_end=c["t_end"])


# ---------------------------------------------------------------- config 3 --
def riemann2d(seed=0, n=2048, split=0.8, gamma=GAMMA):
    """Four-quadrant 2D Riemann problem on [0, 1]^2, quadrant lines x = y =
    split (x >= split is east, y >= split is north); each quadrant's
    (rho, u, v, p) drawn with rho, p log-uniform in [0.1, 10] and u, v
    uniform in [-1, 1]; transmissive boundaries."""
    g = rng(seed)
    q = np.empty((4, 4))
    while True:
        for k in range(4):
            q[k, 0] = np.exp(g.uniform(np.log(0.1), np.log(10.0)))
            q[k, 1:3] = g.uniform(-1.0, 1.0, size=2)
            q[k, 3] = np.exp(g.uniform(np.log(0.1), np.log(10.0)))
        a = np.sqrt(gamma * q[:, 3] / q[:, 0])
        # quadrants: 0 = NE, 1 = NW, 2 = SW, 3 = SE; reject draws whose
        # interfaces come within a factor two of forming vacuum.
        ok = True
        for (l, r, ax) in ((1, 0, 1), (2, 3, 1), (2, 1, 2), (3, 0, 2)):
            if q[r, ax] - q[l, ax] > (a[l] + a[r]) / (gamma - 1.0):
                ok = False
        if ok:
            break
    x, h = node_coords(n, 1.0, 0.0, False)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X[y, x]
    east = X >= split
    north = Y >= split
    quad = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
    prim = q[quad]  # (ny, nx, 4)
    U = prim_to_cons(prim[..., 0], [prim[..., 1], prim[..., 2]], prim[..., 3], gamma)
    prob = dict(system="euler", ndim=2, n=(n, n), h=(h, h), bc="transmissive", gamma=gamma)
    return prob, np.ascontiguousarray(U), dict(quadrants=q)


# ---------------------------------------------------------------- config 4 --
def turbulence3d(seed=0, n=256, mach=0.6, k_peak=8.0, gamma=GAMMA):
    """Decaying compressible turbulence on the periodic box [0, 2 pi)^3:
    solenoidal random velocity with energy spectrum E(k) ~ k^4
    exp(-2 (k / k_peak)^2), scaled to rms |u| = 1; rho = 1 and
    p = 1 / (gamma mach^2) so that the rms Mach number is ``mach``."""
    g = rng(seed)
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    kmag = np.sqrt(k2)
    with np.errstate(divide="ignore", invalid="ignore"):
        # |u_hat|^2 ~ E(k) / (4 pi k^2) in 3D
        amp = np.where(k2 > 0, np.sqrt(kmag ** 2 * np.exp(-2.0 * (kmag / k_peak) ** 2)), 0.0)
    uh = []
    for _ in range(3):
        uh.append(amp * (g.standard_normal(k2.shape) + 1j * g.standard_normal(k2.shape)))
    # Project out the component along k (solenoidal field).
    with np.errstate(divide="ignore", invalid="ignore"):
        kdotu = KX * uh[0] + KY * uh[1] + KZ * uh[2]
        inv = np.where(k2 > 0, 1.0 / k2, 0.0)
    uh = [uh[0] - KX * kdotu * inv, uh[1] - KY * kdotu * inv, uh[2] - KZ * kdotu * inv]
    vel = [np.real(np.fft.ifftn(c)) for c in uh]  # indexed [z, y, x]
    rms = np.sqrt(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    vel = [v / rms for v in vel]
    rho = np.ones_like(vel[0])
    p = np.full_like(vel[0], 1.0 / (gamma * mach * mach))
    U = prim_to_cons(rho, vel, p, gamma)
    h = 2.0 * np.pi / n
    prob = dict(system="euler", ndim=3, n=(n, n, n), h=(h, h, h), bc="periodic", gamma=gamma)
    return prob, np.ascontiguousarray(U), {}


# ---------------------------------------------------------------- config 5 --
def _fourier_density(g, n, nmodes=16, kmax=4, amp=0.2):
    ks = []
    while len(ks) < nmodes:
        k = tuple(int(v) for v in g.integers(-kmax, kmax + 1, size=2))
        if k != (0, 0):
            ks.append(k)
    a = g.uniform(0.5, 1.0, size=nmodes)
    ph = g.uniform(0.0, 2.0 * np.pi, size=nmodes)
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    S = np.zeros((n, n))
    for (kx, ky), am, p in zip(ks, a, ph):
        S += am * np.cos(2.0 * np.pi * (kx * X + ky * Y) + p)
    return 1.0 + amp * S / np.max(np.abs(S))


def adjoint2d(seed=0, n=1024, gamma=GAMMA, flow_amp=0.0):
    """Smooth periodic 2D Euler state on [0, 1)^2: rho0 = 1 + 0.2 * (sum of
    16 seeded Fourier modes, scaled to max |sum| = 1), u = v = 0.5, p = 1.
    ``target_init`` is the same construction drawn with seed + 1 (to be
    advanced by the same run to form the target).

    With ``flow_amp`` > 0, u, v and p also vary: 0.5 + flow_amp * S_u,
    0.5 + flow_amp * S_v and 1 + flow_amp * S_p, each S a sum of 16 modes
    scaled to max |S| = 1 drawn from seeds seed + 10000 + (0, 1, 2) (seed + 1
    + ... for the target), so that every characteristic field is resolved
    well above rounding."""
    def state(sd):
        rho = _fourier_density(rng(sd), n)
        if flow_amp > 0.0:
            u = 0.5 + (_fourier_density(rng(sd + 10000), n, amp=flow_amp) - 1.0)
            v = 0.5 + (_fourier_density(rng(sd + 10001), n, amp=flow_amp) - 1.0)
            p = _fourier_density(rng(sd + 10002), n, amp=flow_amp)
        else:
            u = np.full((n, n), 0.5)
            v = np.full((n, n), 0.5)
            p = np.ones((n, n))
        return prim_to_cons(rho, [u, v], p, gamma)

    U = state(seed)
    Ut = state(seed + 1)
    h = 1.0 / n
    prob = dict(system="euler", ndim=2, n=(n, n), h=(h, h), bc="periodic", gamma=gamma)
    return prob, np.ascontiguousarray(U), dict(target_init=np.ascontiguousarray(Ut))


def random_smooth_state(seed, ndim, n, nmodes=4, gamma=GAMMA, amp=0.1):
    """A small smooth periodic Euler state with every field perturbed (for
    derivative checks): rho, p around 1, velocities around 0.3."""
    g = rng(seed)
    axes = [np.arange(n[k]) / n[k] for k in range(ndim)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")[::-1]  # grids[k] varies along axis k

    def field(base):
        f = np.full(grids[0].shape, base)
        for _ in range(nmodes):
            kv = g.integers(-2, 3, size=ndim)
            ph = g.uniform(0, 2 * np.pi)
            f = f + amp * g.uniform(0.3, 1.0) * np.cos(
                2 * np.pi * sum(kv[k] * grids[k] for k in range(ndim)) + ph)
        return f

    rho = field(1.0)
    vel = [field(0.3) for _ in range(ndim)]
    p = field(1.0)
    U = prim_to_cons(rho, vel, p, gamma)
    h = tuple(1.0 / v for v in n)
    prob = dict(system="euler", ndim=ndim, n=tuple(n), h=h, bc="periodic", gamma=gamma)
    return prob, np.ascontiguousarray(U)
