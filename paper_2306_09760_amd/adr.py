"""Approximate dispersion relation (ADR) of the scheme (Sec. 3.2, eq. 22-28),
evaluated on the GPU.

For the scalar advection u_t + c u_x = 0 (c = 1, h = 1) on a periodic grid of
n points, each wavenumber alpha_m = 2 pi m / n is represented by the sine wave
u_j = cos(alpha_m j + phase).  The scheme's derivative is u'_j = -R_j (R the
residual), and its modified wavenumber is the ratio of the m-th Fourier
coefficients, k(alpha) = FT(u' h)_m / FT(u)_m = k_r + i k_i (eq. 26-28).
The exact derivative gives k_r = 0, k_i = alpha; k_i is the dispersion and
k_r the dissipation of the (nonlinear) scheme at that wavenumber.

All waves are evaluated in one residual call: they are the rows of a 2D
periodic advection problem with velocity (1, 0), so the y sweep contributes
nothing and every row is an independent 1D line.

    python -m paper_2306_09760_amd.adr            # Fig. 5-6 sweeps of kappa and xi
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from .solver import Plan


def adr(n=128, weights="fe", xi=1e6, kappa=0.5, modes=None, phase=0.0, device="cuda", **kw):
    """Returns (alpha, k_r, k_i) for alpha_m = 2 pi m / n, m in ``modes``
    (default 1 .. n/2)."""
    modes = np.arange(1, n // 2 + 1) if modes is None else np.asarray(modes)
    rows = max(len(modes), 9)                  # the library's minimum line length
    m_rows = np.resize(modes, rows)
    j = np.arange(n)
    alpha_rows = 2.0 * np.pi * m_rows / n
    U = np.cos(alpha_rows[:, None] * j[None, :] + phase)[None].copy()   # (1, rows, n)
    P = Plan(device=device, system="advection", ndim=2, n=(n, rows), h=(1.0, 1.0),
             adv=(1.0, 0.0), bc="periodic", weights=weights, xi=xi, kappa=kappa, **kw)
    R = P.residual(torch.from_numpy(U).to(P.device)).cpu().numpy()[0]
    Fu = np.fft.fft(U[0], axis=1)
    Fd = np.fft.fft(-R, axis=1)
    k = Fd[np.arange(rows), m_rows] / Fu[np.arange(rows), m_rows]
    alpha = 2.0 * np.pi * modes / n
    return alpha, k.real[: len(modes)], k.imag[: len(modes)]


def summary(alpha, kr, ki):
    """Largest dispersion overshoot max(k_i - alpha), the wavenumber where
    k_i departs from alpha by 1 %, and the largest dissipation min(k_r)."""
    dep = np.flatnonzero(np.abs(ki - alpha) > 0.01 * alpha)
    return {"max_dispersion_overshoot": float(np.max(ki - alpha)),
            "alpha_1pct": float(alpha[dep[0]]) if dep.size else float(alpha[-1]),
            "min_kr": float(np.min(kr))}


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--curves", action="store_true", help="print the full k(alpha) curves")
    args = ap.parse_args()
    runs = [dict(weights="linear", xi=1e6, kappa=0.5), dict(weights="js", xi=1e6, kappa=0.5),
            dict(weights="z", xi=1e6, kappa=0.5)]
    runs += [dict(weights="fe", xi=1e6, kappa=k) for k in (0.3, 0.4, 0.5, 0.6)]   # Fig. 5
    runs += [dict(weights="fe", xi=x, kappa=0.5) for x in (10.0, 100.0, 1e3)]       # Fig. 6
    for r in runs:
        a, kr, ki = adr(args.n, **r)
        out = dict(r, **summary(a, kr, ki))
        if args.curves:
            out.update(alpha=a.tolist(), k_r=kr.tolist(), k_i=ki.tolist())
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
