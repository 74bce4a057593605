"""Exact solution of the 1D Euler Riemann problem (test infrastructure).

Textbook construction (star-region pressure from the shock / rarefaction
pressure functions, solved by Newton iteration, then sampling of the
self-similar solution), written from the gas-dynamics mathematics; the
WCNS-FE paper does not contain it.  Used only to pin the oracle on shock
tubes; vacuum generation is rejected.
"""
from __future__ import annotations

import numpy as np


def _pressure_fn(p, rho, pk, ck, g):
    """f_K(p) and f_K'(p) for one side."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = np.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rhoL, uL, pL, rhoR, uR, pR, gamma=1.4, tol=1e-14, maxit=200):
    g = gamma
    cL = np.sqrt(g * pL / rhoL)
    cR = np.sqrt(g * pR / rhoR)
    if 2.0 * (cL + cR) / (g - 1.0) <= uR - uL:
        raise ValueError("the data generate vacuum")
    # two-rarefaction initial guess
    z = (g - 1.0) / (2.0 * g)
    p = ((cL + cR - 0.5 * (g - 1.0) * (uR - uL)) / (cL / pL ** z + cR / pR ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(maxit):
        fL, dL = _pressure_fn(p, rhoL, pL, cL, g)
        fR, dR = _pressure_fn(p, rhoR, pR, cR, g)
        pn = p - (fL + fR + uR - uL) / (dL + dR)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _pressure_fn(p, rhoL, pL, cL, g)
    fR, _ = _pressure_fn(p, rhoR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def sample(x, t, x0, rhoL, uL, pL, rhoR, uR, pR, gamma=1.4):
    """Primitive (rho, u, p) at positions x (array) at time t > 0."""
    g = gamma
    ps, us = star_state(rhoL, uL, pL, rhoR, uR, pR, g)
    cL = np.sqrt(g * pL / rhoL)
    cR = np.sqrt(g * pR / rhoR)
    s = (np.asarray(x, dtype=np.float64) - x0) / t
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    gm = (g - 1.0) / (g + 1.0)
    for k, S in enumerate(s):
        if S <= us:  # left of the contact
            if ps > pL:  # left shock
                SL = uL - cL * np.sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g))
                if S <= SL:
                    rho[k], u[k], p[k] = rhoL, uL, pL
                else:
                    rho[k] = rhoL * (ps / pL + gm) / (gm * ps / pL + 1.0)
                    u[k], p[k] = us, ps
            else:  # left rarefaction
                cs = cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
                SH, ST = uL - cL, us - cs
                if S <= SH:
                    rho[k], u[k], p[k] = rhoL, uL, pL
                elif S >= ST:
                    rho[k] = rhoL * (ps / pL) ** (1.0 / g)
                    u[k], p[k] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * (uL - S))
                    u[k] = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * uL + S)
                    rho[k] = rhoL * (c / cL) ** (2.0 / (g - 1.0))
                    p[k] = pL * (c / cL) ** (2.0 * g / (g - 1.0))
        else:  # right of the contact
            if ps > pR:  # right shock
                SR = uR + cR * np.sqrt((g + 1.0) / (2.0 * g) * ps / pR + (g - 1.0) / (2.0 * g))
                if S >= SR:
                    rho[k], u[k], p[k] = rhoR, uR, pR
                else:
                    rho[k] = rhoR * (ps / pR + gm) / (gm * ps / pR + 1.0)
                    u[k], p[k] = us, ps
            else:  # right rarefaction
                cs = cR * (ps / pR) ** ((g - 1.0) / (2.0 * g))
                SH, ST = uR + cR, us + cs
                if S >= SH:
                    rho[k], u[k], p[k] = rhoR, uR, pR
                elif S <= ST:
                    rho[k] = rhoR * (ps / pR) ** (1.0 / g)
                    u[k], p[k] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * (uR - S))
                    u[k] = 2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * uR + S)
                    rho[k] = rhoR * (c / cR) ** (2.0 / (g - 1.0))
                    p[k] = pR * (c / cR) ** (2.0 * g / (g - 1.0))
    return rho, u, p
