"""The paper's 1D Euler test problems (Sec. 4.2) on the GPU.

Sod and Lax (eq. 33-34, shock tubes), Shu-Osher and Titarev-Toro (eq. 35-36,
a shock running into a density wave), with the four-stage Runge-Kutta scheme
of eq. 16 at CFL 0.3 and eps = 1e-40, as in the paper, on the paper's point
counts (201; 2001 for Titarev-Toro).  ``compare`` runs each weight choice and
measures the L1 density distance from a run on ten times as many intervals
(the paper's reference solutions are such finer runs), sampled at the coarse
nodes.  Every step runs in the HIP library.

    python -m paper_2306_09760_amd.paper_problems --problem shu_osher
    python -m paper_2306_09760_amd.paper_problems --stats      # App. A tables
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import workloads as W
from ._lib import WCNSError
from .solver import Plan


def run(name, weights="fe", n=None, xi=100.0, cfl=0.3, method="rk4", t_end=None, device="cuda",
        scheme="wcns"):
    """March problem ``name`` to its end time (or ``t_end``) with the WCNS or
    the filtered embedded WENO (App. B) scheme.  Returns (x, U, steps) with U
    the final conservative state on the host."""
    prob, U, meta = W.paper_problem(name, n)
    P = Plan(device=device, **prob, weights=weights, xi=xi, scheme=scheme)
    Ud = torch.from_numpy(U).to(P.device)
    status = torch.zeros(1, dtype=torch.int32, device=P.device)
    steps, _ = P.run_to_time(Ud, meta["t_end"] if t_end is None else t_end, cfl=cfl,
                             method=method, status=status)
    if int(status.item()) != 0:
        raise WCNSError(f"{name}: a stage produced a non-physical state")
    return meta["x"], Ud.cpu().numpy(), steps


def compare(name, weights=("js", "z", "fe", "pfe"), n=None, ref_factor=10, xi=100.0,
            device="cuda", scheme="wcns"):
    """L1 density distance of each weight choice from a WCNS-FE run on
    ``ref_factor`` times as many intervals (coarse nodes coincide with every
    ref_factor-th fine node)."""
    n = W.PAPER_1D[name]["n"] if n is None else n
    nref = (n - 1) * ref_factor + 1
    _, Uref, _ = run(name, "fe", nref, xi=xi, device=device)
    rho_ref = Uref[0, ::ref_factor]
    out = {"problem": name, "scheme": scheme, "points": n, "reference_points": nref, "schemes": {}}
    for wname in weights:
        x, U, steps = run(name, wname, n, xi=xi, device=device, scheme=scheme)
        out["schemes"][wname] = {"l1_density": float(np.mean(np.abs(U[0] - rho_ref))),
                                 "steps": steps}
    return out


def _ideal_bins(weights, xi, cv, nbins, device):
    """Bins of the ideal region per kind: the weights of every interpolation
    on a uniform state (omega_k = d_k exactly) under this plan."""
    prob, U, _ = W.shock_tube(1.0, 0.0, 1.0, 1.0, 0.0, 1.0, 16)
    P = Plan(device=device, **prob, weights=weights, xi=xi, cv=cv)
    h = P.weight_histogram(torch.from_numpy(U).to(P.device), nbins=nbins).cpu().numpy()
    return [[int(np.flatnonzero(h[kind, k])[0]) for k in range(3)] for kind in range(3)]


def weight_statistics(name, cv=0.0, n=None, nbins=10000, xi=100.0, device="cuda"):
    """App. A statistics: run problem ``name`` with FE weights (cv = 0) or
    PFE weights with switch width cv, and histogram the weights of every
    interpolation of the residual evaluated at the start of every step
    (``nbins`` bins on [0, 1]).  Returns the probability of the ideal region
    for the Z weights, their FE images and the weights used, with the run's
    wall time.  The ideal region of a weight set is the bin that the ideal
    weights d_k fall in under that set's map: d_k itself for the Z weights,
    g_k(d) / sum_l g_l(d) for the FE images (the same bin at large xi, where
    g_k(d_k) = d_k; at xi = 100 the map moves d_0 = 1/16 to about 0.068),
    and for PFE both (the switch keeps d_k on flat stencils and maps the
    others)."""
    import time
    weights = "fe" if cv == 0.0 else "pfe"
    prob, U, meta = W.paper_problem(name, n)
    P = Plan(device=device, **prob, weights=weights, xi=xi, cv=cv)
    Ud = torch.from_numpy(U).to(P.device)
    hist = torch.zeros((3, 3, nbins), dtype=torch.int64, device=P.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, _ = P.run_to_time(Ud, meta["t_end"], cfl=0.3, method="rk4",
                             before_step=lambda X: P.weight_histogram(X, hist))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h = hist.cpu().numpy()
    total = h[0, 0].sum()
    bins = _ideal_bins(weights, xi, cv, nbins, device)
    fe_bins = _ideal_bins("fe", xi, 0.0, nbins, device)[1]
    out = {}
    for i, kind in enumerate(("z", "fe_mapped", "used")):
        ps = []
        for k in range(3):
            b = {bins[i][k]}
            if kind == "used" and weights == "pfe":
                b.add(fe_bins[k])
            ps.append(float(sum(h[i, k, bb] for bb in b) / total))
        out[kind] = ps
    return {"problem": name, "cv": cv, "xi": xi, "steps": steps, "interpolations": int(total),
            "p_ideal": out, "ideal_bins": bins, "wall_s": wall}


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--problem", default="all", choices=["all", *W.PAPER_1D])
    ap.add_argument("--weights", default="js,z,fe,pfe")
    ap.add_argument("--xi", type=float, default=100.0)
    ap.add_argument("--scheme", default="wcns", choices=["wcns", "weno"],
                    help="WCNS (Sec. 2) or the filtered embedded WENO of App. B")
    ap.add_argument("--stats", action="store_true",
                    help="App. A weight statistics for c_v = 0, 1e-4, 1e-3, 1e-2 instead "
                         "(at --xi; 1e6 reproduces the map's control values exactly)")
    args = ap.parse_args()
    names = list(W.PAPER_1D) if args.problem == "all" else [args.problem]
    for name in names:
        if args.stats:
            for cv in (0.0, 1e-4, 1e-3, 1e-2):
                print(json.dumps(weight_statistics(name, cv, xi=args.xi)), flush=True)
        else:
            print(json.dumps(compare(name, tuple(args.weights.split(",")), xi=args.xi,
                                     scheme=args.scheme)), flush=True)


if __name__ == "__main__":
    main()
