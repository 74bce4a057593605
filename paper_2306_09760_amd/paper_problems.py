"""The paper's 1D Euler test problems (Sec. 4.2) on the GPU.

Sod and Lax (eq. 33-34, shock tubes), Shu-Osher and Titarev-Toro (eq. 35-36,
a shock running into a density wave), with the four-stage Runge-Kutta scheme
of eq. 16 at CFL 0.3 and eps = 1e-40, as in the paper, on the paper's point
counts (201; 2001 for Titarev-Toro).  ``compare`` runs each weight choice and
measures the L1 density distance from a run on ten times as many intervals
(the paper's reference solutions are such finer runs), sampled at the coarse
nodes.  Every step runs in the HIP library.

    python -m paper_2306_09760_amd.paper_problems --problem shu_osher
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import workloads as W
from ._lib import WCNSError
from .solver import Plan


def run(name, weights="fe", n=None, xi=100.0, cfl=0.3, method="rk4", t_end=None, device="cuda"):
    """March problem ``name`` to its end time (or ``t_end``).  Returns
    (x, U, steps) with U the final conservative state on the host."""
    prob, U, meta = W.paper_problem(name, n)
    P = Plan(device=device, **prob, weights=weights, xi=xi)
    Ud = torch.from_numpy(U).to(P.device)
    status = torch.zeros(1, dtype=torch.int32, device=P.device)
    steps, _ = P.run_to_time(Ud, meta["t_end"] if t_end is None else t_end, cfl=cfl,
                             method=method, status=status)
    if int(status.item()) != 0:
        raise WCNSError(f"{name}: a stage produced a non-physical state")
    return meta["x"], Ud.cpu().numpy(), steps


def compare(name, weights=("js", "z", "fe", "pfe"), n=None, ref_factor=10, xi=100.0,
            device="cuda"):
    """L1 density distance of each weight choice from a FE run on
    ``ref_factor`` times as many intervals (coarse nodes coincide with every
    ref_factor-th fine node)."""
    n = W.PAPER_1D[name]["n"] if n is None else n
    nref = (n - 1) * ref_factor + 1
    _, Uref, _ = run(name, "fe", nref, xi=xi, device=device)
    rho_ref = Uref[0, ::ref_factor]
    out = {"problem": name, "points": n, "reference_points": nref, "schemes": {}}
    for wname in weights:
        x, U, steps = run(name, wname, n, xi=xi, device=device)
        out["schemes"][wname] = {"l1_density": float(np.mean(np.abs(U[0] - rho_ref))),
                                 "steps": steps}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--problem", default="all", choices=["all", *W.PAPER_1D])
    ap.add_argument("--weights", default="js,z,fe,pfe")
    ap.add_argument("--xi", type=float, default=100.0)
    args = ap.parse_args()
    names = list(W.PAPER_1D) if args.problem == "all" else [args.problem]
    for name in names:
        print(json.dumps(compare(name, tuple(args.weights.split(",")), xi=args.xi)), flush=True)


if __name__ == "__main__":
    main()
