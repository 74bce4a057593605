"""Helpers shared by the GPU tests: host/device copies and the parity norms."""
import sys

import numpy as np
import torch

DEV = "cuda"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(gpu, ref):
    """Per-variable normwise relative error, max over variables, and the
    largest pointwise difference relative to max |ref|."""
    gpu = np.asarray(gpu).reshape(gpu.shape[0], -1)
    ref = np.asarray(ref).reshape(ref.shape[0], -1)
    norm = 0.0
    for v in range(ref.shape[0]):
        den = np.linalg.norm(ref[v])
        num = np.linalg.norm(gpu[v] - ref[v])
        norm = max(norm, num / den if den > 0 else num)
    point = np.abs(gpu - ref).max() / max(np.abs(ref).max(), 1e-300)
    return norm, point


def say(*a):
    """Names the case on stdout before GPU work (flushed)."""
    print(*a, flush=True)
    sys.stdout.flush()


RUN_TOL = 1e-9


def run_tolerance(ref, alt):
    """Bar for a multi-step run: 1e-9 normwise, unless the method itself is
    more sensitive to rounding order on this input.  ``alt`` is the same run
    of the oracle built with FMA contraction (another valid rounding of the
    same arithmetic); the GPU may differ from the oracle by up to ten times
    that spread.  Returns (normwise bar, pointwise bar, spread)."""
    n, p = rel_err(alt, ref)
    return max(RUN_TOL, 10 * n), max(RUN_TOL, 10 * p), (n, p)
