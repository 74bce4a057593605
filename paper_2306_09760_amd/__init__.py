"""MI355X (gfx950) library for the residual of the filtered embedded weighted
compact nonlinear scheme (WCNS-FE, arXiv 2306.09760) and its SSP-RK3 step.

The arithmetic runs in the hand-written HIP kernels of ``libwcns.so``
(C ABI in ``include/wcns.h``); this package only marshals arguments and uses
PyTorch for device memory and streams.  Importing it does not load the
library; the first plan does, and fails loudly if it is not built.
The differentiable checkpointed rollout lives in ``.rollout``.
"""
__all__ = ["Plan", "BatchPlan", "WCNSError", "build"]


def __getattr__(name):
    if name in ("Plan", "BatchPlan"):
        from . import solver
        return getattr(solver, name)
    if name == "WCNSError":
        from ._lib import WCNSError
        return WCNSError
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
