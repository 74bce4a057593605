"""Plain FP64 CPU oracle of the WCNS-FE residual and SSP-RK3 step.

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU-baseline leg; the GPU product path never imports it.
"""
from .oracle import Problem, build, eigenvectors, euler_flux, fe_map, lib, set_threads  # noqa: F401
