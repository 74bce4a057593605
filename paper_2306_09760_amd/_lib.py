"""ctypes loader of ``libwcns.so`` and the mirror of ``include/wcns.h``.

Argument marshalling only: every step of the residual runs in the library's
HIP kernels.  torch is imported first so that the library binds to the same
HIP runtime as PyTorch (both carry the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (load PyTorch's HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
# The in-tree build; WCNS_LIB may name another build of the same library.
LIB_PATH = os.environ.get("WCNS_LIB") or os.path.join(HERE, "libwcns.so")

WCNS_OK, WCNS_EINVAL, WCNS_ENOMEM, WCNS_EDEVICE, WCNS_ENONPHYS, WCNS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SYSTEMS = {"advection": 0, "euler": 1}
BCS = {"periodic": 0, "transmissive": 1}
WEIGHTS = {"js": 0, "z": 1, "fe": 2, "pfe": 3, "linear": 4}
DIFFS = {"mnd6": 0, "md6": 1}
SCHEMES = {"wcns": 0, "weno": 1}

# Every entry point declared in include/wcns.h.
EXPORTS = [
    "wcns_desc_init", "wcns_plan_create", "wcns_plan_destroy", "wcns_state_elems",
    "wcns_workspace_bytes", "wcns_residual", "wcns_cfl_dt", "wcns_rk3_step",
    "wcns_rk3_step_noalloc",
    "wcns_rk3_step_stages", "wcns_rk4_step",
    "wcns_weight_histogram",
    "wcns_residual_adjoint", "wcns_rk3_step_adjoint", "wcns_rk3_step_adjoint_stages",
    "wcns_plan_autotune",
    "wcns_plan_get_tiles", "wcns_plan_set_tiles", "wcns_batch_plan_create",
    "wcns_batch_plan_destroy", "wcns_batch_state_elems", "wcns_batch_workspace_bytes",
    "wcns_batch_residual", "wcns_batch_rk3_step", "wcns_batch_rk3_steps", "wcns_batch_set_graph", "wcns_batch_last_dt",
    "wcns_batch_live_tiles", "wcns_batch_rk3_steps_capped",
    "wcns_batch_autotune", "wcns_batch_get_tile", "wcns_batch_set_tile",
    "wcns_batch_cfl", "wcns_batch_stage", "wcns_probe_fp64_fma", "wcns_probe_copy", "wcns_probe_math",
    "wcns_status_string", "wcns_last_error",
]


class WCNSError(RuntimeError):
    pass


class Desc(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32), ("system", C.c_int32), ("ndim", C.c_int32),
        ("weights", C.c_int32), ("n", C.c_int64 * 3), ("h", C.c_double * 3),
        ("adv_speed", C.c_double * 3), ("bc", C.c_int32 * 3), ("diff", C.c_int32),
        ("gamma", C.c_double), ("eps", C.c_double), ("xi", C.c_double),
        ("kappa", C.c_double), ("cv", C.c_double), ("z_power", C.c_int32),
        ("char_proj", C.c_int32), ("scheme", C.c_int32), ("reserved_", C.c_int32),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WCNSError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2306_09760_amd.build` "
            "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    st = C.c_int
    sig = {
        "wcns_desc_init": (None, [C.POINTER(Desc)]),
        "wcns_plan_create": (st, [C.POINTER(Desc), C.POINTER(vp)]),
        "wcns_plan_destroy": (st, [vp]),
        "wcns_state_elems": (C.c_int64, [vp]),
        "wcns_workspace_bytes": (C.c_size_t, [vp]),
        "wcns_residual": (st, [vp, vp, vp, vp, vp]),
        "wcns_cfl_dt": (st, [vp, vp, C.c_double, vp, vp, vp]),
        "wcns_rk3_step": (st, [vp, vp, vp, vp, C.c_double, vp, vp]),
        "wcns_rk3_step_noalloc": (st, [vp, vp, vp, C.c_double, vp, vp]),
        "wcns_rk3_step_stages": (st, [vp, vp, vp, vp, vp, vp, C.c_double, vp, vp]),
        "wcns_rk4_step": (st, [vp, vp, vp, vp, C.c_double, vp, vp]),
        "wcns_weight_histogram": (st, [vp, vp, vp, C.c_int32, vp]),
        "wcns_residual_adjoint": (st, [vp, vp, vp, vp, vp, vp]),
        "wcns_rk3_step_adjoint": (st, [vp, vp, vp, vp, vp, vp]),
        "wcns_rk3_step_adjoint_stages": (st, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "wcns_plan_autotune": (st, [vp, vp, vp, vp]),
        "wcns_plan_get_tiles": (None, [vp, ip]),
        "wcns_plan_set_tiles": (st, [vp, ip]),
        "wcns_batch_plan_create": (st, [C.POINTER(Desc), C.c_int64, C.POINTER(C.c_int64), dp, C.POINTER(vp)]),
        "wcns_batch_plan_destroy": (st, [vp]),
        "wcns_batch_state_elems": (C.c_int64, [vp]),
        "wcns_batch_workspace_bytes": (C.c_size_t, [vp]),
        "wcns_batch_residual": (st, [vp, vp, vp, vp, vp]),
        "wcns_batch_rk3_step": (st, [vp, vp, vp, vp, C.c_double, C.c_double, vp, vp]),
        "wcns_batch_rk3_steps": (st, [vp, vp, vp, vp, C.c_double, C.c_double, C.c_int32, vp, vp]),
        "wcns_batch_set_graph": (st, [vp, C.c_int32]),
        "wcns_batch_last_dt": (st, [vp, vp, vp, vp]),
        "wcns_batch_live_tiles": (st, [vp, vp, vp, vp]),
        "wcns_batch_rk3_steps_capped": (st, [vp, vp, vp, vp, C.c_double, C.c_double, C.c_int32, vp,
                                             C.c_int32, vp]),
        "wcns_batch_cfl": (st, [vp, vp, vp, vp, C.c_double, C.c_double, vp]),
        "wcns_batch_stage": (st, [vp, C.c_int32, vp, vp, vp, vp, vp, vp]),
        "wcns_batch_autotune": (st, [vp, vp, vp, vp]),
        "wcns_batch_get_tile": (C.c_int32, [vp]),
        "wcns_batch_set_tile": (st, [vp, C.c_int32]),
        "wcns_probe_fp64_fma": (st, [vp, C.c_int32, C.c_int32, vp]),
        "wcns_probe_copy": (st, [vp, vp, C.c_int64, vp]),
        "wcns_probe_math": (st, [vp, vp, C.c_int64, C.c_int32, vp]),
        "wcns_status_string": (C.c_char_p, [st]),
        "wcns_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int, what: str = "") -> None:
    if status != WCNS_OK:
        L = lib()
        msg = L.wcns_last_error().decode()
        name = L.wcns_status_string(status).decode()
        raise WCNSError(f"{what}: {name} ({status}): {msg}")


def make_desc(*, system="euler", ndim=1, n=(16,), h=None, gamma=1.4, adv=(1.0, 1.0, 1.0),
              bc="periodic", weights="fe", zpow=2, diff="mnd6", charproj=True, eps=1e-40,
              xi=100.0, kappa=0.5, cv=1e-3, scheme="wcns") -> Desc:
    d = Desc()
    lib().wcns_desc_init(C.byref(d))
    n = tuple(int(v) for v in n)
    if h is None:
        h = tuple(1.0 / v for v in n)
    if not hasattr(h, "__len__"):
        h = (float(h),) * ndim
    bcs = (bc,) * ndim if isinstance(bc, str) else tuple(bc)
    d.system = SYSTEMS[system]
    d.ndim = ndim
    d.weights = WEIGHTS[weights]
    for k in range(3):
        d.n[k] = n[k] if k < len(n) else 1
        d.h[k] = float(h[k]) if k < len(h) else 1.0
        d.adv_speed[k] = float(adv[k]) if k < len(adv) else 0.0
        d.bc[k] = BCS[bcs[k]] if k < len(bcs) else 0
    d.diff = DIFFS[diff]
    d.gamma = gamma
    d.eps = eps
    d.xi = xi
    d.kappa = kappa
    d.cv = cv
    d.z_power = zpow
    d.char_proj = 1 if charproj else 0
    d.scheme = SCHEMES[scheme]
    return d
