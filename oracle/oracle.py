"""ctypes wrapper of the plain FP64 CPU oracle (``wcns_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg; never by the GPU product path.

Arrays are numpy float64, variable-major: ``U[v, z, y, x]`` flattened, i.e.
``U.reshape(nv, nz, ny, nx)`` for 3D, ``(nv, ny, nx)`` for 2D, ``(nv, nx)``
for 1D.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wcns_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with fused multiply-add contraction: a second, equally
# valid rounding of the same arithmetic, used to measure how sensitive a long
# run is to rounding order.
_LIB_FMA = os.path.join(_HERE, "liboracle_fma.so")

SYSTEMS = {"advection": 0, "euler": 1}
BCS = {"periodic": 0, "transmissive": 1}
WEIGHTS = {"js": 0, "z": 1, "fe": 2, "pfe": 3, "linear": 4}
DIFFS = {"mnd6": 0, "md6": 1}
FAMILIES = {"wcns": 0, "weno": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with g++ into liboracle.so (no FMA contraction) and
    liboracle_fma.so (FMA contraction).  OpenMP shares the lines of a 2D/3D
    residual among threads (OMP_NUM_THREADS); each line's arithmetic is the
    same on any thread, so results do not depend on the thread count."""
    for path, fp in ((_LIB, ["-ffp-contract=off"]), (_LIB_FMA, ["-mfma", "-ffp-contract=fast"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", *fp, "-fPIC",
                                   "-shared", "-o", tmp, _SRC])
            os.replace(tmp, path)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [
        ("n", C.c_int64 * 3), ("h", C.c_double * 3), ("adv", C.c_double * 3),
        ("gamma", C.c_double), ("eps", C.c_double), ("xi", C.c_double),
        ("kappa", C.c_double), ("cv", C.c_double),
        ("system", C.c_int32), ("ndim", C.c_int32), ("bc", C.c_int32 * 3),
        ("weights", C.c_int32), ("zpow", C.c_int32), ("diff", C.c_int32),
        ("charproj", C.c_int32), ("family", C.c_int32),
    ]


_libs = {}


def lib(variant: str = "plain"):
    if variant not in _libs:
        path = {"plain": _LIB, "fma": _LIB_FMA}[variant]
        if not os.path.exists(path):
            build(force=False)
        L = C.CDLL(path)
        P = C.POINTER(C.c_double)
        D = C.POINTER(_Desc)
        L.ora_nvars.argtypes = [D]
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_residual.argtypes = [D, P, P]
        L.ora_residual_jvp.argtypes = [D, P, P, P, P]
        L.ora_cfl_dt.argtypes = [D, P, C.c_double]
        L.ora_cfl_dt.restype = C.c_double
        L.ora_check_state.argtypes = [D, P]
        L.ora_rk3_step.argtypes = [D, P, C.c_double]
        L.ora_rk3_step_jvp.argtypes = [D, P, P, C.c_double]
        L.ora_run_steps.argtypes = [D, P, C.c_double, C.c_double, C.c_int64]
        L.ora_run_dt_sequence.argtypes = [D, P, P, C.c_int64]
        L.ora_run_to_time.argtypes = [D, P, C.c_double, C.c_double, C.c_int64,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ora_rk4_step.argtypes = [D, P, C.c_double]
        L.ora_interpolation_weights.argtypes = [D, P, P, C.c_int64]
        L.ora_interpolation_weights.restype = C.c_int64
        L.ora_run_to_time_rk.argtypes = [D, P, C.c_double, C.c_double, C.c_int64, C.c_int,
                                         C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ora_interpolate.argtypes = [D, P, P, P]
        L.ora_interpolate.restype = C.c_double
        L.ora_interpolate_jvp.argtypes = [D, P, P, P]
        L.ora_interpolate_jvp.restype = C.c_double
        L.ora_fe_map.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.ora_fe_map.restype = C.c_double
        L.ora_fe_map_family.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]
        L.ora_fe_map_family.restype = C.c_double
        L.ora_reconstruct_weno.argtypes = [D, P, P, P]
        L.ora_reconstruct_weno.restype = C.c_double
        L.ora_eigenvectors.argtypes = [C.c_int, C.c_int, C.c_double, P, P, P, P]
        L.ora_euler_flux.argtypes = [C.c_int, C.c_int, C.c_double, P, P]
        L.ora_midpoint_flux.argtypes = [D, C.c_int, P, P]
        L.ora_count_residual_ops.argtypes = [D, P, C.POINTER(C.c_longlong)]
        L.ora_count_interpolate_ops.argtypes = [D, P, C.POINTER(C.c_longlong)]
        L.ora_count_midpoint_flux_ops.argtypes = [D, C.c_int, P, C.POINTER(C.c_longlong)]
        _libs[variant] = L
    return _libs[variant]


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """Problem descriptor of the oracle (its own; shares nothing with the
    GPU library's descriptor)."""

    def __init__(self, *, system="euler", ndim=1, n=(16,), h=None, gamma=1.4,
                 adv=(1.0, 1.0, 1.0), bc="periodic", weights="fe", zpow=2,
                 diff="mnd6", charproj=True, eps=1e-40, xi=1e6, kappa=0.5,
                 cv=1e-3, family="wcns", variant="plain"):
        n = tuple(int(v) for v in n)
        assert len(n) == ndim
        if h is None:
            h = tuple(1.0 / v for v in n)
        h = tuple(float(v) for v in (h if np.ndim(h) else (h,) * ndim))
        bcs = (bc,) * ndim if isinstance(bc, str) else tuple(bc)
        d = _Desc()
        for k in range(3):
            d.n[k] = n[k] if k < ndim else 1
            d.h[k] = h[k] if k < ndim else 1.0
            d.adv[k] = float(adv[k]) if k < len(adv) else 0.0
            d.bc[k] = BCS[bcs[k]] if k < ndim else 0
        d.gamma, d.eps, d.xi, d.kappa, d.cv = gamma, eps, xi, kappa, cv
        d.system = SYSTEMS[system]
        d.ndim = ndim
        d.weights = WEIGHTS[weights]
        d.zpow = zpow
        d.diff = DIFFS[diff]
        d.charproj = 1 if charproj else 0
        d.family = FAMILIES[family]
        self.desc = d
        self.variant = variant
        self.ndim, self.n, self.h = ndim, n, h
        self.nv = 1 if system == "advection" else ndim + 2
        self.npts = int(np.prod(n))

    @property
    def shape(self):
        return (self.nv,) + tuple(reversed(self.n))

    def _ref(self):
        return C.byref(self.desc)

    def _u(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.size == self.nv * self.npts, (U.shape, self.shape)
        return U

    def residual(self, U):
        U = self._u(U)
        R = np.empty_like(U)
        lib(self.variant).ora_residual(self._ref(), _p(U), _p(R))
        return R

    def residual_jvp(self, U, V):
        U = self._u(U)
        V = self._u(V)
        R = np.empty_like(U)
        JV = np.empty_like(U)
        lib(self.variant).ora_residual_jvp(self._ref(), _p(U), _p(V), _p(R), _p(JV))
        return R, JV

    def cfl_dt(self, U, cfl):
        U = self._u(U)
        return lib(self.variant).ora_cfl_dt(self._ref(), _p(U), cfl)

    def check_state(self, U):
        U = self._u(U)
        return lib(self.variant).ora_check_state(self._ref(), _p(U))

    def rk3_step(self, U, dt):
        U = self._u(U).copy()
        bad = lib(self.variant).ora_rk3_step(self._ref(), _p(U), dt)
        return U, bad

    def rk3_step_jvp(self, U, V, dt):
        U = self._u(U).copy()
        V = self._u(V).copy()
        bad = lib(self.variant).ora_rk3_step_jvp(self._ref(), _p(U), _p(V), dt)
        return U, V, bad

    def run_steps(self, U, nsteps, cfl=0.5, dt=0.0):
        U = self._u(U).copy()
        bad = lib(self.variant).ora_run_steps(self._ref(), _p(U), cfl, dt, int(nsteps))
        return U, bad

    def run_dt_sequence(self, U, dts):
        """SSP-RK3 steps of the given sizes (zeros skipped)."""
        U = self._u(U).copy()
        dts = np.ascontiguousarray(dts, dtype=np.float64)
        bad = lib(self.variant).ora_run_dt_sequence(self._ref(), _p(U), _p(dts), len(dts))
        return U, bad

    def rk4_step(self, U, dt):
        """One step of the four-stage scheme of eq. 16."""
        U = self._u(U).copy()
        bad = lib(self.variant).ora_rk4_step(self._ref(), _p(U), dt)
        return U, bad

    def interpolation_weights(self, U):
        """(n_interp, 3, 3): per interpolation of one residual evaluation, the
        JS/Z weights, their renormalised FE images and the weights used."""
        U = self._u(U)
        n = lib(self.variant).ora_interpolation_weights(self._ref(), _p(U), None, 0)
        if n < 0:
            raise ValueError("weight statistics cover the WCNS family only")
        out = np.empty((n, 3, 3))
        lib(self.variant).ora_interpolation_weights(self._ref(), _p(U), _p(out), n)
        return out

    def run_to_time(self, U, t_end, cfl=0.5, max_steps=10**9, method="rk3"):
        """March to t_end (last step clipped) with SSP-RK3 or the RK4 of eq. 16."""
        U = self._u(U).copy()
        s = C.c_int64(0)
        t = C.c_double(0.0)
        if method == "rk3":
            bad = lib(self.variant).ora_run_to_time(self._ref(), _p(U), cfl, t_end, max_steps,
                                                    C.byref(s), C.byref(t))
        elif method == "rk4":
            bad = lib(self.variant).ora_run_to_time_rk(self._ref(), _p(U), cfl, t_end, max_steps,
                                                       4, C.byref(s), C.byref(t))
        else:
            raise ValueError(method)
        return U, s.value, t.value, bad

    def reconstruct_weno(self, f5):
        """One WENO5 reconstruction of App. B: (value, base weights, weights used)."""
        f5 = np.ascontiguousarray(f5, dtype=np.float64)
        wb = np.empty(3)
        wo = np.empty(3)
        v = lib(self.variant).ora_reconstruct_weno(self._ref(), _p(f5), _p(wb), _p(wo))
        return v, wb, wo

    def interpolate(self, u5):
        u5 = np.ascontiguousarray(u5, dtype=np.float64)
        wb = np.empty(3)
        wo = np.empty(3)
        v = lib(self.variant).ora_interpolate(self._ref(), _p(u5), _p(wb), _p(wo))
        return v, wb, wo

    def interpolate_jvp(self, u5, du5):
        u5 = np.ascontiguousarray(u5, dtype=np.float64)
        du5 = np.ascontiguousarray(du5, dtype=np.float64)
        d = C.c_double(0.0)
        v = lib(self.variant).ora_interpolate_jvp(self._ref(), _p(u5), _p(du5), C.byref(d))
        return v, d.value

    def midpoint_flux(self, nodes, d=0):
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        assert nodes.shape == (6, self.nv)
        F = np.empty(self.nv)
        lib(self.variant).ora_midpoint_flux(self._ref(), d, _p(nodes), _p(F))
        return F

    def count_residual_ops(self, U):
        U = self._u(U)
        c = (C.c_longlong * 5)()
        lib(self.variant).ora_count_residual_ops(self._ref(), _p(U), c)
        return dict(zip(("add", "mul", "div", "sqrt", "tanh"), list(c)))

    def count_interpolate_ops(self, u5):
        """Arithmetic tally of one interpolation of the stencil u5."""
        u5 = np.ascontiguousarray(u5, dtype=np.float64)
        c = (C.c_longlong * 5)()
        lib(self.variant).ora_count_interpolate_ops(self._ref(), _p(u5), c)
        return dict(zip(("add", "mul", "div", "sqrt", "tanh"), list(c)))

    def count_midpoint_flux_ops(self, nodes, d=0):
        """Arithmetic tally of one midpoint flux from six nodes (6, nv)."""
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        assert nodes.shape == (6, self.nv)
        c = (C.c_longlong * 5)()
        lib(self.variant).ora_count_midpoint_flux_ops(self._ref(), d, _p(nodes), c)
        return dict(zip(("add", "mul", "div", "sqrt", "tanh"), list(c)))


def set_threads(n: int) -> None:
    """Threads sharing the lines of a 2D/3D residual (0: all processors)."""
    for variant in ("plain", "fma"):
        lib(variant).ora_set_threads(int(n))


def fe_map(i, w, xi, kappa=0.5, family="wcns"):
    """g_i(w) of eq. 20 with the table of Sec. 3.1 (wcns) or Table B.2 (weno)."""
    if family == "wcns":
        return lib().ora_fe_map(i, float(w), float(xi), float(kappa))
    return lib().ora_fe_map_family(i, float(w), float(xi), float(kappa), FAMILIES[family])


def eigenvectors(nd, d, gamma, Ua, Ub):
    Ua = np.ascontiguousarray(Ua, dtype=np.float64)
    Ub = np.ascontiguousarray(Ub, dtype=np.float64)
    L = np.zeros(25)
    R = np.zeros(25)
    lib().ora_eigenvectors(nd, d, gamma, _p(Ua), _p(Ub), _p(L), _p(R))
    nv = nd + 2
    return L.reshape(5, 5)[:nv, :nv], R.reshape(5, 5)[:nv, :nv]


def euler_flux(nd, d, gamma, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    F = np.zeros(nd + 2)
    lib().ora_euler_flux(nd, d, gamma, _p(U), _p(F))
    return F
