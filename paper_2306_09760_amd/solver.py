"""Python face of the WCNS-FE library: plans over torch device tensors.

PyTorch supplies device memory and the current HIP stream; every arithmetic
step runs in ``libwcns.so``.  States are float64 tensors shaped
``(nv, nx)``, ``(nv, ny, nx)`` or ``(nv, nz, ny, nx)`` (contiguous).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _aux(t, name, dtype, device, numel=None, min_numel=1, optional=True):
    """Checks an auxiliary tensor before its address goes to the library: a
    contiguous tensor of `dtype` on `device` with exactly `numel` (or at
    least `min_numel`) elements; None passes when `optional`."""
    if t is None:
        if optional:
            return None
        raise _lib.WCNSError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise _lib.WCNSError(f"{name} must be a torch tensor")
    if t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise _lib.WCNSError(f"{name} must be a contiguous {dtype} tensor on {device} "
                             f"(got {t.dtype} on {t.device})")
    if numel is not None and t.numel() != numel:
        raise _lib.WCNSError(f"{name} must have {numel} elements (got {t.numel()})")
    if t.numel() < min_numel:
        raise _lib.WCNSError(f"{name} must have at least {min_numel} elements")
    return t


def _require_device(device):
    if not torch.cuda.is_available():
        raise _lib.WCNSError("no HIP device is visible: the WCNS library runs on the GPU only")
    d = torch.device(device)
    if d.type != "cuda":
        raise _lib.WCNSError(f"device {d} is not a HIP device")
    if d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


class Plan:
    """A residual / SSP-RK3 plan for one grid (see include/wcns.h)."""

    def __init__(self, device="cuda", **problem):
        self.device = _require_device(device)
        self.problem = dict(problem)
        self.desc = _lib.make_desc(**problem)
        h = C.c_void_p()
        check(lib().wcns_plan_create(C.byref(self.desc), C.byref(h)), "wcns_plan_create")
        self._h = h
        self.ndim = self.desc.ndim
        self.nv = 1 if self.desc.system == 0 else self.ndim + 2
        n = [self.desc.n[k] for k in range(self.ndim)]
        self.shape = (self.nv,) + tuple(reversed(n))
        nbytes = lib().wcns_workspace_bytes(h)
        self.work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().wcns_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def _check_state(self, U):
        if U.dtype != torch.float64 or not U.is_contiguous() or U.device != self.device:
            raise _lib.WCNSError("state must be a contiguous float64 tensor on the plan's device")
        if tuple(U.shape) != self.shape:
            raise _lib.WCNSError(f"state shape {tuple(U.shape)} != {self.shape}")

    def _dt(self, dt, optional=True):
        return _aux(dt, "dt", torch.float64, self.device, optional=optional)

    def _status(self, status):
        return _aux(status, "status", torch.int32, self.device)

    def residual(self, U, out=None):
        self._check_state(U)
        R = torch.empty_like(U) if out is None else out
        self._check_state(R)
        check(lib().wcns_residual(self._h, _ptr(U), _ptr(R), _ptr(self.work), _stream()),
              "wcns_residual")
        return R

    def cfl_dt(self, U, cfl=0.5, out=None):
        self._check_state(U)
        dt = self.dt if out is None else self._dt(out, optional=False)
        check(lib().wcns_cfl_dt(self._h, _ptr(U), cfl, _ptr(dt), _ptr(self.work), _stream()),
              "wcns_cfl_dt")
        return dt

    def rk3_step(self, U, dt=None, cfl=0.5, status=None):
        """In-place SSP-RK3 step; dt: device tensor (1,) or None (cfl-limited)."""
        self._check_state(U)
        self._dt(dt)
        self._status(status)
        check(lib().wcns_rk3_step(self._h, _ptr(U), _ptr(self.work), _ptr(dt), cfl,
                                  _ptr(status), _stream()), "wcns_rk3_step")
        return U

    def rk3_step_noalloc(self, U, dt=None, cfl=0.5, status=None):
        """rk3_step with the step's buffers in the library's own device array
        (wcns_rk3_step_noalloc: no workspace, no allocation; calls on one GPU
        must not overlap)."""
        self._check_state(U)
        self._dt(dt)
        self._status(status)
        check(lib().wcns_rk3_step_noalloc(self._h, _ptr(U), _ptr(dt), cfl, _ptr(status),
                                          _stream()), "wcns_rk3_step_noalloc")
        return U

    def rk3_step_stages(self, U, U1, U2, dt=None, cfl=0.5, status=None):
        """rk3_step that also writes the stage states U^(1), U^(2) to U1, U2."""
        for X in (U, U1, U2):
            self._check_state(X)
        self._dt(dt)
        self._status(status)
        check(lib().wcns_rk3_step_stages(self._h, _ptr(U), _ptr(U1), _ptr(U2), _ptr(self.work),
                                         _ptr(dt), cfl, _ptr(status), _stream()),
              "wcns_rk3_step_stages")
        return U

    def rk4_step(self, U, dt=None, cfl=0.3, status=None):
        """In-place step of the four-stage scheme of eq. 16; dt as rk3_step."""
        self._check_state(U)
        self._dt(dt)
        self._status(status)
        check(lib().wcns_rk4_step(self._h, _ptr(U), _ptr(self.work), _ptr(dt), cfl,
                                  _ptr(status), _stream()), "wcns_rk4_step")
        return U

    def run_to_time(self, U, t_end, cfl=0.5, method="rk3", max_steps=10 ** 7, status=None,
                    before_step=None):
        """March U in place to t_end with CFL-limited steps, the last one
        clipped to land on t_end.  The step size is read back to the host
        once per step (to clip and count).  before_step(U), if given, is
        called with the state at the start of every step.  Returns
        (steps, t)."""
        step = {"rk3": self.rk3_step, "rk4": self.rk4_step}[method]
        dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        t, steps = 0.0, 0
        while t < t_end and steps < max_steps:
            if before_step is not None:
                before_step(U)
            self.cfl_dt(U, cfl, out=dt)
            h = float(dt.item())
            if t + h > t_end:
                h = t_end - t
                dt.fill_(h)
            step(U, dt=dt, status=status)
            t += h
            steps += 1
        return steps, t

    def weight_histogram(self, U, hist=None, nbins=10000):
        """Adds the weight counts of one residual evaluation of U to hist, an
        int64 tensor (3, 3, nbins) = [kind][k][bin] (kind 0: JS/Z weights,
        1: their FE images, 2: the weights the scheme uses); see
        wcns_weight_histogram in include/wcns.h."""
        self._check_state(U)
        if hist is None:
            hist = torch.zeros((3, 3, nbins), dtype=torch.int64, device=self.device)
        if hist.dtype != torch.int64 or not hist.is_contiguous() or hist.numel() % 9 or \
                hist.device != self.device:
            raise _lib.WCNSError("hist must be a contiguous int64 tensor of 3 x 3 x nbins "
                                 "on the plan's device")
        check(lib().wcns_weight_histogram(self._h, _ptr(U), _ptr(hist), hist.numel() // 9,
                                          _stream()), "wcns_weight_histogram")
        return hist

    def residual_adjoint(self, U, Rbar, Ubar=None):
        """Ubar += (dL/dU)^T Rbar (Ubar zero-initialised if None)."""
        self._check_state(U)
        self._check_state(Rbar)
        if Ubar is None:
            Ubar = torch.zeros_like(U)
        self._check_state(Ubar)
        check(lib().wcns_residual_adjoint(self._h, _ptr(U), _ptr(Rbar), _ptr(Ubar),
                                          _ptr(self.work), _stream()), "wcns_residual_adjoint")
        return Ubar

    def rk3_step_adjoint(self, Un, lam, dt, stages=None):
        """lam <- adjoint of U^n from the adjoint of U^{n+1} (step of size
        dt from Un); stages = (U1, U2) from rk3_step_stages skips their
        recomputation."""
        self._check_state(Un)
        self._check_state(lam)
        self._dt(dt, optional=False)
        if stages is None:
            check(lib().wcns_rk3_step_adjoint(self._h, _ptr(Un), _ptr(lam), _ptr(self.work),
                                              _ptr(dt), _stream()), "wcns_rk3_step_adjoint")
        else:
            U1, U2 = stages
            self._check_state(U1)
            self._check_state(U2)
            check(lib().wcns_rk3_step_adjoint_stages(self._h, _ptr(Un), _ptr(U1), _ptr(U2),
                                                     _ptr(lam), _ptr(self.work), _ptr(dt),
                                                     _stream()), "wcns_rk3_step_adjoint_stages")
        return lam

    def autotune(self, U):
        self._check_state(U)
        check(lib().wcns_plan_autotune(self._h, _ptr(U), _ptr(self.work), _stream()),
              "wcns_plan_autotune")
        return self.tiles

    @property
    def tiles(self):
        t = (C.c_int32 * 3)()
        lib().wcns_plan_get_tiles(self._h, t)
        return tuple(t)

    @tiles.setter
    def tiles(self, value):
        t = (C.c_int32 * 3)(*value)
        check(lib().wcns_plan_set_tiles(self._h, t), "wcns_plan_set_tiles")


class BatchPlan:
    """Ragged batch of independent 1D Euler problems (see include/wcns.h)."""

    def __init__(self, offsets, h, device="cuda", **proto):
        self.device = _require_device(device)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        h = np.ascontiguousarray(h, dtype=np.float64)
        self.nprob = len(offsets) - 1
        self.total = int(offsets[-1])
        proto = dict(proto)
        proto.setdefault("system", "euler")
        proto.setdefault("bc", "transmissive")
        proto["ndim"] = 1
        proto["n"] = (9,)
        proto["h"] = (1.0,)
        self.desc = _lib.make_desc(**proto)
        hd = C.c_void_p()
        check(lib().wcns_batch_plan_create(
            C.byref(self.desc), self.nprob, offsets.ctypes.data_as(C.POINTER(C.c_int64)),
            h.ctypes.data_as(C.POINTER(C.c_double)), C.byref(hd)), "wcns_batch_plan_create")
        self._h = hd
        self.shape = (3, self.total)
        nbytes = lib().wcns_batch_workspace_bytes(hd)
        self.work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().wcns_batch_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def _check_state(self, U):
        if U.dtype != torch.float64 or not U.is_contiguous() or U.device != self.device:
            raise _lib.WCNSError("state must be a contiguous float64 tensor on the plan's device")
        if tuple(U.shape) != self.shape:
            raise _lib.WCNSError(f"state shape {tuple(U.shape)} != {self.shape}")

    def _t(self, t):
        return _aux(t, "t", torch.float64, self.device, numel=self.nprob, optional=False)

    def _status(self, status):
        return _aux(status, "status", torch.int32, self.device)

    def residual(self, U, out=None):
        self._check_state(U)
        R = torch.empty_like(U) if out is None else out
        self._check_state(R)
        check(lib().wcns_batch_residual(self._h, _ptr(U), _ptr(R), _ptr(self.work), _stream()),
              "wcns_batch_residual")
        return R

    def rk3_step(self, U, t, t_end, cfl=0.5, status=None):
        self._check_state(U)
        self._t(t)
        self._status(status)
        check(lib().wcns_batch_rk3_step(self._h, _ptr(U), _ptr(self.work), _ptr(t), float(t_end),
                                        float(cfl), _ptr(status), _stream()), "wcns_batch_rk3_step")
        return U

    def rk3_steps(self, U, t, t_end, cfl=0.5, nsteps=1, status=None, max_live=None):
        """nsteps rk3_step calls in one: each step's CFL maximum is taken by
        the previous step's last stage (see include/wcns.h).  max_live: a
        bound on the live-tile list for the whole call (live_tiles() after an
        earlier step of the same run to the same t_end); the stage launches
        are sized to it (status required; bit 1 set if the bound was too
        small)."""
        self._check_state(U)
        self._t(t)
        self._status(status)
        if max_live is None:
            check(lib().wcns_batch_rk3_steps(self._h, _ptr(U), _ptr(self.work), _ptr(t),
                                             float(t_end), float(cfl), int(nsteps), _ptr(status),
                                             _stream()), "wcns_batch_rk3_steps")
        else:
            check(lib().wcns_batch_rk3_steps_capped(self._h, _ptr(U), _ptr(self.work), _ptr(t),
                                                    float(t_end), float(cfl), int(nsteps),
                                                    _ptr(status), int(max_live), _stream()),
                  "wcns_batch_rk3_steps_capped")
        return U

    def live_tiles(self):
        """Length of the live-tile list the last step built (synchronises the
        current stream)."""
        n = C.c_int32(0)
        check(lib().wcns_batch_live_tiles(self._h, _ptr(self.work), C.addressof(n), _stream()),
              "wcns_batch_live_tiles")
        return int(n.value)

    def cfl(self, U, t, t_end, cfl=0.5):
        """Per-problem dt into the workspace; t += dt (first kernel of a step)."""
        self._check_state(U)
        self._t(t)
        check(lib().wcns_batch_cfl(self._h, _ptr(U), _ptr(self.work), _ptr(t), float(t_end),
                                   float(cfl), _stream()), "wcns_batch_cfl")

    def stage(self, stage, Uk, U0, out, status=None):
        """One SSP-RK3 stage with the dt of the last cfl()/rk3_step()."""
        for x in (Uk, U0, out):
            self._check_state(x)
        self._status(status)
        check(lib().wcns_batch_stage(self._h, int(stage), _ptr(Uk), _ptr(U0), _ptr(out),
                                     _ptr(self.work), _ptr(status), _stream()), "wcns_batch_stage")
        return out

    def last_dt(self, out=None):
        """The dt each problem took in the last step (0: finished or stopped),
        copied on the device into `out` (float64, nprob) or a new tensor."""
        out = torch.empty(self.nprob, dtype=torch.float64, device=self.device) if out is None \
            else _aux(out, "out", torch.float64, self.device, numel=self.nprob, optional=False)
        check(lib().wcns_batch_last_dt(self._h, _ptr(self.work), _ptr(out), _stream()),
              "wcns_batch_last_dt")
        return out

    def set_graph(self, enable=True):
        check(lib().wcns_batch_set_graph(self._h, 1 if enable else 0), "wcns_batch_set_graph")

    def autotune(self, U):
        self._check_state(U)
        check(lib().wcns_batch_autotune(self._h, _ptr(U), _ptr(self.work), _stream()),
              "wcns_batch_autotune")
        return self.tile

    @property
    def tile(self):
        return int(lib().wcns_batch_get_tile(self._h))

    @tile.setter
    def tile(self, value):
        check(lib().wcns_batch_set_tile(self._h, int(value)), "wcns_batch_set_tile")

    def run_to_time(self, U, t_end, cfl=0.5, check_every=64, max_steps=10 ** 7, status=None,
                    fused=True):
        """Steps every problem to t_end (host checks completion every
        ``check_every`` steps): with ``fused`` in rk3_steps calls, else one
        rk3_step call per step (graph-replayed if set_graph).  Raises
        WCNSError when a problem's state goes non-physical (the library then
        stops that problem and sets bit 0 of the status word).  Returns (t,
        steps issued)."""
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._status(status)
        t = torch.zeros(self.nprob, dtype=torch.float64, device=self.device)
        steps = 0
        live = None  # bound on the live-tile list, from the last check (fused calls)
        while steps < max_steps:
            if fused:
                self.rk3_steps(U, t, t_end, cfl, check_every, status, max_live=live)
            else:
                for _ in range(check_every):
                    self.rk3_step(U, t, t_end, cfl, status)
            steps += check_every
            word = int(status.item())
            if word & 1:
                bad = torch.nonzero(t < t_end).flatten().tolist()
                raise _lib.WCNSError(f"non-physical state after {steps} steps (problems not at "
                                     f"t_end: {bad[:16]}{' ...' if len(bad) > 16 else ''})")
            if word:
                raise _lib.WCNSError(f"status word {word} after {steps} steps")
            if bool((t >= t_end).all().item()):
                break
            if fused:
                live = max(1, self.live_tiles())
        return t, steps
