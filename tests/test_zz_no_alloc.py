"""The allocation-free SSP-RK3 step (wcns_rk3_step_noalloc), called through
the C ABI: the same step as wcns_rk3_step (its buffers in the library's own
device array instead of the caller's workspace), bitwise, on two calls in a
row, the second with a smaller input; oversized plans are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2306_09760_amd import _lib, solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return _lib, solver


def _abi_step(_lib, plan, U, dt=None, cfl=0.5, status=None):
    p = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = _lib.lib().wcns_rk3_step_noalloc(plan._h, p(U), p(dt), cfl, p(status), stream)
    _lib.check(st, "wcns_rk3_step_noalloc")


@pytest.mark.parametrize("case", ["2d", "3d", "1d"])
def test_noalloc_step_equals_workspace_step(mods, W, case):
    _lib, solver = mods
    if case == "2d":
        big, small = W.riemann2d(seed=1, n=300), W.riemann2d(seed=2, n=70)
    elif case == "3d":
        big, small = W.turbulence3d(seed=1, n=48), W.turbulence3d(seed=2, n=20)
    else:
        big = W.shock_tube(1.0, 0.75, 1.0, 0.125, -0.3, 0.1, 200000)
        small = W.shock_tube(0.5, 0.0, 2.0, 1.0, 0.4, 0.3, 3001)
    for k, (prob, U, _) in enumerate((big, small)):
        say("noalloc step", case, "call", k, "state", U.shape)
        P = solver.Plan(**prob, weights="fe", xi=100.0)
        Ua, Ub = to_dev(U), to_dev(U)
        sa = torch.zeros(1, dtype=torch.int32, device="cuda")
        sb = torch.zeros(1, dtype=torch.int32, device="cuda")
        P.rk3_step(Ua, cfl=0.5, status=sa)           # workspace step, CFL-limited
        _abi_step(_lib, P, Ub, cfl=0.5, status=sb)   # allocation-free step
        assert torch.equal(Ua, Ub), case
        dt = torch.full((1,), 0.3 * float(P.cfl_dt(Ua, 0.5).item()), dtype=torch.float64,
                        device="cuda")
        P.rk3_step(Ua, dt=dt, status=sa)             # fixed dt
        _abi_step(_lib, P, Ub, dt=dt, status=sb)
        assert torch.equal(Ua, Ub), case
        assert int(sa.item()) == 0 and int(sb.item()) == 0


def test_noalloc_refuses_plans_beyond_its_array(mods, W):
    _lib, solver = mods
    prob, U, _ = W.riemann2d(seed=0, n=1024)   # 4 x 1024^2 doubles: 3 states > 48 MiB
    P = solver.Plan(**prob, weights="fe", xi=100.0)
    Ud = to_dev(U)
    with pytest.raises(_lib.WCNSError, match="scratch"):
        _abi_step(_lib, P, Ud)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(Ud), U)  # nothing ran
