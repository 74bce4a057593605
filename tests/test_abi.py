"""The C-ABI library loads, exports every entry point include/wcns.h
declares, and rejects invalid arguments on the host (no device work)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wcns.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(wcns_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2306_09760_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_09760_amd.build import build
        build()
    return _lib


def test_header_declares_the_binding_list(L):
    assert _declared() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing


def test_desc_layout_matches_header(L):
    # sizeof(wcns_desc) is checked by the library through struct_size
    d = L.Desc()
    L.lib().wcns_desc_init(C.byref(d))
    assert d.struct_size == C.sizeof(L.Desc)
    assert d.weights == 2 and d.diff == 0 and d.z_power == 2
    assert d.eps == 1e-40 and d.xi == 100.0 and d.kappa == 0.5 and d.cv == 1e-3


def _create(L, **kw):
    d = L.make_desc(**kw)
    h = C.c_void_p()
    st = L.lib().wcns_plan_create(C.byref(d), C.byref(h))
    if st == 0:
        L.lib().wcns_plan_destroy(h)
    return st, L.lib().wcns_last_error().decode()


def test_valid_plans_are_created_without_a_device(L):
    assert _create(L, system="euler", ndim=2, n=(64, 32))[0] == 0
    assert _create(L, system="advection", ndim=1, n=(200,), h=0.01)[0] == 0
    assert _create(L, system="euler", ndim=3, n=(16, 16, 16), diff="md6", weights="pfe")[0] == 0


@pytest.mark.parametrize("kw,msg", [
    (dict(n=(8,)), "< 9"),
    (dict(gamma=1.0), "gamma"),
    (dict(xi=0.0), "xi"),
    (dict(xi=-1.0), "xi"),
    (dict(zpow=0), "z_power"),
    (dict(eps=-1.0), "eps"),
    (dict(h=(0.0,)), "h[0]"),
])
def test_invalid_descriptors_are_rejected(L, kw, msg):
    args = dict(system="euler", ndim=1, n=(32,))
    args.update(kw)
    st, err = _create(L, **args)
    assert st == L.WCNS_EINVAL
    assert msg in err


def test_bad_enum_and_struct_size_rejected(L):
    d = L.make_desc(system="euler", ndim=1, n=(32,))
    d.weights = 9
    h = C.c_void_p()
    assert L.lib().wcns_plan_create(C.byref(d), C.byref(h)) == L.WCNS_EINVAL
    d = L.make_desc(system="euler", ndim=1, n=(32,))
    d.struct_size = 8
    assert L.lib().wcns_plan_create(C.byref(d), C.byref(h)) == L.WCNS_EINVAL
    assert "struct_size" in L.lib().wcns_last_error().decode()


def test_null_arguments_rejected_before_any_device_work(L):
    lib = L.lib()
    d = L.make_desc(system="euler", ndim=1, n=(32,))
    h = C.c_void_p()
    assert lib.wcns_plan_create(C.byref(d), C.byref(h)) == 0
    try:
        assert lib.wcns_residual(h, None, None, None, None) == L.WCNS_EINVAL
        assert lib.wcns_rk3_step(h, None, None, None, 0.5, None, None) == L.WCNS_EINVAL
        assert lib.wcns_residual_adjoint(h, None, None, None, None, None) == L.WCNS_EINVAL
        x = C.c_void_p(4096)
        assert lib.wcns_residual(h, x, x, x, None) == L.WCNS_EINVAL  # U == R
        assert lib.wcns_rk3_step(h, x, x, None, -1.0, None, None) == L.WCNS_EINVAL  # cfl <= 0
        t = (C.c_int32 * 3)(100, 32, 64)
        assert lib.wcns_plan_set_tiles(h, t) == L.WCNS_EINVAL
    finally:
        lib.wcns_plan_destroy(h)


def test_workspace_size_covers_the_documented_buffers(L):
    lib = L.lib()
    d = L.make_desc(system="euler", ndim=2, n=(100, 50))
    h = C.c_void_p()
    assert lib.wcns_plan_create(C.byref(d), C.byref(h)) == 0
    try:
        elems = lib.wcns_state_elems(h)
        assert elems == 4 * 100 * 50
        # two stage states, the residual accumulator, two stage cotangents
        assert lib.wcns_workspace_bytes(h) >= 5 * 8 * elems
    finally:
        lib.wcns_plan_destroy(h)


def test_batch_plan_validation_on_host(L):
    import numpy as np
    lib = L.lib()
    d = L.make_desc(system="euler", ndim=1, n=(9,), bc="transmissive")
    off = np.array([0, 5, 20], dtype=np.int64)  # first problem too short
    hh = np.array([0.1, 0.1])
    out = C.c_void_p()
    st = lib.wcns_batch_plan_create(C.byref(d), 2, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                    hh.ctypes.data_as(C.POINTER(C.c_double)), C.byref(out))
    assert st == L.WCNS_EINVAL
    d2 = L.make_desc(system="euler", ndim=2, n=(16, 16))
    st = lib.wcns_batch_plan_create(C.byref(d2), 2, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                    hh.ctypes.data_as(C.POINTER(C.c_double)), C.byref(out))
    assert st == L.WCNS_EINVAL


@pytest.mark.parametrize("nprob,offsets,h,msg", [
    (0, [0], [], "nprob"),                          # empty batch
    (2, [1, 20, 40], [0.1, 0.1], "offsets[0]"),     # does not start at node 0
    (2, [0, 30, 25], [0.1, 0.1], "nodes"),          # decreasing offsets
    (2, [0, 9, 18], [0.1, 0.0], "h["),              # zero spacing
    (2, [0, 9, 18], [0.1, -0.2], "h["),             # negative spacing
    (2, [0, 9, 18], [float("nan"), 0.1], "h["),     # NaN spacing
    (2, [0, 9, 18], [0.1, float("inf")], "h["),     # infinite spacing
])
def test_degenerate_batches_rejected_on_host(L, nprob, offsets, h, msg):
    """Batch plans that describe no valid set of problems fail with
    WCNS_EINVAL before any device memory is touched."""
    import numpy as np
    lib = L.lib()
    d = L.make_desc(system="euler", ndim=1, n=(9,), bc="transmissive")
    off = np.array(offsets, dtype=np.int64)
    hh = np.array(h if h else [1.0], dtype=np.float64)
    out = C.c_void_p()
    st = lib.wcns_batch_plan_create(C.byref(d), nprob, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                    hh.ctypes.data_as(C.POINTER(C.c_double)), C.byref(out))
    assert st == L.WCNS_EINVAL
    assert msg in lib.wcns_last_error().decode()
    assert not out.value


def test_math_probe_validates_on_host(L):
    """wcns_probe_math rejects an unknown function, a NULL array or n < 0
    before any device work."""
    lib = L.lib()
    buf = (C.c_double * 4)()
    p = C.cast(buf, C.c_void_p)
    assert lib.wcns_probe_math(p, p, 4, 5, None) == L.WCNS_EINVAL
    assert lib.wcns_probe_math(p, p, 4, -1, None) == L.WCNS_EINVAL
    assert lib.wcns_probe_math(None, p, 4, 0, None) == L.WCNS_EINVAL
    assert lib.wcns_probe_math(p, p, -1, 0, None) == L.WCNS_EINVAL


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle and refuses to run without a
    device."""
    pkg = os.path.join(ROOT, "paper_2306_09760_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
    import torch
    if not torch.cuda.is_available():
        from paper_2306_09760_amd import Plan, WCNSError
        with pytest.raises(WCNSError):
            Plan(system="euler", ndim=1, n=(32,))


def test_adjoint_step_rejects_aliasing_on_host(L):
    """The reverse step writes lambda in place while tiles still read the
    states, and keeps two stage cotangents in the workspace: overlapping
    arguments are rejected before anything is enqueued (the pointers here
    are never dereferenced)."""
    lib = L.lib()
    d = L.make_desc(system="euler", ndim=1, n=(32,))
    h = C.c_void_p()
    assert lib.wcns_plan_create(C.byref(d), C.byref(h)) == 0
    try:
        sb = 8 * lib.wcns_state_elems(h)
        wb = lib.wcns_workspace_bytes(h)
        base = 1 << 40  # distinct, non-overlapping fake addresses
        Un, U1, U2, lam, dt = (C.c_void_p(base + k * (1 << 30)) for k in range(5))
        work = C.c_void_p(base + 8 * (1 << 30))
        step = lib.wcns_rk3_step_adjoint
        stages = lib.wcns_rk3_step_adjoint_stages
        assert step(h, Un, Un, work, dt, None) == L.WCNS_EINVAL            # lambda == Un
        assert "lambda" in lib.wcns_last_error().decode()
        assert step(h, Un, C.c_void_p(base + 8), work, dt, None) == L.WCNS_EINVAL  # overlap
        assert step(h, Un, work, work, dt, None) == L.WCNS_EINVAL          # lambda in work
        assert stages(h, Un, U1, U2, U1, work, dt, None) == L.WCNS_EINVAL  # lambda == U1
        assert stages(h, Un, U1, U2, U2, work, dt, None) == L.WCNS_EINVAL  # lambda == U2
        # a stage state inside the workspace's cotangent buffers (the last
        # two states' worth of the first five)
        inside = C.c_void_p(work.value + 3 * sb)
        assert 3 * sb < wb
        assert stages(h, Un, inside, U2, lam, work, dt, None) == L.WCNS_EINVAL
        assert "cotangent" in lib.wcns_last_error().decode()
    finally:
        lib.wcns_plan_destroy(h)


def test_noalloc_step_refuses_plans_beyond_its_array_on_host(L):
    """wcns_rk3_step_noalloc checks the plan against its 48 MiB array before
    any device work (the pointers here are never dereferenced)."""
    lib = L.lib()
    d = L.make_desc(system="euler", ndim=2, n=(1024, 1024))   # 3 x 32 MiB of states
    h = C.c_void_p()
    assert lib.wcns_plan_create(C.byref(d), C.byref(h)) == 0
    try:
        st = lib.wcns_rk3_step_noalloc(h, C.c_void_p(1 << 40), None, 0.5, None, None)
        assert st == L.WCNS_EINVAL
        assert "scratch" in lib.wcns_last_error().decode()
        assert lib.wcns_rk3_step_noalloc(h, None, None, 0.5, None, None) == L.WCNS_EINVAL
    finally:
        lib.wcns_plan_destroy(h)


def test_capped_batch_steps_refuse_on_host(L):
    """wcns_batch_rk3_steps_capped needs a status word and max_live >= 1;
    wcns_batch_live_tiles refuses NULL arguments (no device work)."""
    lib = L.lib()
    x = C.c_void_p(16)
    n = C.c_int32(0)
    steps = lib.wcns_batch_rk3_steps_capped
    assert steps(None, x, x, x, 0.2, 0.5, 4, None, 8, None) == L.WCNS_EINVAL    # no status
    assert steps(None, x, x, x, 0.2, 0.5, 4, x, 0, None) == L.WCNS_EINVAL       # max_live 0
    assert steps(None, x, x, x, 0.2, 0.5, 4, x, 8, None) == L.WCNS_EINVAL       # no plan
    assert lib.wcns_batch_live_tiles(None, x, C.addressof(n), None) == L.WCNS_EINVAL
