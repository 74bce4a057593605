"""The roof probes compute what their header states (the timing itself is
the bench's): the FMA stream's per-lane sums against the closed form of the
affine recursion, the streaming copy bit for bit (even and odd lengths); and
the device's elementary functions against their error bounds."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2306_09760_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return _lib


def test_fma_probe_matches_the_affine_recursion(L):
    blocks, iters = 3, 1000
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    L.check(L.lib().wcns_probe_fp64_fma(C.c_void_p(out.data_ptr()), blocks, iters, None), "probe")
    got = out.cpu().numpy()
    a, b = 1.0 - 2.0 ** -30, 2.0 ** -30
    g = np.arange(blocks * 256)
    base = 1.0 + (g & 1023) / 1024.0
    an = a ** iters
    # x_n = a^n x_0 + b (1 - a^n) / (1 - a) = a^n x_0 + (1 - a^n) for b = 1 - a
    want = sum(an * (base + k / 16.0) + (1.0 - an) for k in range(8))
    assert np.max(np.abs(got - want) / want) < 1e-13


@pytest.mark.parametrize("n", [0, 1, 4096, 1000001])
def test_copy_probe_is_exact(L, n):
    src = torch.randn(max(n, 1), dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    L.check(L.lib().wcns_probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n,
                                    None), "probe")
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n])


def test_copy_probe_rejects_overlap(L):
    # src = x[0:64], dst = x[32:96]: overlapping, and inside x even if copied
    x = torch.zeros(128, dtype=torch.float64, device="cuda")
    st = L.lib().wcns_probe_copy(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr() + 256), 64, None)
    assert st == L.WCNS_EINVAL


# Error bounds of the device's elementary functions (wcns_probe_math) against
# x86 extended precision (numpy longdouble, 64-bit significand): Tang's
# table-driven e^z and the Cody-Waite e^z within 2 ulp, the reciprocal with
# two Newton steps within 1 ulp and with one within 2^-48 relative (the
# hardware seed's 2^-24.4, squared), the square root within 1 ulp.
MATH_FN = {"exp_tab": 0, "exp_cw": 1, "rcp": 2, "rcp1": 3, "sqrt": 4}


def _math(L, fn, x):
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    out = torch.empty_like(xd)
    L.check(L.lib().wcns_probe_math(C.c_void_p(xd.data_ptr()), C.c_void_p(out.data_ptr()), x.size,
                                    MATH_FN[fn], None), "probe")
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _ulps(y, ref):
    """|y - ref| in units of the spacing of doubles at ref."""
    ulp = np.spacing(np.abs(ref.astype(np.float64))).astype(np.longdouble)
    return np.abs((y.astype(np.longdouble) - ref) / ulp)


@pytest.fixture(scope="module")
def rng():
    assert np.finfo(np.longdouble).nmant >= 63, "the reference needs x86 extended precision"
    return np.random.default_rng(12)


@pytest.mark.parametrize("fn", ["exp_tab", "exp_cw"])
def test_exponentials_within_two_ulp(L, rng, fn):
    z = np.concatenate([rng.uniform(-708.0, 708.0, 400000), rng.uniform(-1.0, 1.0, 100000),
                        [0.0, 1e-300, -1e-300, np.log(2.0), -np.log(2.0) / 128, 708.0, -708.0]])
    y = _math(L, fn, z)
    err = _ulps(y, np.exp(z.astype(np.longdouble)))
    assert y[z.size - 7] == 1.0
    assert float(err.max()) <= 2.0, (fn, float(err.max()), z[int(np.argmax(err))])


def test_reciprocals(L, rng):
    x = 10.0 ** rng.uniform(-300.0, 300.0, 400000) * rng.choice([-1.0, 1.0], 400000)
    x = np.concatenate([x, rng.uniform(1.0, 2.0, 100000), [1.0, -1.0, 3.0, 0.1]])
    ref = 1.0 / x.astype(np.longdouble)
    two = _math(L, "rcp", x)
    one = _math(L, "rcp1", x)
    assert float(_ulps(two, ref).max()) <= 1.0
    rel = np.abs((one.astype(np.longdouble) - ref) / ref)
    assert float(rel.max()) <= 2.0 ** -48, float(np.log2(float(rel.max())))
    assert two[x.size - 4] == 1.0 and two[x.size - 3] == -1.0


def test_square_root_within_one_ulp(L, rng):
    x = np.concatenate([10.0 ** rng.uniform(-228.0, 300.0, 400000),
                        rng.uniform(0.5, 4.0, 100000), [0.0, 1.0, 4.0, 2.0 ** -760]])
    y = _math(L, "sqrt", x)
    assert y[x.size - 4] == 0.0 and y[x.size - 3] == 1.0 and y[x.size - 2] == 2.0
    assert float(_ulps(y, np.sqrt(x.astype(np.longdouble))).max()) <= 1.0
    # a negative argument (a non-physical state) gives NaN, not a number
    assert np.isnan(_math(L, "sqrt", np.array([-1.0, -1e-300]))).all()
