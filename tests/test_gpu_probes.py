"""The roof probes compute what their header states (the timing itself is
the bench's): the FMA stream's per-lane sums against the closed form of the
affine recursion, the streaming copy bit for bit (even and odd lengths)."""
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
