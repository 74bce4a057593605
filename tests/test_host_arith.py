"""Host-side integer and floating-point facts the kernels rely on, checked
without a GPU: the multiply-shift division of tile indices (FastDiv in
wcns_internal.hpp, compiled here as host code) against integer division,
and the offset the device square root adds to its argument."""
import re
import subprocess

import numpy as np
import pytest

from paper_2306_09760_amd import build as B

_HARNESS = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>
#include "wcns_internal.hpp"
using wcns::fast_div;
static long long bad = 0, cases = 0;
static void check(uint32_t d, uint32_t n) {
  ++cases;
  if (fast_div(d).div(n) != n / d && bad++ < 5)
    std::printf("MISMATCH d=%u n=%u\n", d, n);
}
int main() {
  std::mt19937_64 rng(12345);
  const uint32_t top = 0x7fffffffu;  // tile indices and divisors below 2^31
  std::vector<uint32_t> ds;
  for (uint32_t d = 1; d <= 3000; ++d) ds.push_back(d);
  for (int l = 1; l < 31; ++l) {
    const uint32_t p = 1u << l;
    ds.push_back(p - 1); ds.push_back(p); ds.push_back(p + 1);
  }
  ds.push_back(top);
  for (int k = 0; k < 2000; ++k) ds.push_back(1 + (uint32_t)(rng() % top));
  for (uint32_t d : ds) {
    // boundaries of the quotient steps, the largest n, and random n
    const uint64_t qs[5] = {0, 1, 2, (uint64_t)top / d, (uint64_t)top / d - 1};
    for (uint64_t q : qs) {
      for (int64_t o = -1; o <= 1; ++o) {
        const int64_t n = (int64_t)(q * d) + o;
        if (n >= 0 && n <= top) check(d, (uint32_t)n);
      }
    }
    check(d, top);
    for (int k = 0; k < 300; ++k) check(d, (uint32_t)(rng() % ((uint64_t)top + 1)));
  }
  // every n for a few divisors used by real tile grids
  for (uint32_t d : {3u, 7u, 37u, 251u, 1021u})
    for (uint32_t n = 0; n < (1u << 22); ++n) check(d, n);
  std::printf("cases %lld bad %lld\n", cases, bad);
  return bad ? 1 : 0;
}
"""


def test_fast_div_matches_integer_division(tmp_path):
    src = tmp_path / "fastdiv.cpp"
    src.write_text(_HARNESS)
    exe = tmp_path / "fastdiv"
    cmd = [B.hipcc(), "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", B.CSRC,
           str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        pytest.fail("host build of the FastDiv harness failed:\n" + r.stderr[-2000:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    m = re.search(r"cases (\d+) bad (\d+)", out.stdout)
    assert m and int(m.group(2)) == 0 and int(m.group(1)) > 20_000_000, out.stdout


def test_square_root_offset_leaves_its_domain_unchanged():
    # sqrt_pos seeds its reciprocal square root at x + 2^-1000: for every x
    # from 2^-760 up (its documented domain) that sum rounds back to x
    rng = np.random.default_rng(0)
    lo = np.float64(2.0) ** -760
    x = np.concatenate([lo * (1.0 + np.arange(0, 64) * 2.0 ** -52),
                        10.0 ** rng.uniform(-228.0, 300.0, 200000),
                        [lo, np.nextafter(lo, np.inf), 1.0, np.finfo(np.float64).max]])
    assert np.all(x + np.float64(2.0) ** -1000 == x)
    # and 2^-1000 is a normal number, so the seed at x = 0 is finite
    assert np.float64(2.0) ** -1000 > np.finfo(np.float64).tiny
