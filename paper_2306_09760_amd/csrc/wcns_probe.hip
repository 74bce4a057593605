// Roof probes of gfx950 (measurement only, not part of the method): a
// register-resident FP64 FMA stream for the vector-ALU roof and a 16-byte
// streaming copy for the HBM roof.  Both sizes come from the caller, which
// times them.  And the device's elementary functions (exp_tab, exp_cw, rcp,
// rcp1, sqrt_pos) applied to an array, for checks of their error bounds.
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"

namespace wcns {

// Eight independent chains x <- x a + b per lane (16 flops per round); the
// lane's sum of the chains is written so that no chain is dead code.
__global__ void __launch_bounds__(256) probe_fma_kernel(double* __restrict__ out, int iters) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  constexpr double a = 1.0 - 0x1p-30, b = 0x1p-30;
  const double base = 1.0 + (double)(gid & 1023) * (1.0 / 1024.0);
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = base + k * 0.0625;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __builtin_fma(x[k], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[gid] = s;
}

// dst[i] = src[i]: pairs of doubles per lane per access, four accesses in
// flight per lane (all loads of a round issued before its stores),
// grid-stride over rounds.
__global__ void __launch_bounds__(256) probe_copy_kernel(const double2* __restrict__ src,
                                                         double2* __restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const double2 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride],
                  v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n2; i += stride) dst[i] = src[i];
}

__global__ void probe_copy_tail_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                       int64_t i) {
  dst[i] = src[i];
}

// out[i] = f(x[i]) for the elementary function f selected by fn (0 exp_tab,
// 1 exp_cw, 2 rcp, 3 rcp1, 4 sqrt_pos), grid-stride; exp_tab reads the
// 2^(k/64) table from LDS as the sweep kernels do.
__global__ void __launch_bounds__(256) probe_math_kernel(const double* __restrict__ x,
                                                         double* __restrict__ out, int64_t n,
                                                         int fn) {
  __shared__ double sX[64];
  if (threadIdx.x < 64) sX[threadIdx.x] = kExp2Tab64[threadIdx.x];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = x[i];
    double y;
    switch (fn) {
      case 0: y = exp_tab(v, sX); break;
      case 1: y = exp_cw(v); break;
      case 2: y = rcp(v); break;
      case 3: y = rcp1(v); break;
      default: y = sqrt_pos(v); break;
    }
    out[i] = y;
  }
}

hipError_t launch_probe_math(const double* x, double* out, int64_t n, int fn, hipStream_t stream) {
  if (n > 0) {
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(probe_math_kernel, dim3(blocks), dim3(256), 0, stream, x, out, n, fn);
  }
  return hipGetLastError();
}

hipError_t launch_probe_fma(double* out, int blocks, int iters, hipStream_t stream) {
  hipLaunchKernelGGL(probe_fma_kernel, dim3(blocks), dim3(256), 0, stream, out, iters);
  return hipGetLastError();
}

hipError_t launch_probe_copy(const double* src, double* dst, int64_t n, hipStream_t stream) {
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    // about one round of four accesses per lane
    const int64_t want = (n2 + 1023) / 1024;
    const int blocks = (int)(want < (1 << 20) ? want : (1 << 20));
    hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(256), 0, stream,
                       reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), n2);
  }
  if (n & 1) hipLaunchKernelGGL(probe_copy_tail_kernel, dim3(1), dim3(1), 0, stream, src, dst, n - 1);
  return hipGetLastError();
}

}  // namespace wcns
