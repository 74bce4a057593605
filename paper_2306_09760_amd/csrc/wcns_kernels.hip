// Time-step and elementwise kernels of the WCNS-FE library on gfx950 (the
// directional sweeps are in wcns_sweep.hip).
//
//  cfl      two deterministic passes: per-block maxima of
//           sum_d (|u_d| + c)/h_d (wavefront shuffles, then LDS), then one
//           block that turns the maximum into dt = cfl / max.
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"

namespace wcns {

// --------------------------------------------------------------------- CFL --
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = (w > v) ? w : v;
  }
  return v;
}

// Block maximum for blockDim.x == 256; result valid in thread 0.
__device__ __forceinline__ double block_max256(double v) {
  __shared__ double red[4];
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  r = red[1] > r ? red[1] : r;
  r = red[2] > r ? red[2] : r;
  r = red[3] > r ? red[3] : r;
  __syncthreads();
  return r;
}

template <int NV>
__global__ void __launch_bounds__(256) cfl_partial_kernel(const double* __restrict__ U,
                                                          int64_t npts, double gamma,
                                                          double ih0, double ih1, double ih2,
                                                          double adv_rate,
                                                          double* __restrict__ partial) {
  double m = 0.0;
  if constexpr (NV == 1) {
    m = adv_rate;
  } else {
    constexpr int ND = NV - 2;
    const double ih[3] = {ih0, ih1, ih2};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts;
         i += (int64_t)gridDim.x * blockDim.x) {
      double u[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = U[v * npts + i];
      const double r = wave_rate<ND>(u, gamma, ih);
      // NaN-propagating max: a non-finite state gives a non-finite dt
      m = (r > m || r != r) ? r : m;
    }
  }
  m = block_max256(m);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) cfl_final_kernel(const double* __restrict__ partial,
                                                        int n, double cfl,
                                                        double* __restrict__ dt) {
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = partial[i];
    m = (r > m || r != r) ? r : m;
  }
  m = block_max256(m);
  if (threadIdx.x == 0) dt[0] = cfl / m;
}

// The batch maxima use wave_max_bits (wcns_device.hpp).
// dt_p = min(cfl / m, t_end - t_p) for a problem with t_p < t_end (0
// otherwise); t_p advances by dt_p.  A maximum rate m that is not positive and
// finite (a non-finite or non-physical state; NaN bit patterns order above
// every rate) stops the problem where it is: dt_p = 0, t_p unchanged, bit 0
// of *status set.
__device__ __forceinline__ void batch_dt(const BatchArgs& b, int p, double m, double* t,
                                         double t_end, double cfl, int32_t* status) {
  const double tp = t[p];
  if (!(m > 0.0 && m <= 1.79769313486231570815e308)) {
    b.dtp[p] = 0.0;
    if (status) atomicOr(status, 1);
    return;
  }
  double dt = cfl / m;
  double tn = tp + dt;
  if (!(dt < t_end - tp)) {
    dt = t_end - tp;
    tn = t_end;
  }
  b.dtp[p] = dt;
  t[p] = tn;
}

// One block per problem: the maximum wave rate of its nodes, then batch_dt.
// wmax, when given, is cleared for the fused maximum of the step's last stage.
__global__ void __launch_bounds__(256) batch_cfl_kernel(const double* __restrict__ U,
                                                        int64_t total, BatchArgs b,
                                                        double gamma, double* __restrict__ t,
                                                        double t_end, double cfl,
                                                        unsigned long long* wmax,
                                                        int32_t* status, int32_t* nlive) {
  __shared__ unsigned long long red[4];
  const int p = blockIdx.x;
  if (nlive && p == 0 && threadIdx.x == 0) *nlive = 0;
  if (wmax && threadIdx.x == 0) wmax[p] = 0;
  if (!(t[p] < t_end)) {  // uniform: the whole block leaves
    if (threadIdx.x == 0) b.dtp[p] = 0.0;
    return;
  }
  const int64_t o0 = b.offset[p], o1 = b.offset[p + 1];
  const double ih[1] = {b.ih[p]};
  unsigned long long m = 0;
  for (int64_t i = o0 + threadIdx.x; i < o1; i += blockDim.x) {
    double u[3] = {U[i], U[total + i], U[2 * total + i]};
    const unsigned long long r = __builtin_bit_cast(unsigned long long, wave_rate<1>(u, gamma, ih));
    m = r > m ? r : m;
  }
  m = wave_max_bits(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) m = red[w] > m ? red[w] : m;  // m = red[0] here
    batch_dt(b, p, __builtin_bit_cast(double, m), t, t_end, cfl, status);
  }
}

// The same dt from the maxima that the previous step's last stage took as it
// wrote the state (sweep kernel, SweepArgs::wmax); clears them for this
// step's.  One thread per problem.
__global__ void __launch_bounds__(256) batch_dt_kernel(BatchArgs b, double* __restrict__ t,
                                                       double t_end, double cfl,
                                                       unsigned long long* __restrict__ wmax,
                                                       int32_t* status, int32_t* nlive) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (nlive && p == 0) *nlive = 0;
  if (p >= b.nprob) return;
  const double m = __builtin_bit_cast(double, wmax[p]);
  wmax[p] = 0;
  if (!(t[p] < t_end)) {
    b.dtp[p] = 0.0;
    return;
  }
  batch_dt(b, p, m, t, t_end, cfl, status);
}

// The live-tile list: lane k tests tile k (live if one of its problems has
// dt > 0); each wavefront appends its live tiles in order with one atomic,
// so the list holds runs of up to 64 consecutive tiles.
__global__ void __launch_bounds__(256) batch_live_kernel(BatchArgs b, int32_t* __restrict__ live,
                                                         int32_t* __restrict__ nlive) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  bool on = false;
  if (k < b.ntiles) {
    const int p1 = b.tile_p1[k];
    for (int p = b.tile_p0[k]; p <= p1 && !on; ++p) on = b.dtp[p] != 0.0;
  }
  const unsigned long long mask = __ballot(on);
  if (mask == 0) return;  // uniform across the wavefront
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0) base = atomicAdd(nlive, __popcll(mask));
  base = __shfl(base, 0, 64);
  if (on) live[base + __popcll(mask & ((1ull << lane) - 1ull))] = k;
}

// ------------------------------------------------------------ elementwise --
__global__ void lincomb_kernel(double* __restrict__ out, const double* __restrict__ x, double ax,
                               const double* __restrict__ y, double ay,
                               const double* __restrict__ dt, double ydt, int64_t n) {
  // out = ax*x + (ay + ydt*dt)*y
  const double cy = ay + (dt ? ydt * dt[0] : 0.0);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r = cy * y[i];
    if (x) r = __builtin_fma(ax, x[i], r);
    out[i] = r;
  }
}

// --------------------------------------------------------------- launchers --
static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int cfl_blocks(int64_t npts) {
  int64_t b = ceil_div(npts, 256 * 8);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

hipError_t launch_cfl(int nv, int ndim, const double* U, int64_t npts, double gamma,
                      const double* ih, const double* adv, double cfl, double* partial,
                      int nblocks, double* dt_out, hipStream_t stream) {
  double adv_rate = 0.0;
  for (int d = 0; d < ndim; ++d) adv_rate += (adv[d] < 0 ? -adv[d] : adv[d]) * ih[d];
  const double ih0 = ih[0], ih1 = ndim > 1 ? ih[1] : 0.0, ih2 = ndim > 2 ? ih[2] : 0.0;
  switch (nv) {
    case 1:
      hipLaunchKernelGGL(cfl_partial_kernel<1>, dim3(nblocks), dim3(256), 0, stream, U, npts,
                         gamma, ih0, ih1, ih2, adv_rate, partial);
      break;
    case 3:
      hipLaunchKernelGGL(cfl_partial_kernel<3>, dim3(nblocks), dim3(256), 0, stream, U, npts,
                         gamma, ih0, ih1, ih2, adv_rate, partial);
      break;
    case 4:
      hipLaunchKernelGGL(cfl_partial_kernel<4>, dim3(nblocks), dim3(256), 0, stream, U, npts,
                         gamma, ih0, ih1, ih2, adv_rate, partial);
      break;
    case 5:
      hipLaunchKernelGGL(cfl_partial_kernel<5>, dim3(nblocks), dim3(256), 0, stream, U, npts,
                         gamma, ih0, ih1, ih2, adv_rate, partial);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cfl_final_kernel, dim3(1), dim3(256), 0, stream, partial, nblocks, cfl,
                     dt_out);
  return hipGetLastError();
}

hipError_t launch_batch_cfl(const double* U, int64_t total, const BatchArgs& b, double gamma,
                            double* t, double t_end, double cfl, unsigned long long* wmax,
                            int32_t* status, int32_t* nlive, hipStream_t stream) {
  hipLaunchKernelGGL(batch_cfl_kernel, dim3(b.nprob), dim3(256), 0, stream, U, total, b, gamma,
                     t, t_end, cfl, wmax, status, nlive);
  return hipGetLastError();
}

hipError_t launch_batch_dt(const BatchArgs& b, double* t, double t_end, double cfl,
                           unsigned long long* wmax, int32_t* status, int32_t* nlive,
                           hipStream_t stream) {
  hipLaunchKernelGGL(batch_dt_kernel, dim3((unsigned)ceil_div(b.nprob, 256)), dim3(256), 0,
                     stream, b, t, t_end, cfl, wmax, status, nlive);
  return hipGetLastError();
}

hipError_t launch_batch_live(const BatchArgs& b, int32_t* live, int32_t* nlive,
                             hipStream_t stream) {
  hipLaunchKernelGGL(batch_live_kernel, dim3((unsigned)ceil_div(b.ntiles, 256)), dim3(256), 0,
                     stream, b, live, nlive);
  return hipGetLastError();
}

static inline int elem_grid(int64_t n) {
  int64_t g = ceil_div(n, 256 * 4);
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (int)g;
}

hipError_t launch_lincomb(double* out, const double* x, double ax, const double* y, double ay,
                          const double* dt, double ydt, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(elem_grid(n)), dim3(256), 0, stream, out, x, ax, y, ay,
                     dt, ydt, n);
  return hipGetLastError();
}

hipError_t launch_axpy_state(double* y, const double* x, double a, int64_t n,
                             hipStream_t stream) {
  return launch_lincomb(y, y, 1.0, x, a, nullptr, 0.0, n, stream);
}

}  // namespace wcns
