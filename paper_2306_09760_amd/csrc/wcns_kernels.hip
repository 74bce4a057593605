// Forward kernels of the WCNS-FE residual on gfx950.
//
//  xsweep   lines along x (contiguous): one workgroup = one tile of TM
//           midpoints; the TM+5 nodes under it are staged in LDS with the
//           boundary ghosts applied, each lane computes one midpoint flux into
//           LDS, then TM-3 (MND6) or TM-5 (MD6) lanes form the flux
//           difference of one node each and write R, R+=, or the fused
//           SSP-RK3 stage combine.  The same kernel serves regular grids and
//           ragged batches (a tile table), looping over tiles persistently.
//  march    lines along y or z (strided): lanes run across x so every load
//           is a coalesced row segment; each lane marches along its line
//           over a segment, keeping the six-node stencil and the last
//           midpoint fluxes in registers (a sliding window), so each
//           midpoint flux is computed once per segment.
//  cfl      two deterministic passes: per-block maxima of
//           sum_d (|u_d| + c)/h_d (wavefront shuffles, then LDS), then one
//           block that turns the maximum into dt = cfl / max.
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"

namespace wcns {

__device__ __forceinline__ int64_t bc_index(int64_t j, int64_t N, int bc) {
  if (bc == 0) {  // periodic
    j %= N;
    return j < 0 ? j + N : j;
  }
  return j < 0 ? 0 : (j >= N ? N - 1 : j);  // transmissive: zeroth-order copy
}

__device__ __forceinline__ void flag_status(int32_t* status) {
  if (status) atomicOr(status, 1);
}

// Writes one node's result according to the sweep mode.  Un is the state
// under the stencil at that node (needed by the stage combine).
template <int NV, int MODE>
__device__ __forceinline__ void emit(const SweepArgs& a, int64_t gidx, int64_t vstride,
                                     const double (&res)[NV], const double (&Un)[NV],
                                     double dt) {
  if constexpr (MODE == MODE_RES) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = res[v];
  } else if constexpr (MODE == MODE_ACC) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = a.Rin[v * vstride + gidx] + res[v];
  } else {
    double y[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = res[v];
      if (a.Rin) r += a.Rin[v * vstride + gidx];
      double s = a.cb * __builtin_fma(dt, r, Un[v]);
      if (a.ca != 0.0) s = __builtin_fma(a.ca, a.U0[v * vstride + gidx], s);
      y[v] = s;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = y[v];
    if (!physical<NV>(y, a.pp.gamma)) flag_status(a.status);
  }
}

// ------------------------------------------------------------------ xsweep --
// LDS: sU[v][TM+5] then sF[v][TM] (doubles), TM = blockDim.x.
template <int NV, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) xsweep_kernel(SweepArgs a, BatchArgs b, int64_t ntiles,
                                                     int64_t tiles_per_line) {
  extern __shared__ double smem[];
  const int TM = blockDim.x;
  const int TN = TM + 5;
  double* sU = smem;
  double* sF = smem + NV * TN;
  const int t = threadIdx.x;
  const int G = a.diff ? 5 : 4;
  const int TL = TM - (a.diff ? 5 : 3);

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int64_t base, N, i0;
    double ih = a.ih, dt = 0.0;
    if constexpr (BATCH) {
      const int p = b.tile_prob[tile];
      base = b.offset[p];
      N = b.offset[p + 1] - base;
      i0 = b.tile_i0[tile];
      ih = b.ih[p];
      if constexpr (MODE == MODE_STAGE) {
        dt = b.dtp[p];
        if (dt == 0.0) continue;  // finished problem (uniform across the block)
      }
    } else {
      const int64_t line = tile / tiles_per_line;
      i0 = (tile - line * tiles_per_line) * TL;
      N = a.n[0];
      base = line * N;
      if constexpr (MODE == MODE_STAGE) dt = *a.dt;
    }
    const int64_t nb = i0 - G;
    __syncthreads();  // LDS reuse across tiles
#pragma unroll
    for (int v = 0; v < NV; ++v)
      for (int k = t; k < TN; k += TM)
        sU[v * TN + k] = a.U[v * a.npts + base + bc_index(nb + k, N, a.bc)];
    __syncthreads();
    {
      double s[6][NV], F[NV];
#pragma unroll
      for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) s[j][v] = sU[v * TN + t + j];
      midpoint_flux<NV, 0>(a.ip, a.pp, s, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[v * TM + t] = F[v];
    }
    __syncthreads();
    const int64_t i = i0 + t;
    if (t < TL && i < N) {
      double res[NV], Un[NV];
      if (a.diff == 0) {
        double Um[NV], Up[NV], Fm[NV], Fp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Um[v] = sU[v * TN + t + 3];
          Un[v] = sU[v * TN + t + 4];
          Up[v] = sU[v * TN + t + 5];
        }
        node_flux<NV, 0>(a.pp, Um, Fm);
        node_flux<NV, 0>(a.pp, Up, Fp);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double* f = sF + v * TM + t;
          const double d = 1.5 * (f[2] - f[1]) - 0.3 * (Fp[v] - Fm[v]) + (1.0 / 30.0) * (f[3] - f[0]);
          res[v] = -ih * d;
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Un[v] = sU[v * TN + t + 5];
          const double* f = sF + v * TM + t;
          const double d = (75.0 / 64.0) * (f[3] - f[2]) + (-25.0 / 384.0) * (f[4] - f[1]) +
                           (3.0 / 640.0) * (f[5] - f[0]);
          res[v] = -ih * d;
        }
      }
      const int64_t vstride = a.npts;
      emit<NV, MODE>(a, base + i, vstride, res, Un, dt);
    }
  }
}

// ------------------------------------------------------------------- march --
template <int NV>
__device__ __forceinline__ void load_node(const double* U, int64_t npts, int64_t idx,
                                          double (&x)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] = U[v * npts + idx];
}

template <int NV, int DIR, int MODE, int DIFF>
__global__ void __launch_bounds__(256) march_kernel(SweepArgs a, int seg, int nseg) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nx = a.n[0];
  if (x >= nx) return;
  const int64_t other = blockIdx.y / nseg;
  const int64_t sidx = blockIdx.y - other * nseg;
  int64_t N, stride, base;
  if constexpr (DIR == 1) {
    N = a.n[1];
    stride = nx;
    base = x + nx * a.n[1] * other;
  } else {
    N = a.n[2];
    stride = nx * a.n[1];
    base = x + nx * other;
  }
  const int64_t j0 = sidx * seg;
  const int64_t j1 = (j0 + seg < N) ? j0 + seg : N;
  double dt = 0.0;
  if constexpr (MODE == MODE_STAGE) dt = *a.dt;

  constexpr int NF = DIFF ? 6 : 4;   // midpoint fluxes in the window
  constexpr int LAG = DIFF ? 2 : 1;  // output node j = m - LAG
  double s[6][NV];
  double Fh[NF][NV];
  const int64_t mstart = j0 - (DIFF ? 3 : 2);
#pragma unroll
  for (int k = 0; k < 6; ++k) load_node<NV>(a.U, a.npts, base + bc_index(mstart - 2 + k, N, a.bc) * stride, s[k]);

  for (int64_t m = mstart; m <= j1 - 1 + (DIFF ? 2 : 1); ++m) {
#pragma unroll
    for (int q = 0; q < NF - 1; ++q)
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[q][v] = Fh[q + 1][v];
    midpoint_flux<NV, DIR>(a.ip, a.pp, s, Fh[NF - 1]);
    const int64_t j = m - LAG;
    if (j >= j0) {
      double res[NV], Un[NV];
      if constexpr (DIFF == 0) {
        // window: s[0] = node j-1, s[1] = node j, s[2] = node j+1;
        // Fh[0..3] = F~ at j-3/2, j-1/2, j+1/2, j+3/2.
        double Fm[NV], Fp[NV];
        node_flux<NV, DIR>(a.pp, s[0], Fm);
        node_flux<NV, DIR>(a.pp, s[2], Fp);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Un[v] = s[1][v];
          const double d = 1.5 * (Fh[2][v] - Fh[1][v]) - 0.3 * (Fp[v] - Fm[v]) +
                           (1.0 / 30.0) * (Fh[3][v] - Fh[0][v]);
          res[v] = -a.ih * d;
        }
      } else {
        // s[0] = node j, Fh[0..5] = F~ at j-5/2 .. j+5/2.
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Un[v] = s[0][v];
          const double d = (75.0 / 64.0) * (Fh[3][v] - Fh[2][v]) +
                           (-25.0 / 384.0) * (Fh[4][v] - Fh[1][v]) +
                           (3.0 / 640.0) * (Fh[5][v] - Fh[0][v]);
          res[v] = -a.ih * d;
        }
      }
      emit<NV, MODE>(a, base + j * stride, a.npts, res, Un, dt);
    }
    // Slide the stencil: drop node m-2, load node m+4.
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) s[k][v] = s[k + 1][v];
    load_node<NV>(a.U, a.npts, base + bc_index(m + 4, N, a.bc) * stride, s[5]);
  }
}

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

// One block per problem: dt_p = min(cfl / max rate, t_end - t_p) for
// problems with t_p < t_end (0 otherwise); t_p advances by dt_p.
__global__ void __launch_bounds__(256) batch_cfl_kernel(const double* __restrict__ U,
                                                        int64_t total, BatchArgs b,
                                                        double gamma, double* __restrict__ t,
                                                        double t_end, double cfl) {
  const int p = blockIdx.x;
  const double tp = t[p];
  if (!(tp < t_end)) {  // uniform: the whole block leaves
    if (threadIdx.x == 0) b.dtp[p] = 0.0;
    return;
  }
  const int64_t o0 = b.offset[p], o1 = b.offset[p + 1];
  const double ih[1] = {b.ih[p]};
  double m = 0.0;
  for (int64_t i = o0 + threadIdx.x; i < o1; i += blockDim.x) {
    double u[3] = {U[i], U[total + i], U[2 * total + i]};
    const double r = wave_rate<1>(u, gamma, ih);
    m = (r > m || r != r) ? r : m;
  }
  m = block_max256(m);
  if (threadIdx.x == 0) {
    double dt = cfl / m;
    double tn = tp + dt;
    if (!(dt < t_end - tp)) {
      dt = t_end - tp;
      tn = t_end;
    }
    b.dtp[p] = dt;
    t[p] = tn;
  }
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

__global__ void zero_kernel(double* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = 0.0;
}

// --------------------------------------------------------------- launchers --
static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int cfl_blocks(int64_t npts) {
  int64_t b = ceil_div(npts, 256 * 8);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

template <int NV, int MODE, bool BATCH>
static hipError_t xsweep_go(const SweepArgs& a, const BatchArgs& b, int tm, int64_t ntiles,
                            int64_t tpl, int grid, hipStream_t s) {
  const size_t lds = sizeof(double) * NV * (2 * tm + 5);
  hipLaunchKernelGGL((xsweep_kernel<NV, MODE, BATCH>), dim3(grid), dim3(tm), lds, s, a, b,
                     ntiles, tpl);
  return hipGetLastError();
}

template <bool BATCH>
static hipError_t xsweep_dispatch(int nv, int mode, const SweepArgs& a, const BatchArgs& b,
                                  int tm, int64_t ntiles, int64_t tpl, int grid, hipStream_t s) {
#define WCNS_X(NVV)                                                                 \
  if (nv == NVV) {                                                                  \
    if (mode == MODE_RES) return xsweep_go<NVV, MODE_RES, BATCH>(a, b, tm, ntiles, tpl, grid, s); \
    if (mode == MODE_ACC) return xsweep_go<NVV, MODE_ACC, BATCH>(a, b, tm, ntiles, tpl, grid, s); \
    return xsweep_go<NVV, MODE_STAGE, BATCH>(a, b, tm, ntiles, tpl, grid, s);       \
  }
  if constexpr (BATCH) {
    WCNS_X(3)
  } else {
    WCNS_X(1)
    WCNS_X(3)
    WCNS_X(4)
    WCNS_X(5)
  }
#undef WCNS_X
  return hipErrorInvalidValue;
}

hipError_t launch_xsweep(int nv, const SweepArgs& a, int mode, int tm, hipStream_t stream) {
  const int TL = tm - (a.diff ? 5 : 3);
  const int64_t tpl = ceil_div(a.n[0], TL);
  const int64_t lines = a.n[1] * a.n[2];
  const int64_t ntiles = tpl * lines;
  const int64_t grid = ntiles < (1 << 30) ? ntiles : (1 << 30);
  BatchArgs b{};
  return xsweep_dispatch<false>(nv, mode, a, b, tm, ntiles, tpl, (int)grid, stream);
}

hipError_t launch_batch_xsweep(const SweepArgs& a, const BatchArgs& b, int mode, int tm,
                               int grid, hipStream_t stream) {
  return xsweep_dispatch<true>(3, mode, a, b, tm, b.ntiles, 1, grid, stream);
}

template <int NV, int DIR, int MODE, int DIFF>
static hipError_t march_go(const SweepArgs& a, int seg, int bw, hipStream_t s) {
  const int64_t N = (DIR == 1) ? a.n[1] : a.n[2];
  const int64_t others = (DIR == 1) ? a.n[2] : a.n[1];
  const int nseg = (int)ceil_div(N, seg);
  if (others * nseg > 65535) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)ceil_div(a.n[0], bw), (unsigned)(others * nseg));
  hipLaunchKernelGGL((march_kernel<NV, DIR, MODE, DIFF>), grid, dim3(bw), 0, s, a, seg, nseg);
  return hipGetLastError();
}

template <int NV, int DIR>
static hipError_t march_mode(int mode, const SweepArgs& a, int seg, int bw, hipStream_t s) {
  if (a.diff == 0) {
    if (mode == MODE_RES) return march_go<NV, DIR, MODE_RES, 0>(a, seg, bw, s);
    if (mode == MODE_ACC) return march_go<NV, DIR, MODE_ACC, 0>(a, seg, bw, s);
    return march_go<NV, DIR, MODE_STAGE, 0>(a, seg, bw, s);
  }
  if (mode == MODE_RES) return march_go<NV, DIR, MODE_RES, 1>(a, seg, bw, s);
  if (mode == MODE_ACC) return march_go<NV, DIR, MODE_ACC, 1>(a, seg, bw, s);
  return march_go<NV, DIR, MODE_STAGE, 1>(a, seg, bw, s);
}

hipError_t launch_march(int nv, int dir, const SweepArgs& a, int mode, int seg, int bw,
                        hipStream_t stream) {
  if (nv == 1 && dir == 1) return march_mode<1, 1>(mode, a, seg, bw, stream);
  if (nv == 1 && dir == 2) return march_mode<1, 2>(mode, a, seg, bw, stream);
  if (nv == 4 && dir == 1) return march_mode<4, 1>(mode, a, seg, bw, stream);
  if (nv == 5 && dir == 1) return march_mode<5, 1>(mode, a, seg, bw, stream);
  if (nv == 5 && dir == 2) return march_mode<5, 2>(mode, a, seg, bw, stream);
  return hipErrorInvalidValue;
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
                            double* t, double t_end, double cfl, hipStream_t stream) {
  hipLaunchKernelGGL(batch_cfl_kernel, dim3(b.nprob), dim3(256), 0, stream, U, total, b, gamma,
                     t, t_end, cfl);
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

hipError_t launch_zero(double* y, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(zero_kernel, dim3(elem_grid(n)), dim3(256), 0, stream, y, n);
  return hipGetLastError();
}

}  // namespace wcns
