// Forward kernels of the WCNS-FE residual on gfx950.
//
//  xsweep   lines along x (contiguous): one workgroup = one tile of TM
//           midpoints with the nodes staged in LDS; one lane per
//           (midpoint, field, side) interpolation, then the flux and the
//           difference (R, R+=, or the fused SSP-RK3 stage combine).  The same
//           kernel serves regular grids and ragged batches (a longest-first
//           tile table).
//  (the y/z sweeps are in wcns_march.hip)
//  cfl      two deterministic passes: per-block maxima of
//           sum_d (|u_d| + c)/h_d (wavefront shuffles, then LDS), then one
//           block that turns the maximum into dt = cfl / max.
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

// ------------------------------------------------------------------ xsweep --
// One workgroup = one tile of TM midpoints of one line, TM lanes by 2*NV
// slots (blockDim = (TM, 2 NV); TM is a multiple of 64, so the slot is uniform
// across a wavefront).  Phases, separated by barriers:
//   load   the TM + 5 nodes under the tile, ghosts applied, into LDS;
//   roe    slot 0: Roe average of the two nodes around each midpoint;
//   interp every lane: ONE nonlinear interpolation - field v = slot % NV of
//          the left-biased (slot < NV) or mirrored right-biased stencil,
//          projected on the fly from the LDS nodes;
//   flux   slot 0: back-projection of the two states and the LLF flux;
//   diff   slot 0, TL = TM - 3 (MND6) or TM - 5 (MD6) lanes: the flux
//          difference of one node and the output (R, R+= or stage combine).
// One interpolation per lane keeps the live state small (high occupancy);
// the interpolations are ~85% of the arithmetic.
// LDS (doubles): sU[NV][TM+5] | sR[NR][TM] | sW[2 NV][TM] | sF[NV][TM].
template <int NV>
struct XTile {
  static constexpr int ND = NV > 1 ? NV - 2 : 1;
  static constexpr int NR = NV > 1 ? NV - 2 + 6 : 0;  // vel[ND], H, c, ic, q2h, b1, b2
  static constexpr int kMaxTM = NV <= 3 ? 128 : 64;       // midpoints per tile (upper bound)
  static constexpr int kMaxThreads = kMaxTM * 2 * NV;
  static size_t lds_doubles(int tm) { return (size_t)NV * (tm + 5) + (size_t)(NR + 3 * NV) * tm; }
};

template <int NV, int MODE, bool BATCH, int SPEC>
__global__ void __launch_bounds__(XTile<NV>::kMaxThreads) xsweep_kernel(SweepArgs a, BatchArgs b, int64_t ntiles,
                                                      int64_t tiles_per_line) {
  constexpr int ND = XTile<NV>::ND;
  constexpr int NR = XTile<NV>::NR;
  extern __shared__ double smem[];
  const int TM = blockDim.x;
  const int TN = TM + 5;
  double* sU = smem;
  double* sR = sU + NV * TN;
  double* sW = sR + NR * TM;
  double* sF = sW + 2 * NV * TM;
  const int t = threadIdx.x;
  const int slot = threadIdx.y;
  const int tid = slot * TM + t;
  const int nthr = TM * blockDim.y;
  const int G = a.diff ? 5 : 4;
  const int TL = TM - (a.diff ? 5 : 3);

  const int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
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
      if (dt == 0.0) return;  // finished problem: uniform across the block
    }
  } else {
    const int64_t line = tile / tiles_per_line;
    i0 = (tile - line * tiles_per_line) * TL;
    N = a.n[0];
    base = line * N;
    if constexpr (MODE == MODE_STAGE) dt = *a.dt;
  }
  const int64_t nb = i0 - G;
  for (int idx = tid; idx < NV * TN; idx += nthr) {
    const int v = idx / TN, k = idx - v * TN;
    sU[v * TN + k] = a.U[v * a.npts + base + bc_index(nb + k, N, a.bc)];
  }
  __syncthreads();

  const bool proj = (NV > 1) && a.pp.charproj;
  if constexpr (NV > 1) {
    if (proj && slot == 0) {
      double UA[NV], UB[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UA[v] = sU[v * TN + t + 2];
        UB[v] = sU[v * TN + t + 3];
      }
      const RoeState<ND> r = roe_average<ND>(UA, UB, a.pp.gamma);
#pragma unroll
      for (int k = 0; k < ND; ++k) sR[k * TM + t] = r.vel[k];
      sR[(ND + 0) * TM + t] = r.H;
      sR[(ND + 1) * TM + t] = r.c;
      sR[(ND + 2) * TM + t] = r.ic;
      sR[(ND + 3) * TM + t] = r.q2h;
      sR[(ND + 4) * TM + t] = r.b1;
      sR[(ND + 5) * TM + t] = r.b2;
    }
    __syncthreads();
  }

  {  // one interpolation per lane
    const int side = slot >= NV;
    const int v = side ? slot - NV : slot;
    double w[5];
    if (proj) {
      if constexpr (NV > 1) {
        RoeState<ND> r;
#pragma unroll
        for (int k = 0; k < ND; ++k) r.vel[k] = sR[k * TM + t];
        r.ic = sR[(ND + 2) * TM + t];
        r.b1 = sR[(ND + 4) * TM + t];
        r.b2 = sR[(ND + 5) * TM + t];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const int j = side ? 5 - q : q;
          double U[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) U[c] = sU[c * TN + t + j];
          w[q] = project_field<ND, 0>(r, U, v);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 5; ++q) w[q] = sU[v * TN + t + (side ? 5 - q : q)];
    }
    sW[slot * TM + t] = interp5<SPEC>(a.ip, w[0], w[1], w[2], w[3], w[4]);
  }
  __syncthreads();

  if (slot == 0) {  // midpoint flux
    double F[NV];
    if constexpr (NV == 1) {
      const double uL = sW[t], uR = sW[TM + t];
      F[0] = 0.5 * a.pp.adv * (uL + uR) - 0.5 * __builtin_fabs(a.pp.adv) * (uR - uL);
    } else {
      double WL[NV], WR[NV], UL[NV], UR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        WL[v] = sW[v * TM + t];
        WR[v] = sW[(NV + v) * TM + t];
      }
      if (proj) {
        RoeState<ND> r;
#pragma unroll
        for (int k = 0; k < ND; ++k) r.vel[k] = sR[k * TM + t];
        r.H = sR[(ND + 0) * TM + t];
        r.c = sR[(ND + 1) * TM + t];
        r.q2h = sR[(ND + 3) * TM + t];
        unproject<ND, 0>(r, WL, UL);
        unproject<ND, 0>(r, WR, UR);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          UL[v] = WL[v];
          UR[v] = WR[v];
        }
      }
      llf_flux<ND, 0>(UL, UR, a.pp.gamma, F);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * TM + t] = F[v];
  }
  __syncthreads();

  const int64_t i = i0 + t;
  if (slot == 0 && t < TL && i < N) {
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
    emit<NV, MODE>(a, base + i, a.npts, res, Un, dt);
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

int xsweep_max_tm(int nv) {
  return nv <= 3 ? XTile<3>::kMaxTM : XTile<5>::kMaxTM;
}

int cfl_blocks(int64_t npts) {
  int64_t b = ceil_div(npts, 256 * 8);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

template <int NV, int MODE, bool BATCH>
static hipError_t xsweep_go(const SweepArgs& a, const BatchArgs& b, int tm, int64_t ntiles,
                            int64_t tpl, hipStream_t s) {
  if (tm > XTile<NV>::kMaxTM || tm % 64 != 0) return hipErrorInvalidConfiguration;
  const size_t lds = sizeof(double) * XTile<NV>::lds_doubles(tm);
  const dim3 block(tm, 2 * NV);
  if (spec_of(a.ip) == SPEC_FE)
    hipLaunchKernelGGL((xsweep_kernel<NV, MODE, BATCH, SPEC_FE>), dim3((unsigned)ntiles), block, lds,
                       s, a, b, ntiles, tpl);
  else
    hipLaunchKernelGGL((xsweep_kernel<NV, MODE, BATCH, SPEC_GENERIC>), dim3((unsigned)ntiles), block,
                       lds, s, a, b, ntiles, tpl);
  return hipGetLastError();
}

template <bool BATCH>
static hipError_t xsweep_dispatch(int nv, int mode, const SweepArgs& a, const BatchArgs& b,
                                  int tm, int64_t ntiles, int64_t tpl, hipStream_t s) {
#define WCNS_X(NVV)                                                                 \
  if (nv == NVV) {                                                                  \
    if (mode == MODE_RES) return xsweep_go<NVV, MODE_RES, BATCH>(a, b, tm, ntiles, tpl, s); \
    if (mode == MODE_ACC) return xsweep_go<NVV, MODE_ACC, BATCH>(a, b, tm, ntiles, tpl, s); \
    return xsweep_go<NVV, MODE_STAGE, BATCH>(a, b, tm, ntiles, tpl, s);       \
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
  if (ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  BatchArgs b{};
  return xsweep_dispatch<false>(nv, mode, a, b, tm, ntiles, tpl, stream);
}

hipError_t launch_batch_xsweep(const SweepArgs& a, const BatchArgs& b, int mode, int tm,
                               int grid, hipStream_t stream) {
  (void)grid;
  return xsweep_dispatch<true>(3, mode, a, b, tm, b.ntiles, 1, stream);
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
