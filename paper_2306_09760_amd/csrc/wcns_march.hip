// y/z sweeps of the WCNS-FE residual on gfx950 (lines strided in memory).
//
// Lanes run across x so every load is a coalesced row segment; each lane
// marches along its line (y or z) over a segment of SEG nodes, keeping the
// six-node stencil and the last midpoint fluxes in registers (a sliding
// window), so each midpoint flux is computed once per segment and the
// difference, the accumulation of earlier directions and the SSP-RK3 stage
// combine are fused into the same pass.
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------- march --
template <int NV>
__device__ __forceinline__ void load_node(const double* U, int64_t npts, int64_t idx,
                                          double (&x)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] = U[v * npts + idx];
}

template <int NV, int DIR, int MODE, int DIFF, int SPEC>
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
    midpoint_flux<NV, DIR, SPEC>(a.ip, a.pp, s, Fh[NF - 1]);
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

template <int NV, int DIR, int MODE, int DIFF>
static hipError_t march_go(const SweepArgs& a, int seg, int bw, hipStream_t s) {
  const int64_t N = (DIR == 1) ? a.n[1] : a.n[2];
  const int64_t others = (DIR == 1) ? a.n[2] : a.n[1];
  const int nseg = (int)ceil_div(N, seg);
  if (others * nseg > 65535) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)ceil_div(a.n[0], bw), (unsigned)(others * nseg));
  if (spec_of(a.ip) == SPEC_FE)
    hipLaunchKernelGGL((march_kernel<NV, DIR, MODE, DIFF, SPEC_FE>), grid, dim3(bw), 0, s, a, seg,
                       nseg);
  else
    hipLaunchKernelGGL((march_kernel<NV, DIR, MODE, DIFF, SPEC_GENERIC>), grid, dim3(bw), 0, s, a,
                       seg, nseg);
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

}  // namespace wcns
