// Device helpers shared by the sweep kernels: boundary index map, status
// flag and the per-node epilogue (R, R+= or the fused SSP-RK3 stage combine).
#pragma once

#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"

namespace wcns {

__device__ __forceinline__ int64_t bc_index(int64_t j, int64_t N, int bc) {
  if (bc == 0) {  // periodic: one wrap covers the ghosts; a general modulo otherwise
    if (j < 0) j += N;
    if (j >= N) j -= N;
    if (j < 0 || j >= N) {
      j %= N;
      if (j < 0) j += N;
    }
    return j;
  }
  return j < 0 ? 0 : (j >= N ? N - 1 : j);  // transmissive: zeroth-order copy
}

__device__ __forceinline__ void flag_status(int32_t* status) {
  if (status) atomicOr(status, 1);
}

// Writes one node's result according to the sweep mode (MODE_RES, MODE_ACC,
// MODE_STAGE or MODE_LIN; `mode` is uniform, so the switch costs a scalar
// branch).
template <int NV>
__device__ __forceinline__ void emit_rt(int mode, const SweepArgs& a, int64_t gidx, int64_t vstride,
                                        const double (&res)[NV], const double (&Un)[NV],
                                        double dt);

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
  } else if constexpr (MODE == MODE_LIN) {
    double y[NV];
    const double crdt = a.cr * dt;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = res[v];
      if (a.Rin) r += a.Rin[v * vstride + gidx];
      double s = __builtin_fma(crdt, r, a.cb * Un[v]);
      if (a.ca != 0.0) s = __builtin_fma(a.ca, a.U0[v * vstride + gidx], s);
      y[v] = s;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = y[v];
    if (!physical<NV>(y, a.pp.gamma)) flag_status(a.status);
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

template <int NV>
__device__ __forceinline__ void emit_rt(int mode, const SweepArgs& a, int64_t gidx, int64_t vstride,
                                        const double (&res)[NV], const double (&Un)[NV],
                                        double dt) {
  if (mode == MODE_RES)
    emit<NV, MODE_RES>(a, gidx, vstride, res, Un, dt);
  else if (mode == MODE_ACC)
    emit<NV, MODE_ACC>(a, gidx, vstride, res, Un, dt);
  else if (mode == MODE_STAGE)
    emit<NV, MODE_STAGE>(a, gidx, vstride, res, Un, dt);
  else
    emit<NV, MODE_LIN>(a, gidx, vstride, res, Un, dt);
}

}  // namespace wcns
