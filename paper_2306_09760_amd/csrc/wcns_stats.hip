// Histograms of the interpolation weights of one residual evaluation
// (App. A statistics of the Z, FE and PFE weights).  A diagnostic pass, not
// part of the residual: one lane per (line, midpoint) evaluates the same
// interpolations as the residual sweep (every field, left and mirrored right
// stencil) and counts, per weight k, three quantities into 64-bit bins:
//   kind 0  the normalised JS/Z weights omega_k,
//   kind 1  their FE images g_k(omega_k) / sum_l g_l(omega_l),
//   kind 2  the weights the configured scheme uses (PFE: switched).
// Bin b of nbins covers [b/nbins, (b+1)/nbins); 1.0 falls in the last bin.
// The weights follow the generic instantiation of the interpolation (one
// reciprocal per Z weight), so that weights equal to d_k on flat stencils are
// exactly d_k.
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

struct StatsGeom {
  int64_t nlines, nmid, mlo;  // lines, midpoints per line, first midpoint
  int64_t N, stride;          // nodes and node stride along the direction
};

__device__ __forceinline__ void interp_weights(const InterpParams& P, double a, double b,
                                               double c, double e, double f, double (&wb)[3],
                                               double (&wm)[3], double (&wo)[3]) {
  const double d0 = b - a, d1 = c - b, d2 = e - c, d3 = f - e;
  const double f0 = 0.5 * (3.0 * d1 - d0), s0 = d1 - d0;
  const double f1 = 0.5 * (d1 + d2), s1 = d2 - d1;
  const double f2 = 0.5 * (3.0 * d2 - d3), s2 = d3 - d2;
  const double IS0 = f0 * f0 + s0 * s0, IS1 = f1 * f1 + s1 * s1, IS2 = f2 * f2 + s2 * s2;
  double a0, a1, a2;
  if (P.weights == WLIN) {
    a0 = D0;
    a1 = D1;
    a2 = D2;
  } else if (P.weights == WJS) {
    const double r0 = rcp(IS0 + P.eps), r1 = rcp(IS1 + P.eps), r2 = rcp(IS2 + P.eps);
    a0 = D0 * r0 * r0;
    a1 = D1 * r1 * r1;
    a2 = D2 * r2 * r2;
  } else {
    const double tau = __builtin_fabs(IS0 - IS2);
    const double q0 = tau * rcp(IS0 + P.eps), q1 = tau * rcp(IS1 + P.eps), q2 = tau * rcp(IS2 + P.eps);
    double p0 = q0, p1 = q1, p2 = q2;
    for (int k = 1; k < P.zpow; ++k) {
      p0 *= q0;
      p1 *= q1;
      p2 *= q2;
    }
    a0 = D0 * (1.0 + p0);
    a1 = D1 * (1.0 + p1);
    a2 = D2 * (1.0 + p2);
  }
  const double inv = rcp(a0 + a1 + a2);
  wb[0] = a0 * inv;
  wb[1] = a1 * inv;
  wb[2] = a2 * inv;
  const double g0 = fe_g0<SPEC_GENERIC>(wb[0], P), g1 = fe_g1<SPEC_GENERIC>(wb[1], P),
               g2 = fe_g2<SPEC_GENERIC>(wb[2], P);
  const double gi = rcp(g0 + g1 + g2);
  wm[0] = g0 * gi;
  wm[1] = g1 * gi;
  wm[2] = g2 * gi;
  bool map = P.weights == WFE;
  if (P.weights == WPFE)
    map = !(__builtin_fabs(wb[0] - D0) <= P.cv && __builtin_fabs(wb[1] - D1) <= P.cv &&
            __builtin_fabs(wb[2] - D2) <= P.cv);
  for (int k = 0; k < 3; ++k) wo[k] = map ? wm[k] : wb[k];
}

__device__ __forceinline__ void count_bin(unsigned long long* h, double w, int nbins) {
  int bin = (int)(w * (double)nbins);
  bin = bin < 0 ? 0 : (bin >= nbins ? nbins - 1 : bin);
  atomicAdd(h + bin, 1ULL);
}

template <int NV, int DIR>
__global__ void __launch_bounds__(256) weight_hist_kernel(SweepArgs a, StatsGeom g,
                                                          unsigned long long* hist, int nbins) {
  const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lin >= g.nlines * g.nmid) return;
  const int64_t line = lin / g.nmid;
  const int64_t m = g.mlo + lin % g.nmid;
  int64_t base;
  if constexpr (DIR == 0) {
    base = line * a.n[0];
  } else if constexpr (DIR == 1) {
    base = line % a.n[0] + (line / a.n[0]) * a.n[0] * a.n[1];
  } else {
    base = line;  // (x, y) of the z-line: x + n0 y
  }
  double s[6][NV];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int64_t gi = base + bc_index(m - 2 + j, g.N, a.bc) * g.stride;
#pragma unroll
    for (int v = 0; v < NV; ++v) s[j][v] = a.U[v * a.npts + gi];
  }
  double W[6][NV];
  if constexpr (NV > 1) {
    constexpr int ND = NV - 2;
    if (a.pp.charproj) {
      const RoeState<ND> rs = roe_average<ND>(s[2], s[3], a.pp.gamma);
#pragma unroll
      for (int j = 0; j < 6; ++j) project<ND, DIR>(rs, s[j], W[j]);
    } else {
#pragma unroll
      for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) W[j][v] = s[j][v];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 6; ++j) W[j][0] = s[j][0];
  }
#pragma unroll 1
  for (int v = 0; v < NV; ++v)
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
      double w[5];
      for (int k = 0; k < 5; ++k) w[k] = side == 0 ? W[k][v] : W[5 - k][v];
      double wb[3], wm[3], wo[3];
      interp_weights(a.ip, w[0], w[1], w[2], w[3], w[4], wb, wm, wo);
      for (int k = 0; k < 3; ++k) {
        count_bin(hist + (0 * 3 + k) * (int64_t)nbins, wb[k], nbins);
        count_bin(hist + (1 * 3 + k) * (int64_t)nbins, wm[k], nbins);
        count_bin(hist + (2 * 3 + k) * (int64_t)nbins, wo[k], nbins);
      }
    }
}

template <int NV, int DIR>
static hipError_t hist_go(const SweepArgs& a, unsigned long long* hist, int nbins, hipStream_t s) {
  StatsGeom g;
  g.N = a.n[DIR];
  g.stride = DIR == 0 ? 1 : (DIR == 1 ? a.n[0] : a.n[0] * a.n[1]);
  g.nlines = a.n[0] * a.n[1] * a.n[2] / g.N;
  const int G = a.diff ? 5 : 4;
  if (a.bc == 0) {
    g.mlo = 0;
    g.nmid = g.N;
  } else {
    g.mlo = -G + 2;
    g.nmid = g.N + 2 * G - 5;
  }
  const int64_t total = g.nlines * g.nmid;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((weight_hist_kernel<NV, DIR>), dim3((unsigned)blocks), dim3(256), 0, s, a, g,
                     hist, nbins);
  return hipGetLastError();
}

hipError_t launch_weight_hist(int nv, int dir, const SweepArgs& a, unsigned long long* hist,
                              int nbins, hipStream_t stream) {
#define WCNS_H(NVV, DD) \
  if (nv == NVV && dir == DD) return hist_go<NVV, DD>(a, hist, nbins, stream);
  WCNS_H(1, 0) WCNS_H(1, 1) WCNS_H(1, 2)
  WCNS_H(3, 0)
  WCNS_H(4, 0) WCNS_H(4, 1)
  WCNS_H(5, 0) WCNS_H(5, 1) WCNS_H(5, 2)
#undef WCNS_H
  return hipErrorInvalidValue;
}

}  // namespace wcns
