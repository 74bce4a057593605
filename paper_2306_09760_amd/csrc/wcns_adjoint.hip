// Adjoint (vector-Jacobian product) of the WCNS-FE residual on gfx950:
// Ubar += scale * (dL/dU)^T Rbar, one direction at a time, in gather form.
//
//  adj_midpoint  one lane per midpoint: forms the midpoint-flux cotangent from
//                Rbar (transpose of the flux difference), recomputes the
//                forward midpoint flux and propagates the cotangent back to
//                its six stencil nodes; the 6*NV contributions are stored in a
//                midpoint-major buffer (variable-major, x fastest, so both
//                writes and later reads are coalesced).
//  adj_gather    one lane per node: sums the contributions of every (midpoint,
//                stencil slot) that reads this node (ghost positions folded
//                back through the boundary map) and the node-flux term of
//                the midpoint-and-node difference.  No atomics: the result
//                is deterministic.
#include <hip/hip_runtime.h>

#include "wcns_adjoint_device.hpp"
#include "wcns_internal.hpp"

namespace wcns {

struct AdjGeom {
  int64_t n[3];      // node grid
  int64_t nm[3];     // midpoint grid (n with n[dir] replaced by nmid)
  int64_t Mtot;      // product of nm
  int64_t N;         // n[dir]
  int64_t mlo, mhi;  // midpoint range along dir (m + 1/2 between nodes m, m+1)
  int64_t stride;    // node stride along dir
};

__device__ __forceinline__ int64_t wrap_or_clamp(int64_t j, int64_t N, int bc) {
  if (bc == 0) {
    j %= N;
    return j < 0 ? j + N : j;
  }
  return j < 0 ? 0 : (j >= N ? N - 1 : j);
}

// Rbar at position j along the line (0 outside a transmissive line).
__device__ __forceinline__ double rbar_at(const double* Rb, int64_t base, int64_t stride,
                                          int64_t j, int64_t N, int bc) {
  if (bc == 0) return Rb[base + wrap_or_clamp(j, N, 0) * stride];
  if (j < 0 || j >= N) return 0.0;
  return Rb[base + j * stride];
}

template <int NV, int DIR, int SPEC>
__global__ void __launch_bounds__(256) adj_midpoint_kernel(AdjArgs a, AdjGeom g) {
  const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lin >= g.Mtot) return;
  int64_t c[3];
  c[0] = lin % g.nm[0];
  const int64_t rest = lin / g.nm[0];
  c[1] = rest % g.nm[1];
  c[2] = rest / g.nm[1];
  const int64_t m = g.mlo + c[DIR];
  c[DIR] = 0;
  const int64_t base = c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
  const int64_t N = g.N;
  // Cotangent of the midpoint flux F~_{m+1/2} (transpose of the difference).
  double Fb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double* Rb = a.Rbar + v * a.npts;
    auto R = [&](int64_t j) { return rbar_at(Rb, base, g.stride, j, N, a.bc); };
    double d;
    if (a.diff == 0)
      d = 1.5 * (R(m) - R(m + 1)) + (1.0 / 30.0) * (R(m - 1) - R(m + 2));
    else
      d = (75.0 / 64.0) * (R(m) - R(m + 1)) + (-25.0 / 384.0) * (R(m - 1) - R(m + 2)) +
          (3.0 / 640.0) * (R(m - 2) - R(m + 3));
    Fb[v] = -a.ih * d;
  }
  double s[6][NV], sb[6][NV];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int64_t idx = base + wrap_or_clamp(m - 2 + k, N, a.bc) * g.stride;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      s[k][v] = a.U[v * a.npts + idx];
      sb[k][v] = 0.0;
    }
  }
  midpoint_flux_vjp<NV, DIR, SPEC>(a.ip, a.pp, s, Fb, sb);
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v) a.contrib[(k * NV + v) * g.Mtot + lin] = sb[k][v];
}

template <int NV, int DIR>
__global__ void __launch_bounds__(256) adj_gather_kernel(AdjArgs a, AdjGeom g) {
  const int64_t np = a.npts;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= np) return;
  int64_t c[3];
  c[0] = node % g.n[0];
  const int64_t rest = node / g.n[0];
  c[1] = rest % g.n[1];
  c[2] = rest / g.n[1];
  const int64_t i = c[DIR];
  const int64_t N = g.N;
  int64_t cm[3] = {c[0], c[1], c[2]};
  cm[DIR] = 0;
  const int64_t mbase = cm[0] + g.nm[0] * (cm[1] + g.nm[1] * cm[2]);
  const int64_t mstride = (DIR == 0) ? 1 : (DIR == 1 ? g.nm[0] : g.nm[0] * g.nm[1]);
  const int G = a.diff ? 5 : 4;

  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  auto gather_pos = [&](int64_t pos) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int64_t m = pos + 2 - k;
      if (m >= g.mlo && m <= g.mhi) {
        const int64_t l = mbase + (m - g.mlo) * mstride;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += a.contrib[(k * NV + v) * g.Mtot + l];
      }
    }
  };
  gather_pos(i);
  if (a.bc == 0) {
    gather_pos(i - N);
    gather_pos(i + N);
  } else {
    if (i == 0)
      for (int q = 1; q <= G; ++q) gather_pos(-q);
    if (i == N - 1)
      for (int q = 0; q < G; ++q) gather_pos(N + q);
  }
  if (a.diff == 0) {
    // Node-flux term: F_j enters D_{j+1} with +3/10 and D_{j-1} with -3/10.
    const int64_t base = node - i * g.stride;
    double Fb[NV], U[NV], Ub[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double* Rb = a.Rbar + v * np;
      auto R = [&](int64_t j) { return rbar_at(Rb, base, g.stride, j, N, a.bc); };
      double f = -0.3 * a.ih * (R(i + 1) - R(i - 1));
      if (a.bc != 0) {
        if (i == 0) f += -0.3 * a.ih * (R(0) - R(-2));          // ghost node -1
        if (i == N - 1) f += -0.3 * a.ih * (R(N + 1) - R(N - 1)); // ghost node N
      }
      Fb[v] = f;
      U[v] = a.U[v * np + node];
      Ub[v] = 0.0;
    }
    node_flux_vjp<NV, DIR>(a.pp, U, Fb, Ub);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += Ub[v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) a.Ubar[v * np + node] += a.scale * acc[v];
}

static AdjGeom make_geom(int dir, const int64_t n[3], int diff, int bc) {
  AdjGeom g;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = n[k];
    g.nm[k] = n[k];
  }
  g.N = n[dir];
  if (bc == 0) {
    g.mlo = 0;
    g.mhi = g.N - 1;
  } else {
    g.mlo = diff ? -3 : -2;
    g.mhi = diff ? g.N + 1 : g.N;
  }
  g.nm[dir] = g.mhi - g.mlo + 1;
  g.Mtot = g.nm[0] * g.nm[1] * g.nm[2];
  g.stride = (dir == 0) ? 1 : (dir == 1 ? n[0] : n[0] * n[1]);
  return g;
}

size_t adjoint_contrib_elems(int nv, int dir, const int64_t n[3], int diff) {
  AdjGeom g = make_geom(dir, n, diff, 1);
  return (size_t)6 * nv * g.Mtot;
}

template <int NV, int DIR>
static hipError_t adj_go(const AdjArgs& a, hipStream_t s) {
  const AdjGeom g = make_geom(DIR, a.n, a.diff, a.bc);
  const int64_t b1 = (g.Mtot + 255) / 256;
  if (spec_of(a.ip) == SPEC_FE)
    hipLaunchKernelGGL((adj_midpoint_kernel<NV, DIR, SPEC_FE>), dim3((unsigned)b1), dim3(256), 0, s,
                       a, g);
  else
    hipLaunchKernelGGL((adj_midpoint_kernel<NV, DIR, SPEC_GENERIC>), dim3((unsigned)b1), dim3(256),
                       0, s, a, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t b2 = (a.npts + 255) / 256;
  hipLaunchKernelGGL((adj_gather_kernel<NV, DIR>), dim3((unsigned)b2), dim3(256), 0, s, a, g);
  return hipGetLastError();
}

hipError_t launch_adjoint_dir(int nv, int dir, const AdjArgs& a, hipStream_t stream) {
  if (nv == 1 && dir == 0) return adj_go<1, 0>(a, stream);
  if (nv == 1 && dir == 1) return adj_go<1, 1>(a, stream);
  if (nv == 1 && dir == 2) return adj_go<1, 2>(a, stream);
  if (nv == 3 && dir == 0) return adj_go<3, 0>(a, stream);
  if (nv == 4 && dir == 0) return adj_go<4, 0>(a, stream);
  if (nv == 4 && dir == 1) return adj_go<4, 1>(a, stream);
  if (nv == 5 && dir == 0) return adj_go<5, 0>(a, stream);
  if (nv == 5 && dir == 1) return adj_go<5, 1>(a, stream);
  if (nv == 5 && dir == 2) return adj_go<5, 2>(a, stream);
  return hipErrorInvalidValue;
}

}  // namespace wcns
