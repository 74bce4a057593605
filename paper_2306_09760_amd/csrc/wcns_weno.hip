// Directional sweep of the filtered embedded WENO scheme of App. B on gfx950:
// finite-difference WENO5 with Lax-Friedrichs flux splitting and a
// conservative difference, same tile organisation as the WCNS sweep.
//
// A workgroup of 256 lanes owns TM midpoints (TM*W = 128) of W adjacent
// columns and writes the TL = TM - 1 nodes between them.  Phases:
//   load     the TM+5 nodes of every column into LDS, ghosts applied;
//   node     physical flux F(U) and wave speed |u_n| + c of every node;
//   mid      Roe state (vel, H, c, ic) of nodes m, m+1 and the splitting speed
//            alpha_m = max of the wave speed over the six stencil nodes;
//   recon    one task per (side, field, midpoint): the field-v projection of
//            f+ = (F + alpha U)/2 on the left-biased stencil (side 0) or of
//            f- = (F - alpha U)/2 on the mirrored one (side 1), then the WENO5
//            reconstruction;
//   flux     F~ = R (f+^ + f-^) per midpoint;
//   diff     -(F~_{i+1/2} - F~_{i-1/2}) / h, written as R, R+= or a stage.
// LDS (doubles): sU[NV][TM+5][W] | sF[NV][TM+5][W] | sL[TM+5][W] | sR[ND+3][TMW]
// | sA[TMW] | sW[2 NV][TMW] | the 64-entry exp table (FE specialisation).
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

template <int NV, int TM, int W>
struct WenoLayout {
  static constexpr int ND = NV > 1 ? NV - 2 : 1;
  static constexpr int NR = NV > 1 ? NV - 2 + 3 : 0;  // vel[ND], H, c, ic
  static constexpr int TN = TM + 5;
  static constexpr int TMW = TM * W;
  static constexpr int SV = TN * W;
  static constexpr int LW = W == 1 ? 0 : W == 2 ? 1 : W == 4 ? 2 : 3;
  static constexpr size_t lds_doubles =
      (size_t)(2 * NV + 1) * SV + (size_t)(NR + 1 + 2 * NV) * TMW + 64;
  static_assert(TMW == 128, "WENO tiles hold 128 midpoints");
};

template <int NV, int DIR, int SPEC, int TM, int W>
__global__ void __launch_bounds__(256) weno_sweep_kernel(SweepArgs a, TileGeom g, int mode) {
  using L = WenoLayout<NV, TM, W>;
  constexpr int ND = L::ND, NR = L::NR, TMW = L::TMW, SV = L::SV, LW = L::LW;
  constexpr int NT = 256;
  constexpr int TL = TM - 1;
  extern __shared__ double smem[];
  double* sU = smem;
  double* sF = sU + NV * SV;
  double* sL = sF + NV * SV;
  double* sR = sL + SV;
  double* sA = sR + NR * TMW;
  double* sW = sA + TMW;
  double* sX = sW + 2 * NV * TMW;  // kExp2Tab64
  const int tid = threadIdx.x;

  if ((int64_t)blockIdx.x >= g.ntiles) return;
  const int64_t tile = xcd_tile(blockIdx.x, g.ntiles);
  int64_t base, N, stride;
  int ncol = 1;
  // column groups fastest: adjacent groups split the same cache lines
  // tile < 2^31 (checked at launch): multiply-shift divisions
  const uint32_t t32 = (uint32_t)tile;
  const uint32_t r32 = g.dxg.div(t32);
  const uint32_t o32 = g.dseg.div(r32);
  const int64_t xg = t32 - r32 * (uint32_t)g.xgroups;
  const int64_t seg = r32 - o32 * (uint32_t)g.segs;
  const int64_t other = o32;
  const int64_t i0 = seg * TL;
  if constexpr (DIR == 0) {
    N = a.n[0];
    base = other * N;
    stride = 1;
  } else {
    const int64_t x0 = xg * W;
    ncol = (int)((a.n[0] - x0) < W ? (a.n[0] - x0) : W);
    if constexpr (DIR == 1) {
      N = a.n[1];
      stride = a.n[0];
      base = x0 + other * a.n[0] * a.n[1];
    } else {
      N = a.n[2];
      stride = a.n[0] * a.n[1];
      base = x0 + other * a.n[0];
    }
  }
  const double dt = (mode >= MODE_STAGE) ? *a.dt : 0.0;
  const int64_t nb = i0 - 3;  // position of LDS node 0; midpoint t is m = i0 - 1 + t

  // load
  if constexpr (SPEC == SPEC_FE) {
    if (tid < 64) sX[tid] = kExp2Tab64[tid];
  }
  for (int idx = tid; idx < SV; idx += NT) {
    const int k = idx >> LW, c = idx & (W - 1);
    const int cc = c < ncol ? c : ncol - 1;
    const int64_t gi = base + bc_index(nb + k, N, a.bc) * stride + cc;
#pragma unroll
    for (int v = 0; v < NV; ++v) sU[v * SV + idx] = a.U[v * a.npts + gi];
  }
  __syncthreads();

  const bool proj = (NV > 1) && a.pp.charproj;
  if constexpr (NV > 1) {
    // node fluxes and wave speeds
    for (int idx = tid; idx < SV; idx += NT) {
      double U[NV], F[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) U[v] = sU[v * SV + idx];
      euler_flux<ND, DIR>(U, a.pp.gamma, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[v * SV + idx] = F[v];
      sL[idx] = dir_speed<ND, DIR>(U, a.pp.gamma);
    }
    __syncthreads();
    // Roe state and splitting speed per midpoint
#pragma unroll 1
    for (int q = tid; q < TMW; q += NT) {
      double al = sL[q];
#pragma unroll
      for (int j = 1; j < 6; ++j) al = __builtin_fmax(al, sL[q + j * W]);
      sA[q] = al;
      if (proj) {
        const double* u = sU + q + 2 * W;
        double UA[NV], UB[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          UA[v] = u[v * SV];
          UB[v] = u[v * SV + W];
        }
        const RoeState<ND> rs = roe_average<ND>(UA, UB, a.pp.gamma);
        double* rr = sR + q;
#pragma unroll
        for (int k = 0; k < ND; ++k) rr[k * TMW] = rs.vel[k];
        rr[(ND + 0) * TMW] = rs.H;
        rr[(ND + 1) * TMW] = rs.c;
        rr[(ND + 2) * TMW] = rs.ic;
      }
    }
    __syncthreads();
  }

  // reconstruction, one task per (side, field, midpoint)
#pragma unroll 1
  for (int q = tid; q < 2 * NV * TMW; q += NT) {
    const int slot = q / TMW;
    const int rem = q - slot * TMW;
    const int side = slot >= NV;
    const int v = side ? slot - NV : slot;
    double w[5];
    if constexpr (NV == 1) {
      const double s = side ? 0.5 * (a.pp.adv - __builtin_fabs(a.pp.adv))
                            : 0.5 * (a.pp.adv + __builtin_fabs(a.pp.adv));
#pragma unroll
      for (int s5 = 0; s5 < 5; ++s5) w[s5] = s * sU[rem + (side ? 5 - s5 : s5) * W];
    } else {
      const double al = side ? -sA[rem] : sA[rem];
      // the split flux of node k: (F + al U) / 2, component e
      auto split = [&](int e, int k) { return 0.5 * __builtin_fma(al, sU[e * SV + k], sF[e * SV + k]); };
      if (proj) {
        const double* rr = sR + rem;
        if (v >= 2 && v < NV - 1) {  // shear field: X_ax - vel_ax X_rho
          const int ax = tangential_axis<ND, DIR>(v - 2);
          const double va = rr[ax * TMW];
#pragma unroll
          for (int s5 = 0; s5 < 5; ++s5) {
            const int k = rem + (side ? 5 - s5 : s5) * W;
            w[s5] = __builtin_fma(-va, split(0, k), split(1 + ax, k));
          }
        } else {
          RoeState<ND> rs;
#pragma unroll
          for (int k = 0; k < ND; ++k) rs.vel[k] = rr[k * TMW];
          rs.ic = rr[(ND + 2) * TMW];
          roe_derived<ND>(rs, a.pp.gamma);
          double l[NV];
          field_row<ND, DIR>(rs, v, l);
#pragma unroll
          for (int s5 = 0; s5 < 5; ++s5) {
            const int k = rem + (side ? 5 - s5 : s5) * W;
            double acc = l[0] * split(0, k);
#pragma unroll
            for (int e = 1; e < NV; ++e) acc = __builtin_fma(l[e], split(e, k), acc);
            w[s5] = acc;
          }
        }
      } else {
#pragma unroll
        for (int s5 = 0; s5 < 5; ++s5) w[s5] = split(v, rem + (side ? 5 - s5 : s5) * W);
      }
    }
    if constexpr (SPEC == SPEC_FE)
      sW[q] = weno5_fe<true>(a.ip, w[0], w[1], w[2], w[3], w[4], sX);
    else
      sW[q] = weno5(a.ip, w[0], w[1], w[2], w[3], w[4]);
  }
  __syncthreads();

  // midpoint flux F~ = R (f+^ + f-^) into sW rows 0..NV-1
#pragma unroll 1
  for (int q = tid; q < TMW; q += NT) {
    double G[NV], F[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) G[v] = sW[v * TMW + q] + sW[(NV + v) * TMW + q];
    if constexpr (NV > 1) {
      if (proj) {
        RoeState<ND> rs;
        const double* rr = sR + q;
#pragma unroll
        for (int k = 0; k < ND; ++k) rs.vel[k] = rr[k * TMW];
        rs.H = rr[(ND + 0) * TMW];
        rs.c = rr[(ND + 1) * TMW];
        rs.ic = rr[(ND + 2) * TMW];
        roe_derived<ND>(rs, a.pp.gamma);
        unproject<ND, DIR>(rs, G, F);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = G[v];
      }
    } else {
      F[0] = G[0];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sW[v * TMW + q] = F[v];
  }
  __syncthreads();

  // conservative difference
#pragma unroll 1
  for (int q = tid; q < TL * W; q += NT) {
    const int t = q >> LW, c = q & (W - 1);
    const int64_t i = i0 + t;
    if (i >= N || c >= ncol) continue;
    double res[NV], Un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double* fv = sW + v * TMW + q;   // F~ of midpoint t at fv[0], t + 1 at fv[W]
      res[v] = -a.ih * (fv[W] - fv[0]);
      Un[v] = sU[v * SV + q + 3 * W];
    }
    emit_rt<NV>(mode, a, base + i * stride + c, a.npts, res, Un, dt);
  }
}

// --------------------------------------------------------------- launchers --
template <int NV, int DIR, int TM, int W>
static hipError_t weno_go(const SweepArgs& a, int mode, hipStream_t s) {
  using L = WenoLayout<NV, TM, W>;
  static_assert(L::lds_doubles * sizeof(double) <= 64 * 1024, "WENO tile exceeds 64 KB of LDS");
  TileGeom g{};
  g.tm = TM;
  g.w = W;
  g.lw = L::LW;
  g.ltmw = 7;
  g.tl = TM - 1;
  g.segs = (a.n[DIR] + g.tl - 1) / g.tl;
  g.xgroups = DIR == 0 ? 1 : (a.n[0] + W - 1) / W;
  // (both below 2^31 whenever the tile count is, which the launch checks)
  g.dxg = fast_div((uint32_t)g.xgroups);
  g.dseg = fast_div((uint32_t)g.segs);
  const int64_t others = DIR == 0 ? a.n[1] * a.n[2] : (DIR == 1 ? a.n[2] : a.n[1]);
  g.ntiles = g.segs * g.xgroups * others;
  if (g.ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (spec_of(a.ip) == SPEC_FE)
    hipLaunchKernelGGL((weno_sweep_kernel<NV, DIR, SPEC_FE, TM, W>), dim3((unsigned)g.ntiles),
                       dim3(256), sizeof(double) * L::lds_doubles, s, a, g, mode);
  else
    hipLaunchKernelGGL((weno_sweep_kernel<NV, DIR, SPEC_GENERIC, TM, W>), dim3((unsigned)g.ntiles),
                       dim3(256), sizeof(double) * L::lds_doubles, s, a, g, mode);
  return hipGetLastError();
}

hipError_t launch_weno_sweep(int nv, int dir, const SweepArgs& a, int mode, hipStream_t stream) {
#define WCNS_W(NVV, DD, TMM, WW) \
  if (nv == NVV && dir == DD) return weno_go<NVV, DD, TMM, WW>(a, mode, stream);
  WCNS_W(1, 0, 128, 1) WCNS_W(1, 1, 32, 4) WCNS_W(1, 2, 32, 4)
  WCNS_W(3, 0, 128, 1)
  WCNS_W(4, 0, 128, 1) WCNS_W(4, 1, 32, 4)
  WCNS_W(5, 0, 128, 1) WCNS_W(5, 1, 32, 4) WCNS_W(5, 2, 32, 4)
#undef WCNS_W
  return hipErrorInvalidValue;
}

}  // namespace wcns
