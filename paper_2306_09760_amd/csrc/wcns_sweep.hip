// Directional sweep of the WCNS-FE residual on gfx950 (all directions and
// the ragged batch).
//
// A workgroup of 256 lanes owns one tile: TM midpoints along the sweep
// direction by W adjacent x-columns (W = 1 for the x direction; for y and z
// the columns make the global loads coalesced rows).  TM*W is 128 or 256.
// Phases, separated by barriers, with every lane looping over the phase's
// tasks (no wavefront idles while one phase belongs to a subset of lanes):
//   load    the TM+5 nodes of every column into LDS, ghosts applied;
//   roe     Roe average of the two nodes around each midpoint;
//   interp  one task = ONE nonlinear interpolation: field v of the
//           left-biased or mirrored right-biased stencil of one midpoint,
//           projected on the fly from the LDS nodes.  TM*W is a multiple of
//           64, so the field and side are uniform across a wavefront;
//   flux    back-projection of the two interpolated states and the local
//           Lax-Friedrichs flux;
//   diff    MND6 or MD6 flux difference of TL = TM-3 (TM-5) nodes per
//           column, written as R, R+= or the fused SSP-RK3 stage combine.
// One interpolation per task keeps the live state small (about 50 VGPRs),
// so occupancy, not the register file, bounds the kernel.
// LDS (doubles): sU[NV][TM+5][W] | sR[NR][TM*W] | sW[2 NV][TM*W]; the flux
// overwrites sW rows 0..NV-1 (each task reads its midpoint's two states
// before writing that midpoint's flux).
#include <hip/hip_runtime.h>

#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

template <int NV>
struct SweepLayout {
  static constexpr int ND = NV > 1 ? NV - 2 : 1;
  static constexpr int NR = NV > 1 ? NV - 2 + 6 : 0;  // vel[ND], H, c, ic, q2h, b1, b2
  static size_t lds_doubles(int tm, int w) {
    return (size_t)NV * (tm + 5) * w + (size_t)(NR + 2 * NV) * tm * w;
  }
};

template <int NV, int DIR, int MODE, bool BATCH, int SPEC>
__global__ void __launch_bounds__(256) sweep_kernel(SweepArgs a, BatchArgs b, TileGeom g) {
  constexpr int ND = SweepLayout<NV>::ND;
  constexpr int NR = SweepLayout<NV>::NR;
  extern __shared__ double smem[];
  const int TM = g.tm, W = g.w, LW = g.lw, LTMW = g.ltmw;
  const int TN = TM + 5, TMW = TM * W;
  double* sU = smem;
  double* sR = sU + NV * TN * W;
  double* sW = sR + NR * TMW;
  const int tid = threadIdx.x;
  constexpr int NT = 256;
  const int G = a.diff ? 5 : 4;

  const int64_t tile = blockIdx.x;
  if (tile >= g.ntiles) return;
  int64_t base, N, stride, i0;
  int ncol = 1;
  double ih = a.ih, dt = 0.0;
  if constexpr (BATCH) {
    const int p = b.tile_prob[tile];
    base = b.offset[p];
    N = b.offset[p + 1] - base;
    stride = 1;
    i0 = b.tile_i0[tile];
    ih = b.ih[p];
    if constexpr (MODE == MODE_STAGE) {
      dt = b.dtp[p];
      if (dt == 0.0) return;  // finished problem: uniform across the block
    }
  } else {
    const int64_t seg = tile % g.segs;
    const int64_t r = tile / g.segs;
    i0 = seg * g.tl;
    if constexpr (DIR == 0) {
      N = a.n[0];
      base = r * N;
      stride = 1;
    } else {
      const int64_t xg = r % g.xgroups;
      const int64_t other = r / g.xgroups;
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
    if constexpr (MODE == MODE_STAGE) dt = *a.dt;
  }
  const int64_t nb = i0 - G;

  // load
#pragma unroll
  for (int v = 0; v < NV; ++v)
    for (int idx = tid; idx < TN * W; idx += NT) {
      const int k = idx >> LW, c = idx & (W - 1);
      const int cc = c < ncol ? c : ncol - 1;
      sU[(v * TN + k) * W + c] = a.U[v * a.npts + base + bc_index(nb + k, N, a.bc) * stride + cc];
    }
  __syncthreads();

  const bool proj = (NV > 1) && a.pp.charproj;
  if constexpr (NV > 1) {
    if (proj) {
#pragma unroll 1
      for (int q = tid; q < TMW; q += NT) {
        const int m = q >> LW, c = q & (W - 1);
        double UA[NV], UB[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          UA[v] = sU[(v * TN + m + 2) * W + c];
          UB[v] = sU[(v * TN + m + 3) * W + c];
        }
        const RoeState<ND> rs = roe_average<ND>(UA, UB, a.pp.gamma);
#pragma unroll
        for (int k = 0; k < ND; ++k) sR[k * TMW + q] = rs.vel[k];
        sR[(ND + 0) * TMW + q] = rs.H;
        sR[(ND + 1) * TMW + q] = rs.c;
        sR[(ND + 2) * TMW + q] = rs.ic;
        sR[(ND + 3) * TMW + q] = rs.q2h;
        sR[(ND + 4) * TMW + q] = rs.b1;
        sR[(ND + 5) * TMW + q] = rs.b2;
      }
      __syncthreads();
    }
  }

  // one interpolation per task
#pragma unroll 1
  for (int q = tid; q < 2 * NV * TMW; q += NT) {
    const int slot = q >> LTMW;
    const int rem = q & (TMW - 1);
    const int m = rem >> LW, c = rem & (W - 1);
    const int side = slot >= NV;
    const int v = side ? slot - NV : slot;
    double w[5];
    if (proj) {
      if constexpr (NV > 1) {
        RoeState<ND> rs;
#pragma unroll
        for (int k = 0; k < ND; ++k) rs.vel[k] = sR[k * TMW + rem];
        rs.ic = sR[(ND + 2) * TMW + rem];
        rs.b1 = sR[(ND + 4) * TMW + rem];
        rs.b2 = sR[(ND + 5) * TMW + rem];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          const int k = m + (side ? 5 - s : s);
          double U[NV];
#pragma unroll
          for (int e = 0; e < NV; ++e) U[e] = sU[(e * TN + k) * W + c];
          w[s] = project_field<ND, DIR>(rs, U, v);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < 5; ++s) w[s] = sU[(v * TN + m + (side ? 5 - s : s)) * W + c];
    }
    sW[slot * TMW + rem] = interp5<SPEC>(a.ip, w[0], w[1], w[2], w[3], w[4]);
  }
  __syncthreads();

  // midpoint flux (overwrites sW rows 0..NV-1 of the same midpoint)
#pragma unroll 1
  for (int q = tid; q < TMW; q += NT) {
    double F[NV];
    if constexpr (NV == 1) {
      const double uL = sW[q], uR = sW[TMW + q];
      F[0] = 0.5 * a.pp.adv * (uL + uR) - 0.5 * __builtin_fabs(a.pp.adv) * (uR - uL);
    } else {
      double WL[NV], WR[NV], UL[NV], UR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        WL[v] = sW[v * TMW + q];
        WR[v] = sW[(NV + v) * TMW + q];
      }
      if (proj) {
        RoeState<ND> rs;
#pragma unroll
        for (int k = 0; k < ND; ++k) rs.vel[k] = sR[k * TMW + q];
        rs.H = sR[(ND + 0) * TMW + q];
        rs.c = sR[(ND + 1) * TMW + q];
        rs.q2h = sR[(ND + 3) * TMW + q];
        unproject<ND, DIR>(rs, WL, UL);
        unproject<ND, DIR>(rs, WR, UR);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          UL[v] = WL[v];
          UR[v] = WR[v];
        }
      }
      llf_flux<ND, DIR>(UL, UR, a.pp.gamma, F);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sW[v * TMW + q] = F[v];
  }
  __syncthreads();

  // flux difference and output
  const double* sF = sW;
#pragma unroll 1
  for (int q = tid; q < g.tl * W; q += NT) {
    const int t = q >> LW, c = q & (W - 1);
    const int64_t i = i0 + t;
    if (i >= N || c >= ncol) continue;
    double res[NV], Un[NV];
    if (a.diff == 0) {
      double Um[NV], Up[NV], Fm[NV], Fp[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Um[v] = sU[(v * TN + t + 3) * W + c];
        Un[v] = sU[(v * TN + t + 4) * W + c];
        Up[v] = sU[(v * TN + t + 5) * W + c];
      }
      node_flux<NV, DIR>(a.pp, Um, Fm);
      node_flux<NV, DIR>(a.pp, Up, Fp);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double* f = sF + v * TMW + t * W + c;  // f[k W] = F~ at midpoint t + k
        const double d = 1.5 * (f[2 * W] - f[W]) - 0.3 * (Fp[v] - Fm[v]) +
                         (1.0 / 30.0) * (f[3 * W] - f[0]);
        res[v] = -ih * d;
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Un[v] = sU[(v * TN + t + 5) * W + c];
        const double* f = sF + v * TMW + t * W + c;
        const double d = (75.0 / 64.0) * (f[3 * W] - f[2 * W]) +
                         (-25.0 / 384.0) * (f[4 * W] - f[W]) + (3.0 / 640.0) * (f[5 * W] - f[0]);
        res[v] = -ih * d;
      }
    }
    emit<NV, MODE>(a, base + i * stride + c, a.npts, res, Un, dt);
  }
}

// --------------------------------------------------------------- launchers --
static inline int64_t ceil_div64(int64_t x, int64_t y) { return (x + y - 1) / y; }
static inline int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

bool sweep_shape_ok(int nv, int dir, int tm, int w) {
  if (tm < 16 || w < 1 || (tm & (tm - 1)) || (w & (w - 1))) return false;
  if (dir == 0 && w != 1) return false;
  const int tmw = tm * w;
  if (tmw != 128 && tmw != 256) return false;
  const size_t lds = sizeof(double) * ((size_t)nv * (tm + 5) * w + (size_t)(nv + 4 + 2 * nv) * tmw);
  return lds <= 64 * 1024;
}

template <int NV, int DIR, int MODE, bool BATCH>
static hipError_t sweep_go(const SweepArgs& a, const BatchArgs& b, const TileGeom& g,
                           hipStream_t s) {
  const size_t lds = sizeof(double) * SweepLayout<NV>::lds_doubles(g.tm, g.w);
  if (spec_of(a.ip) == SPEC_FE)
    hipLaunchKernelGGL((sweep_kernel<NV, DIR, MODE, BATCH, SPEC_FE>), dim3((unsigned)g.ntiles),
                       dim3(256), lds, s, a, b, g);
  else
    hipLaunchKernelGGL((sweep_kernel<NV, DIR, MODE, BATCH, SPEC_GENERIC>),
                       dim3((unsigned)g.ntiles), dim3(256), lds, s, a, b, g);
  return hipGetLastError();
}

template <int NV, int DIR, bool BATCH>
static hipError_t sweep_mode(int mode, const SweepArgs& a, const BatchArgs& b, const TileGeom& g,
                             hipStream_t s) {
  if (mode == MODE_RES) return sweep_go<NV, DIR, MODE_RES, BATCH>(a, b, g, s);
  if (mode == MODE_ACC) return sweep_go<NV, DIR, MODE_ACC, BATCH>(a, b, g, s);
  return sweep_go<NV, DIR, MODE_STAGE, BATCH>(a, b, g, s);
}

static TileGeom make_geom(int dir, const int64_t n[3], int diff, int tm, int w) {
  TileGeom g;
  g.tm = tm;
  g.w = w;
  g.lw = ilog2(w);
  g.ltmw = ilog2(tm * w);
  g.tl = tm - (diff ? 5 : 3);
  g.segs = ceil_div64(n[dir], g.tl);
  g.xgroups = dir == 0 ? 1 : ceil_div64(n[0], w);
  const int64_t others = dir == 0 ? n[1] * n[2] : (dir == 1 ? n[2] : n[1]);
  g.ntiles = g.segs * g.xgroups * others;
  return g;
}

hipError_t launch_sweep(int nv, int dir, const SweepArgs& a, int mode, int tm, int w,
                        hipStream_t stream) {
  if (!sweep_shape_ok(nv, dir, tm, w)) return hipErrorInvalidConfiguration;
  const TileGeom g = make_geom(dir, a.n, a.diff, tm, w);
  if (g.ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  BatchArgs b{};
#define WCNS_S(NVV, DD) \
  if (nv == NVV && dir == DD) return sweep_mode<NVV, DD, false>(mode, a, b, g, stream);
  WCNS_S(1, 0) WCNS_S(1, 1) WCNS_S(1, 2)
  WCNS_S(3, 0)
  WCNS_S(4, 0) WCNS_S(4, 1)
  WCNS_S(5, 0) WCNS_S(5, 1) WCNS_S(5, 2)
#undef WCNS_S
  return hipErrorInvalidValue;
}

hipError_t launch_batch_sweep(const SweepArgs& a, const BatchArgs& b, int mode, int tm,
                              hipStream_t stream) {
  if (!sweep_shape_ok(3, 0, tm, 1)) return hipErrorInvalidConfiguration;
  TileGeom g;
  g.tm = tm;
  g.w = 1;
  g.lw = 0;
  g.ltmw = ilog2(tm);
  g.tl = tm - (a.diff ? 5 : 3);
  g.segs = 1;
  g.xgroups = 1;
  g.ntiles = b.ntiles;
  return sweep_mode<3, 0, true>(mode, a, b, g, stream);
}

}  // namespace wcns
