// Adjoint (vector-Jacobian product) of the WCNS-FE residual on gfx950, one
// direction per launch: Ubar += s (dL/dU)^T Rbar, or, for the first direction
// of a step's stage, Ubar = ca A + cb B + cc C + s (dL/dU)^T Rbar (s = scale,
// times *dt when given; see AdjArgs).
//
// A workgroup of 256 lanes owns the nodes i0 .. i0+TL-1 (TL = TM - 5) of W
// adjacent lines and recomputes the TM midpoints i0-3 .. i0+TL+1 whose
// fluxes read them, so every node's cotangent is completed inside one tile
// (no atomics: the result is deterministic and independent of the launch
// shape's scheduling).  Phases, separated by barriers:
//   load     the TM+5 nodes of every column into LDS, ghosts applied;
//   roe      Roe average per midpoint;
//   interp   forward interpolation, one task per (field, midpoint), both
//            sides, with the gradient of each interpolated value with
//            respect to its five stencil values (interp5_grad: the same
//            intermediates give both);
//   flux     per midpoint: flux cotangent from Rbar (transpose of the MND6 /
//            MD6 difference), local Lax-Friedrichs VJP, back-projection VJP
//            -> cotangents of the interpolated characteristic values and of
//            the Roe quantities;
//   interp^T one task per (field, midpoint): the cotangents of the six
//            projected stencil values, the two interpolations' gradients
//            times their values' cotangents (no second evaluation of the
//            weights);
//   proj^T   per midpoint: projection VJP of the six stencil nodes (in place
//            in LDS) and the Roe-average VJP onto the two centre nodes;
//   gather   per node: the six midpoint contributions, ghost positions folded
//            onto the boundary node (transmissive), the node-flux term of
//            MND6, and the epilogue above.
// LDS (doubles): sU[NV][TM+5][W] | sR[NR][TMW] | sWB[12 NV][TMW] | sRB[NV][TM+5][W]
// | the 64-entry exp table, TMW = TM W.  Slot s of task (field v, midpoint
// q) is sWB[(s NV + v) TMW + q]: slots 0, 1 hold the left and right
// interpolated values, then their cotangents; slots 2-6 and 7-11 the two
// gradients; the interpolation VJP overwrites slots 0-5 with the cotangents
// of the six stencil values (each task reads its own slots first).  sRB holds
// Rbar of the tile's nodes for the flux VJP.  The Roe-quantity cotangent of a
// midpoint stays in its lane's registers from the flux VJP to the projection
// VJP.
#include <hip/hip_runtime.h>

#include "wcns_adjoint_device.hpp"
#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

template <int NV, int TM, int W>
struct AdjLayout {
  static constexpr int ND = NV > 1 ? NV - 2 : 1;
  static constexpr int NR = NV > 1 ? NV - 2 + 6 : 0;
  static constexpr int TN = TM + 5;
  static constexpr int TMW = TM * W;
  static constexpr int SV = TN * W;
  static constexpr int LW = W == 1 ? 0 : W == 2 ? 1 : W == 4 ? 2 : W == 8 ? 3 : 4;
  static constexpr int LTMW = TMW == 64 ? 6 : TMW == 128 ? 7 : 8;
  static constexpr int NS = 12;  // LDS slots per (field, midpoint) task
  static constexpr size_t lds_doubles =
      2 * (size_t)NV * SV + (size_t)(NR + NS * NV) * TMW + 64;
  static_assert(TMW == 64 || TMW == 128 || TMW == 256, "tile must hold 64, 128 or 256 midpoints");
  static_assert((1 << LW) == W, "W must be a power of two up to 16");
  // Workgroups (of four waves) a CU's 160 KB of LDS holds, at most four:
  // the waves per SIMD, and so the register budget, of the instance.
  static constexpr int per_cu = (int)((160 * 1024) / (lds_doubles * sizeof(double)));
  static constexpr int waves = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
};

// Register budget for the waves per SIMD that the tile's LDS allows.
template <int NV, int DIR, int SPEC, int TM, int W>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(AdjLayout<NV, TM, W>::waves)))
    adj_sweep_kernel(AdjArgs a, TileGeom g) {
  using L = AdjLayout<NV, TM, W>;
  constexpr int ND = L::ND, NR = L::NR, TMW = L::TMW, SV = L::SV;
  constexpr int LW = L::LW, LTMW = L::LTMW;
  constexpr int NT = 256;
  constexpr int TL = TM - 5;
  extern __shared__ double smem[];
  static_assert(TMW <= NT, "one midpoint per lane in the per-midpoint phases");
  constexpr int NS = L::NS;
  double* sU = smem;
  double* sR = sU + NV * SV;
  double* sWB = sR + NR * TMW;
  // Interpolated values and their cotangents: left field v in row v, right in
  // row NV + v (slots 0 and 1).
  double* sW = sWB;
  double* sRB = sWB + NS * NV * TMW;  // Rbar of the tile's nodes
  double* sX = sRB + NV * SV;         // kExp2Tab64
  constexpr bool TAB = SPEC == SPEC_FE;
  const int tid = threadIdx.x;

  if ((int64_t)blockIdx.x >= g.ntiles) return;
  const int64_t tile = xcd_tile(blockIdx.x, g.ntiles);
  // Along x the lines are packed end to end with 5 ghost slots on each side
  // (TileGeom::lines, L = n[0] + 10): every position a node's cotangent
  // gathers from (nodes j-5 .. j+5) then lies in its own line's slots.
  constexpr int P = 5;
  int64_t base = 0, N, stride = 1, i0;
  int ncol = 1;
  BatchTile bt{};
  bool near = true;  // the tile spans at most two lines
  if constexpr (DIR == 0) {
    N = a.n[0];
    i0 = tile * TL;
    bt = line_tile(i0, N, g.lines, P, TL, g.inv_line);
    near = bt.p1 <= bt.p0 + 1;
  } else {
    // column groups fastest: adjacent groups split the same cache lines
    // tile < 2^31 (checked at launch): multiply-shift divisions
    const uint32_t t32 = (uint32_t)tile;
    const uint32_t r32 = g.dxg.div(t32);
    const uint32_t o32 = g.dseg.div(r32);
    const int64_t xg = t32 - r32 * (uint32_t)g.xgroups;
    const int64_t seg = r32 - o32 * (uint32_t)g.segs;
    const int64_t other = o32;
    i0 = seg * TL;
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
  const int64_t nb = i0 - 5;  // position of LDS node 0

  // load: all global reads of the tile issued before the first LDS write
  constexpr int NIT = (SV + NT - 1) / NT;
  static_assert(NIT <= 2, "a tile holds at most two nodes per lane");
  // Rbar of the same nodes (the transposed difference of the flux VJP reads
  // nodes m-2 .. m+3 of every midpoint m) goes to sRB.
  double buf[NIT][NV], rbuf[NIT][NV];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = tid + it * NT;
    if (idx < SV) {
      const int k = idx >> LW, c = idx & (W - 1);
      const int cc = c < ncol ? c : ncol - 1;
      if constexpr (DIR == 0) {
        const BatchSlot sl =
            near ? batch_slot_near(bt, k - P) : line_slot(nb + k, N, g.lines, P, g.inv_line);
        // slots before the first line or after the last load a ghost (no
        // node gathers from them)
        const int j = sl.j < -P ? -P : (sl.j >= sl.n + P ? sl.n + P - 1 : sl.j);
        const int64_t gi = sl.o + bc_index_near(j, sl.n, a.bc);
        const bool ghost = j < 0 || j >= sl.n;
#pragma unroll
        for (int v = 0; v < NV; ++v) buf[it][v] = a.U[v * a.npts + gi];
#pragma unroll
        for (int v = 0; v < NV; ++v)  // Rbar: zero at a transmissive ghost
          rbuf[it][v] = (ghost && a.bc != 0) ? 0.0 : a.Rbar[v * a.npts + gi];
      } else {
        // one index for both arrays: Rbar is zero where a transmissive
        // line's ghost copies its end node
        const int64_t j = nb + k;
        const int64_t gi = base + bc_index(j, N, a.bc) * stride + cc;
        const bool ghost = a.bc != 0 && (j < 0 || j >= N);
#pragma unroll
        for (int v = 0; v < NV; ++v) buf[it][v] = a.U[v * a.npts + gi];
#pragma unroll
        for (int v = 0; v < NV; ++v) rbuf[it][v] = ghost ? 0.0 : a.Rbar[v * a.npts + gi];
      }
    }
  }
  double xv = 0.0;
  if constexpr (TAB) {
    if (tid < 64) xv = kExp2Tab64[tid];
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = tid + it * NT;
    if (idx < SV) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        sU[v * SV + idx] = buf[it][v];
        sRB[v * SV + idx] = rbuf[it][v];
      }
    }
  }
  if constexpr (TAB) {
    if (tid < 64) sX[tid] = xv;
  }
  __syncthreads();

  const bool proj = (NV > 1) && a.pp.charproj;
  if constexpr (NV > 1) {
    if (proj) {
#pragma unroll 1
      for (int q = tid; q < TMW; q += NT) {
        const double* u = sU + q + 2 * W;  // nodes m, m+1 of midpoint q
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
        rr[(ND + 3) * TMW] = rs.q2h;
        rr[(ND + 4) * TMW] = rs.b1;
        rr[(ND + 5) * TMW] = rs.b2;
      }
      __syncthreads();
    }
  }

  auto load_roe = [&](int q) {
    RoeState<ND> rs;
    const double* rr = sR + q;
#pragma unroll
    for (int k = 0; k < ND; ++k) rs.vel[k] = rr[k * TMW];
    rs.H = rr[(ND + 0) * TMW];
    rs.c = rr[(ND + 1) * TMW];
    rs.ic = rr[(ND + 2) * TMW];
    rs.q2h = rr[(ND + 3) * TMW];
    rs.b1 = rr[(ND + 4) * TMW];
    rs.b2 = rr[(ND + 5) * TMW];
    return rs;
  };
  // the six (projected) stencil values of field v around midpoint rem
  auto stencil = [&](int rem, int v, double (&w)[6]) {
    const double* u = sU + rem;
    if (proj) {
      if constexpr (NV > 1) {
        const double* rr = sR + rem;
        if (v >= 2 && v < NV - 1) {  // shear field: m_ax - vel_ax rho
          const int ax = tangential_axis<ND, DIR>(v - 2);
          const double va = rr[ax * TMW];
#pragma unroll
          for (int s = 0; s < 6; ++s) w[s] = __builtin_fma(-va, u[s * W], u[(1 + ax) * SV + s * W]);
        } else {
          RoeState<ND> rs;
#pragma unroll
          for (int k = 0; k < ND; ++k) rs.vel[k] = rr[k * TMW];
          rs.ic = rr[(ND + 2) * TMW];
          rs.b1 = rr[(ND + 4) * TMW];
          rs.b2 = rr[(ND + 5) * TMW];
          double l[NV];
          field_row<ND, DIR>(rs, v, l);
#pragma unroll
          for (int s = 0; s < 6; ++s) {
            double acc = l[0] * u[s * W];
#pragma unroll
            for (int e = 1; e < NV; ++e) acc = __builtin_fma(l[e], u[e * SV + s * W], acc);
            w[s] = acc;
          }
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < 6; ++s) w[s] = u[v * SV + s * W];
    }
  };

  // forward interpolation, one task per (field, midpoint): both sides, each
  // with its gradient (slots 2-6: left, over w[0..4]; 7-11: right, over
  // w[5], w[4], .., w[1])
#pragma unroll 1
  for (int q = tid; q < NV * TMW; q += NT) {
    double w[6], G[5];
    stencil(q & (TMW - 1), q >> LTMW, w);
    sW[q] = interp5_grad<SPEC, TAB>(a.ip, w[0], w[1], w[2], w[3], w[4], G, sX);
#pragma unroll
    for (int j = 0; j < 5; ++j) sWB[(2 + j) * NV * TMW + q] = G[j];
    sW[NV * TMW + q] = interp5_grad<SPEC, TAB>(a.ip, w[5], w[4], w[3], w[2], w[1], G, sX);
#pragma unroll
    for (int j = 0; j < 5; ++j) sWB[(7 + j) * NV * TMW + q] = G[j];
  }
  __syncthreads();

  // flux VJP per midpoint: sW <- cotangents of the interpolated values; the
  // cotangent of the Roe quantities stays in this lane's registers until the
  // projection VJP below
  RoeBar<ND> rb;
#pragma unroll
  for (int k = 0; k < ND; ++k) rb.vel[k] = 0.0;
  rb.H = rb.c = rb.ic = rb.q2h = rb.b1 = rb.b2 = 0.0;
  if (tid < TMW) {
    const int q = tid;
    const int t = q >> LW, c = q & (W - 1);
    double Fb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // Rbar at node m + d (m = i0 - 3 + t) is staged at LDS node t + 2 + d
      const double* Rb = sRB + v * SV + t * W + c;
      const double r0 = Rb[2 * W], r1 = Rb[3 * W], rm1 = Rb[W], r2 = Rb[4 * W];
      double d;
      if (a.diff == 0) {
        d = 1.5 * (r0 - r1) + (1.0 / 30.0) * (rm1 - r2);
      } else {
        const double rm2 = Rb[0], r3 = Rb[5 * W];
        d = (75.0 / 64.0) * (r0 - r1) + (-25.0 / 384.0) * (rm1 - r2) + (3.0 / 640.0) * (rm2 - r3);
      }
      Fb[v] = -a.ih * d;
    }
    if constexpr (NV == 1) {
      sW[q] = 0.5 * (a.pp.adv + __builtin_fabs(a.pp.adv)) * Fb[0];
      sW[TMW + q] = 0.5 * (a.pp.adv - __builtin_fabs(a.pp.adv)) * Fb[0];
    } else {
      double WL[NV], WR[NV], UL[NV], UR[NV], ULb[NV], URb[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        WL[v] = sW[v * TMW + q];
        WR[v] = sW[(NV + v) * TMW + q];
      }
      if (proj) {
        const RoeState<ND> rs = load_roe(q);
        unproject<ND, DIR>(rs, WL, UL);
        unproject<ND, DIR>(rs, WR, UR);
        llf_vjp<ND, DIR>(UL, UR, a.pp.gamma, Fb, ULb, URb);
        double WLb[NV], WRb[NV];
        unproject_vjp<ND, DIR>(rs, WL, ULb, WLb, rb);
        unproject_vjp<ND, DIR>(rs, WR, URb, WRb, rb);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          sW[v * TMW + q] = WLb[v];
          sW[(NV + v) * TMW + q] = WRb[v];
        }
      } else {
        llf_vjp<ND, DIR>(WL, WR, a.pp.gamma, Fb, ULb, URb);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          sW[v * TMW + q] = ULb[v];
          sW[(NV + v) * TMW + q] = URb[v];
        }
      }
    }
  }
  __syncthreads();

  // interpolation VJP, one task per (field, midpoint): slot j <- cotangent
  // of stencil value j of the field, from the task's own slots (the
  // neighbouring tasks write the other fields' rows)
#pragma unroll 1
  for (int q = tid; q < NV * TMW; q += NT) {
    const double ybL = sWB[q], ybR = sWB[NV * TMW + q];
    double GL[5], GR[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      GL[j] = sWB[(2 + j) * NV * TMW + q];
      GR[j] = sWB[(7 + j) * NV * TMW + q];
    }
    double wb[6];
    wb[0] = ybL * GL[0];
#pragma unroll
    for (int j = 1; j < 5; ++j) wb[j] = __builtin_fma(ybR, GR[5 - j], ybL * GL[j]);
    wb[5] = ybR * GR[0];
#pragma unroll
    for (int j = 0; j < 6; ++j) sWB[j * NV * TMW + q] = wb[j];
  }
  __syncthreads();

  // projection and Roe-average VJP per midpoint (in place: slot j's NV rows)
  if constexpr (NV > 1) {
    if (proj) {
      if (tid < TMW) {
        const int q = tid;
        const RoeState<ND> rs = load_roe(q);
        const double* u = sU + q;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          double U[NV], Wb[NV], Ub[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            U[v] = u[v * SV + j * W];
            Wb[v] = sWB[(j * NV + v) * TMW + q];
            Ub[v] = 0.0;
          }
          project_vjp<ND, DIR>(rs, U, Wb, Ub, rb);
#pragma unroll
          for (int v = 0; v < NV; ++v) sWB[(j * NV + v) * TMW + q] = Ub[v];
        }
        double UA[NV], UB[NV], UbA[NV], UbB[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          UA[v] = u[v * SV + 2 * W];
          UB[v] = u[v * SV + 3 * W];
          UbA[v] = 0.0;
          UbB[v] = 0.0;
        }
        roe_vjp<ND>(UA, UB, a.pp.gamma, rs, rb, UbA, UbB);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          sWB[(2 * NV + v) * TMW + q] += UbA[v];
          sWB[(3 * NV + v) * TMW + q] += UbB[v];
        }
      }
      __syncthreads();
    }
  }

  // gather per node
  const int G = a.diff ? 5 : 4;
  if constexpr (DIR == 0) {
    // The line mapping is recomputed here rather than kept from the load
    // phase: held in scalar registers through the VJP phases it would be
    // spilled (the empty asm hides that the slot is the same, so the two
    // computations are not merged).
    int64_t i0r = i0;
    asm volatile("" : "+s"(i0r));
    bt = line_tile(i0r, N, g.lines, P, TL, g.inv_line);
    near = bt.p1 <= bt.p0 + 1;
  }
#pragma unroll 1
  for (int q = tid; q < TL * W; q += NT) {
    const int t = q >> LW, c = q & (W - 1);
    int64_t i = i0 + t;
    if constexpr (DIR == 0) {
      const BatchSlot sl = near ? batch_slot_near(bt, t) : line_slot(i, N, g.lines, P, g.inv_line);
      if (sl.j < 0 || sl.j >= sl.n) continue;  // a ghost slot
      base = sl.o;
      i = sl.j;
    } else {
      if (i >= N || c >= ncol) continue;
    }
    const int k = t + 5;  // LDS node index of node i
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    // contributions at LDS position kk: midpoints kk - j, j = 0..5, inside the tile
    auto add_position = [&](int kk) {
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const int tm = kk - j;
        if (tm >= 0 && tm < TM) {
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] += sWB[(j * NV + v) * TMW + tm * W + c];
        }
      }
    };
    add_position(k);
    if (a.bc != 0) {
      if (i == 0)
        for (int gg = 1; gg <= G; ++gg) add_position(k - gg);
      if (i == N - 1)
        for (int gg = 1; gg <= G; ++gg) add_position(k + gg);
    }
    if (a.diff == 0) {
      // node flux F_i enters D_{i+1} with -3/10 and D_{i-1} with +3/10;
      // Rbar of nodes i - 1 .. i + 1 from the tile's copy (sRB: the line's
      // ghosts applied, zero beyond a transmissive end)
      double Fb[NV], U[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double* Rb = sRB + v * SV + k * W + c;  // Rbar of node i
        double f = -0.3 * a.ih * (Rb[W] - Rb[-W]);
        if (a.bc != 0) {
          if (i == 0)  // ghost node -1 carries U_0
            f += -0.3 * a.ih * Rb[0];
          if (i == N - 1)  // ghost node N carries U_{N-1}
            f += 0.3 * a.ih * Rb[0];
        }
        Fb[v] = f;
        U[v] = sU[v * SV + k * W + c];
      }
      node_flux_vjp<NV, DIR>(a.pp, U, Fb, acc);
    }
    const int64_t gidx = base + i * stride + c;
    const double sc = a.dt ? a.scale * *a.dt : a.scale;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t e = v * a.npts + gidx;
      double y;
      if (a.A) {
        y = a.ca * a.A[e];
        if (a.B) y = __builtin_fma(a.cb, a.B[e], y);
        if (a.C) y = __builtin_fma(a.cc, a.C[e], y);
      } else {
        y = a.Ubar[e];
      }
      a.Ubar[e] = __builtin_fma(sc, acc[v], y);
    }
  }
}

// --------------------------------------------------------------- launchers --
static inline int64_t ceil_div64(int64_t x, int64_t y) { return (x + y - 1) / y; }

// Tile shape per variable count: 128 midpoints per tile for the scalar
// equation and the 1D Euler system, 64 for the 2D and 3D Euler systems (LDS
// per tile 33 KB and 41 KB: four and three tiles per CU; the 2D residual
// adjoint at 1024^2 measured faster with 64 than with 128).  y and z tiles are two columns
// wide: a taller tile recomputes fewer overlap rows (5 of 64 instead of 5
// of 32 with four columns), and the XCD-aware order keeps the column pairs
// that share a cache line on one L2 (2D 1024^2 residual adjoint: 2 % faster
// than four columns, 1 % faster than one).
#ifndef WCNS_ADJ_YZ_W
#define WCNS_ADJ_YZ_W 2
#endif
#ifndef WCNS_ADJ_TMW4
#define WCNS_ADJ_TMW4 64
#endif
template <int NV, int DIR>
struct AdjShape {
  static constexpr int TMW = NV == 5 ? 64 : (NV == 4 ? WCNS_ADJ_TMW4 : 128);
  static constexpr int W = DIR == 0 ? 1 : WCNS_ADJ_YZ_W;
  static constexpr int TM = TMW / W;
};

template <int NV, int DIR>
static hipError_t adj_go(const AdjArgs& a, hipStream_t s) {
  constexpr int TM = AdjShape<NV, DIR>::TM, W = AdjShape<NV, DIR>::W;
  using L = AdjLayout<NV, TM, W>;
  static_assert(L::lds_doubles * sizeof(double) <= 160 * 1024, "adjoint tile exceeds 160 KB of LDS");
  TileGeom g{};
  g.tm = TM;
  g.w = W;
  g.lw = L::LW;
  g.ltmw = L::LTMW;
  g.tl = TM - 5;
  g.segs = ceil_div64(a.n[DIR], g.tl);
  g.xgroups = DIR == 0 ? 1 : ceil_div64(a.n[0], W);
  // (both below 2^31 whenever the tile count is, which the launch checks)
  g.dxg = fast_div((uint32_t)g.xgroups);
  g.dseg = fast_div((uint32_t)g.segs);
  const int64_t others = DIR == 0 ? a.n[1] * a.n[2] : (DIR == 1 ? a.n[2] : a.n[1]);
  g.ntiles = g.segs * g.xgroups * others;
  g.lines = 0;
  g.inv_line = 0.0;
  if (DIR == 0) {  // packed x-lines, 5 ghost slots per side
    const int64_t L = a.n[0] + 10;
    g.lines = others;
    g.inv_line = 1.0 / (double)L;
    g.ntiles = ceil_div64(others * L, g.tl);
  }
  if (g.ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  const size_t lds = sizeof(double) * L::lds_doubles;
  if (spec_of(a.ip) == SPEC_FE)
    hipLaunchKernelGGL((adj_sweep_kernel<NV, DIR, SPEC_FE, TM, W>), dim3((unsigned)g.ntiles),
                       dim3(256), lds, s, a, g);
  else
    hipLaunchKernelGGL((adj_sweep_kernel<NV, DIR, SPEC_GENERIC, TM, W>), dim3((unsigned)g.ntiles),
                       dim3(256), lds, s, a, g);
  return hipGetLastError();
}

hipError_t launch_adjoint_dir(int nv, int dir, const AdjArgs& a, hipStream_t stream) {
#define WCNS_A(NVV, DD) \
  if (nv == NVV && dir == DD) return adj_go<NVV, DD>(a, stream);
  WCNS_A(1, 0) WCNS_A(1, 1) WCNS_A(1, 2)
  WCNS_A(3, 0)
  WCNS_A(4, 0) WCNS_A(4, 1)
  WCNS_A(5, 0) WCNS_A(5, 1) WCNS_A(5, 2)
#undef WCNS_A
  return hipErrorInvalidValue;
}

}  // namespace wcns
