// Directional sweep of the WCNS-FE residual on gfx950 (all directions and
// the ragged batch).
//
// A workgroup of 256 lanes owns one tile: TM midpoints along the sweep
// direction by W adjacent x-columns (W = 1 for the x direction; for y and z
// the columns make the global loads coalesced rows).  TM*W is 128 or 256 and
// both are compile-time, so every LDS address is a lane base plus an
// immediate offset.  Phases, with every lane looping over the phase's tasks
// (no wavefront idles through a short phase):
//   load    the TM+5 nodes of every column into LDS, ghosts applied (all
//           global reads issued before the first LDS write);
//   roe     Roe average of the two nodes around each midpoint;
//   interp  one task = one field of one midpoint: its six stencil values
//           projected on the fly from the LDS nodes, then the left-biased
//           and the mirrored right-biased nonlinear interpolation
//           (interp5_pair).  TM*W is a multiple of 64, so the field is
//           uniform across a wavefront;
//   flux    back-projection of the two interpolated states and the local
//           Lax-Friedrichs flux;
//   diff    MND6 or MD6 flux difference of TL = TM-3 (TM-5) nodes per
//           column, written as R, R+= or the fused SSP-RK3 stage combine.
// The ragged batch packs its tiles across problem ends (BatchArgs): a tile's
// slots may belong to two or more problems, each slot mapped to its problem,
// node or ghost in the load phase.
// Barriers separate load | roe | interp | flux | diff; with TM*W = 256 every
// lane owns one midpoint column through roe, interp and flux, and only
// load | roe and flux | diff are synchronised.
// LDS (doubles): sU[NV][TM+5][W] | sR[NR][TM*W] | sW[2 NV][TM*W] | the
// 64-entry exp table; the flux overwrites sW rows 0..NV-1 (each task reads
// its midpoint's two states before writing that midpoint's flux), and with
// MND6 rows NV..2NV-1 with the physical flux of node m + 2.  On the
// register path (sweep_reg: 4 and 5 variables, TM*W = 256) each lane keeps
// its midpoint's Roe state in registers and sR is left out.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "wcns_internal.hpp"
#include "wcns_sweep_common.hpp"

namespace wcns {

#ifndef WCNS_REG_MIN_NV  // fewest variables of a register-path tile
#define WCNS_REG_MIN_NV 4
#endif

// With TM W = 256 every lane owns one midpoint column through the Roe,
// interpolation and flux phases.  From WCNS_REG_MIN_NV variables on, that
// lane keeps its Roe state in registers instead of LDS: the 5-variable tile
// then needs 31 KB of LDS instead of 43 KB (five workgroups per CU instead of
// three), the 4-variable one 25 KB instead of 35 KB.
constexpr bool sweep_reg(int nv, int tmw) { return tmw == 256 && nv > 1 && nv >= WCNS_REG_MIN_NV; }

// LDS doubles of a tile: nodes sU[NV][TM+5][W] | Roe states sR[NR][TM W]
// (none on the register path) | interpolated states sW[2 NV][TM W] | the
// 64-entry exp table.
constexpr size_t sweep_lds_doubles(int nv, int tm, int w) {
  const size_t nr = (nv > 1 && !sweep_reg(nv, tm * w)) ? (size_t)nv + 1 : 0;
  return (size_t)nv * (tm + 5) * w + (nr + 2 * (size_t)nv) * ((size_t)tm * w) + 64;
}

template <int NV, int TM, int W>
struct SweepLayout {
  static constexpr int ND = NV > 1 ? NV - 2 : 1;
  static constexpr bool REG = sweep_reg(NV, TM * W);
  static constexpr int NR = (NV > 1 && !REG) ? NV - 2 + 3 : 0;  // vel[ND], H, c, ic
  static constexpr int TN = TM + 5;                    // nodes per column
  static constexpr int TMW = TM * W;                   // midpoints per tile
  static constexpr int SV = TN * W;                    // LDS stride between variables
  static constexpr int LW = W == 1 ? 0 : W == 2 ? 1 : W == 4 ? 2 : W == 8 ? 3 : 4;
  static constexpr int LTMW = TMW == 128 ? 7 : 8;
  static constexpr size_t lds_doubles = sweep_lds_doubles(NV, TM, W);
  static_assert(lds_doubles == (size_t)NV * SV + (size_t)(NR + 2 * NV) * TMW + 64, "LDS layout");
  static_assert(TMW == 128 || TMW == 256, "tile must hold 128 or 256 midpoints");
  static_assert((1 << LW) == W, "W must be a power of two up to 16");
};

// The sweep kernel's arguments, one struct so that its layout in the kernel
// argument segment is the struct's.
struct SweepKernArgs {
  SweepArgs a;
  BatchArgs b;
  TileGeom g;
  int mode;
};
using SweepKernArgsPtr = const __attribute__((address_space(4))) SweepKernArgs*;

// The kernel's arguments for a late phase.  Values held in scalar registers
// from the kernel's start through the interpolation spill to VGPR lanes
// (every reload a VALU instruction per lane) once the FE constants fill the
// scalar file; the empty asm hides that the segment does not change, so the
// late phase reads what it needs with scalar loads at that point instead.
__device__ __forceinline__ SweepKernArgsPtr sweep_kernargs_late() {
  unsigned long long p = reinterpret_cast<unsigned long long>(__builtin_amdgcn_kernarg_segment_ptr());
  asm volatile("" : "+s"(p));
  return reinterpret_cast<SweepKernArgsPtr>(p);
}

// One tile (logical index `tile`) of a sweep; every lane of the workgroup
// calls it from sweep_kernel (its late phases re-read the kernel arguments).
template <int NV, int DIR, bool BATCH, int SPEC, int TM, int W>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, const BatchArgs& b,
                                           const TileGeom& g, int mode, int64_t tile,
                                           double* smem) {
  using L = SweepLayout<NV, TM, W>;
  constexpr int ND = L::ND, NR = L::NR, TN = L::TN, TMW = L::TMW, SV = L::SV;
  constexpr int LW = L::LW, LTMW = L::LTMW;
  constexpr bool REG = L::REG;
  constexpr int NT = 256;
  double* sU = smem;
  double* sR = sU + NV * SV;
  double* sW = sR + NR * TMW;
  double* sX = sW + 2 * NV * TMW;  // kExp2Tab64
  const int tid = threadIdx.x;
  const int G = a.diff ? 5 : 4;
  const int TL = TM - (a.diff ? 5 : 3);

  int64_t base = 0, N = 0, stride = 1, i0;
  int ncol = 1;
  double ih = a.ih, dt = 0.0;
  // Along x (and in the batch) the lines are packed end to end: i0 is a slot
  // of the packed index space (BatchArgs, TileGeom::lines).
  constexpr bool LINES = BATCH || DIR == 0;
  BatchTile bt{};
  bool near = true;  // the tile spans at most two lines or problems
  if constexpr (BATCH) {
    i0 = tile * TL;
    bt = batch_tile(b, tile, i0, G);
    near = bt.p1 <= bt.p0 + 1;
    if (mode == MODE_STAGE) {
      bool live = false;  // uniform across the block
      for (int p = bt.p0; p <= bt.p1; ++p) live |= (b.dtp[p] != 0.0);
      if (!live) return;  // every problem of the tile has finished
    }
  } else if constexpr (DIR == 0) {
    i0 = tile * TL;
    N = a.n[0];
    bt = line_tile(i0, N, g.lines, G, TL, g.inv_line);
    near = bt.p1 <= bt.p0 + 1;
    if (mode >= MODE_STAGE) dt = *a.dt;
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
    if (mode >= MODE_STAGE) dt = *a.dt;
  }
  const int64_t nb = i0 - G;

  // load: every global read of the tile (at most two nodes per lane, and the
  // exp table) is issued before the first LDS write, so their latencies
  // overlap
  constexpr int NIT = (SV + NT - 1) / NT;
  static_assert(NIT <= 2, "a tile holds at most two nodes per lane");
  double buf[NIT][NV];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = tid + it * NT;
    if (idx < SV) {
      const int k = idx >> LW, c = idx & (W - 1);
      const int cc = c < ncol ? c : ncol - 1;
      int64_t gi;
      if constexpr (LINES) {
        BatchSlot sl;
        if (near)
          sl = batch_slot_near(bt, k - G);
        else if constexpr (BATCH)
          sl = batch_slot(b, bt.p0, bt.p1, G, nb + k);
        else
          sl = line_slot(nb + k, N, g.lines, G, g.inv_line);
        // slots outside every problem's range (before the first, after the
        // last) load a ghost; no output node uses them
        const int j = sl.j < -G ? -G : (sl.j >= sl.n + G ? sl.n + G - 1 : sl.j);
        gi = sl.o + bc_index_near(j, sl.n, a.bc);
      } else {
        gi = base + bc_index(nb + k, N, a.bc) * stride + cc;
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) buf[it][v] = a.U[v * a.npts + gi];
    }
  }
  // the lane's output node in a tile of packed lines (-1: none, or a ghost
  // slot)
  int64_t onode = -1;
  int oprob = 0;
  if constexpr (LINES) {
    static_assert(W == 1 && TM <= NT, "one output node per lane");
    if (tid < TL) {
      BatchSlot sl;
      if (near)
        sl = batch_slot_near(bt, tid);
      else if constexpr (BATCH)
        sl = batch_slot(b, bt.p0, bt.p1, G, i0 + tid);
      else
        sl = line_slot(i0 + tid, N, g.lines, G, g.inv_line);
      if (sl.j >= 0 && sl.j < sl.n) {
        onode = sl.o + sl.j;
        oprob = sl.p;
      }
    }
  }
  double xv = 0.0;
  if constexpr (SPEC == SPEC_FE) {
    if (tid < 64) xv = kExp2Tab64[tid];
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = tid + it * NT;
    if (idx < SV) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sU[v * SV + idx] = buf[it][v];
    }
  }
  if constexpr (SPEC == SPEC_FE) {
    if (tid < 64) sX[tid] = xv;
  }
  __syncthreads();

  // With one midpoint column per lane (TM W = 256), lane q computes the Roe
  // state, all interpolations and the flux of midpoint column q itself, so
  // the Roe, interpolation and flux phases need no barrier between them.
  constexpr bool OWN = (TMW == NT);
  const bool proj = (NV > 1) && a.pp.charproj;
  RoeState<ND> rsq{};  // the register path: Roe state of the lane's midpoint column
  if constexpr (REG) {
    if (proj) {
      const double* u = sU + tid + 2 * W;
      double UA[NV], UB[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UA[v] = u[v * SV];
        UB[v] = u[v * SV + W];
      }
      rsq = roe_average<ND>(UA, UB, a.pp.gamma);
    }
  } else if constexpr (NV > 1) {
    if (proj) {
#pragma unroll 1
      for (int q = tid; q < TMW; q += NT) {
        // node m+2 of column c sits at LDS index q + 2W (q = m W + c)
        const double* u = sU + q + 2 * W;
        double UA[NV], UB[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          UA[v] = u[v * SV];
          UB[v] = u[v * SV + W];
        }
        const RoeState<ND> rs = roe_average<ND>(UA, UB, a.pp.gamma);
        double* r = sR + q;
#pragma unroll
        for (int k = 0; k < ND; ++k) r[k * TMW] = rs.vel[k];
        r[(ND + 0) * TMW] = rs.H;
        r[(ND + 1) * TMW] = rs.c;
        r[(ND + 2) * TMW] = rs.ic;
      }
      if constexpr (!OWN) __syncthreads();
    }
  }

  // one field of one midpoint per task: its left- and right-biased
  // interpolations share the six projected stencil values
#pragma unroll 1
  for (int q = tid; q < NV * TMW; q += NT) {
    const int v = q >> LTMW;
    const int rem = q & (TMW - 1);  // = m W + c
    const double* u = sU + rem;     // node m of column c; node m + j at u[j W]
    double w[6];
    if (proj) {
      if constexpr (NV > 1) {
        const double* r = sR + rem;
        if (v >= 2 && v < NV - 1) {  // shear field: m_ax - vel_ax rho
          const int ax = tangential_axis<ND, DIR>(v - 2);
          double va;
          if constexpr (REG) {
            va = rsq.vel[0];
#pragma unroll
            for (int k = 1; k < ND; ++k) va = (ax == k) ? rsq.vel[k] : va;
          } else {
            va = r[ax * TMW];
          }
          const double* um = u + (1 + ax) * SV;
#pragma unroll
          for (int j = 0; j < 6; ++j) w[j] = __builtin_fma(-va, u[j * W], um[j * W]);
        } else {
          RoeState<ND> rs;
          if constexpr (REG) {
            // recomputed per field from vel and ic, which are all the loop
            // keeps of the Roe state besides H and c (the empty asm hides
            // that they are loop-invariant)
#pragma unroll
            for (int k = 0; k < ND; ++k) {
              rs.vel[k] = rsq.vel[k];
              asm volatile("" : "+v"(rs.vel[k]));
            }
            rs.ic = rsq.ic;
            asm volatile("" : "+v"(rs.ic));
          } else {
#pragma unroll
            for (int k = 0; k < ND; ++k) rs.vel[k] = r[k * TMW];
            rs.ic = r[(ND + 2) * TMW];
          }
          roe_derived<ND>(rs, a.pp.gamma);
          double l[NV];
          field_row<ND, DIR>(rs, v, l);
          project_stencil<NV, SV, W>(u, l, w);
        }
      }
    } else {
      const double* uv = u + v * SV;
#pragma unroll
      for (int j = 0; j < 6; ++j) w[j] = uv[j * W];
    }
    interp5_pair<SPEC, SPEC == SPEC_FE>(a.ip, w, sW + q, sW + NV * TMW + q, sX);
  }
  if constexpr (!OWN) __syncthreads();

  // A batch tile has at most one output node per lane (TL < 256): the lane
  // locates it during the load phase and reads its problem's 1/h and dt
  // here, so that these reads overlap the flux phase rather than the
  // epilogue.
  double oih = 0.0, odt = 0.0;
  if constexpr (BATCH) {
    if (onode >= 0) {
      const SweepKernArgsPtr k = sweep_kernargs_late();
      oih = k->b.ih[oprob];
      if (mode == MODE_STAGE) odt = k->b.dtp[oprob];
    }
  }

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
        RoeState<ND> rs = rsq;
        if constexpr (!REG) {
          const double* r = sR + q;
#pragma unroll
          for (int k = 0; k < ND; ++k) rs.vel[k] = r[k * TMW];
          rs.H = r[(ND + 0) * TMW];
          rs.c = r[(ND + 1) * TMW];
          rs.ic = r[(ND + 2) * TMW];
          roe_derived<ND>(rs, a.pp.gamma);
        }
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
    if (a.diff == 0) {
      // the physical flux of node m + 2 (q = m W + c) for the MND6
      // difference, into the right-state rows this lane has just read: each
      // node's flux is computed once instead of by both its neighbours
      double Uc[NV], Fc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Uc[v] = sU[v * SV + q + 2 * W];
      node_flux<NV, DIR>(a.pp, Uc, Fc);
#pragma unroll
      for (int v = 0; v < NV; ++v) sW[(NV + v) * TMW + q] = Fc[v];
    }
  }
  __syncthreads();

  // flux difference and output
  EmitArgs ea = emit_args(sweep_kernargs_late()->a);
  // a batch stage has no residual of earlier sweeps (one direction):
  // known here, its reads and selects drop out of the epilogue
  if constexpr (BATCH) ea.Rin = nullptr;
  unsigned long long rbits = 0;  // wave rate of the lane's written node (SweepArgs::wmax)
#pragma unroll 1
  for (int q = tid; q < TL * W; q += NT) {
    const int t = q >> LW, c = q & (W - 1);
    int64_t i = i0 + t;
    if constexpr (LINES) {
      // q == tid here (one output node per lane)
      if (onode < 0) continue;  // a ghost slot
      if constexpr (BATCH) {
        dt = odt;
        if (mode == MODE_STAGE && dt == 0.0) continue;  // finished problem
        ih = oih;
      }
      base = onode;
      i = 0;
    } else {
      if (i >= N || c >= ncol) continue;
    }
    const double* f = sW + q;        // F~ of midpoint t + k of column c at f[k W]
    const double* u = sU + q;        // node t + k of column c at u[k W]
    double res[NV], Un[NV];
    if (a.diff == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Un[v] = u[v * SV + 4 * W];
        const lds_cptr fv = lds_row(f + v * TMW);
        // F of node t + k + 2 at nf[k W]: nodes t + 3 and t + 5 around t + 4
        const lds_cptr nf = lds_row(f + (NV + v) * TMW);
        const double d = 1.5 * (fv[2 * W] - fv[W]) - 0.3 * (nf[3 * W] - nf[W]) +
                         (1.0 / 30.0) * (fv[3 * W] - fv[0]);
        res[v] = -ih * d;
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Un[v] = u[v * SV + 5 * W];
        const lds_cptr fv = lds_row(f + v * TMW);
        const double d = (75.0 / 64.0) * (fv[3 * W] - fv[2 * W]) +
                         (-25.0 / 384.0) * (fv[4 * W] - fv[W]) + (3.0 / 640.0) * (fv[5 * W] - fv[0]);
        res[v] = -ih * d;
      }
    }
    if constexpr (BATCH) {
      double y[NV];
      emit_rt<NV>(mode, ea, base + i * stride + c, a.npts, res, Un, dt, y);
      if (a.wmax && mode == MODE_STAGE) {
        const double ihv[1] = {ih};
        rbits = __builtin_bit_cast(unsigned long long, wave_rate<1>(y, a.pp.gamma, ihv));
      }
    } else {
      emit_rt<NV>(mode, ea, base + i * stride + c, a.npts, res, Un, dt);
    }
  }
  // The batch's last stage of a step also takes each problem's maximum wave
  // rate of the state it writes (uniform branch; every lane reaches it).
  if constexpr (BATCH) {
    if (a.wmax && mode == MODE_STAGE) {
      if (near) {
        // The lanes' nodes belong to p0 or p0 + 1, in order, so at most one
        // wavefront of the tile holds both: reduce only for the problems a
        // wavefront holds (the ballots are uniform across it).
        const bool s1 = oprob != bt.p0;
        if (__ballot(rbits != 0 && !s1)) {
          const unsigned long long m0 = wave_max_bits(s1 ? 0ull : rbits);
          if ((tid & 63) == 0) atomicMax(a.wmax + bt.p0, m0);
        }
        if (__ballot(rbits != 0 && s1)) {
          const unsigned long long m1 = wave_max_bits(s1 ? rbits : 0ull);
          if ((tid & 63) == 0) atomicMax(a.wmax + bt.p0 + 1, m1);
        }
      } else if (rbits) {
        atomicMax(a.wmax + oprob, rbits);
      }
    }
  }
}

// The FE specialisation runs at six waves per SIMD: the compiler keeps it
// within 80 VGPRs without spilling, and the largest tile (NV = 3, 256
// midpoints, 27.3 KB of LDS) still fits six workgroups in a CU's 160 KB.
// The register path runs at five (at most 102 VGPRs; 86-90 used, no spills):
// at six its Roe state spills, and LDS allows five 5-variable tiles per CU
// (four for the 32 x 8 tile) against three before.
// The generic interpolation needs ~110 VGPRs and is left unconstrained
// (capped at 80 it spills); the saturating FE one (SPEC_FE_SAT) needs ~118
// and runs at four.
// The sweep kernel: one tile per workgroup, in XCD-aware order.  A batch
// launch with a live list (BatchArgs::live) maps workgroup b to list
// position xcd_tile(b, nlive) (each XCD a contiguous range of the list, so
// neighbouring tiles, which share halo lines, run on one L2 at about the same
// time) and workgroups b >= nlive leave after reading the count: the list is
// read on the device, so the host launches the same grid whatever the number
// of live tiles.
#ifndef WCNS_REG_WAVES
#define WCNS_REG_WAVES 5
#endif
constexpr int sweep_waves(int nv, int tmw, int spec) {
  return spec == SPEC_GENERIC ? 1
         : spec != SPEC_FE    ? 4
         : sweep_reg(nv, tmw) ? WCNS_REG_WAVES
                              : 6;
}

template <int NV, int DIR, bool BATCH, int SPEC, int TM, int W>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(sweep_waves(NV, TM * W, SPEC))))
    sweep_kernel(SweepKernArgs k) {
  extern __shared__ double smem[];
  const SweepArgs& a = k.a;
  const BatchArgs& b = k.b;
  const TileGeom& g = k.g;
  const int mode = k.mode;
  int64_t tile;
  if (BATCH && b.live) {
    const int n = *b.nlive;
    // a launch capped below the list's length leaves tiles out: say so
    if (n > (int)gridDim.x && blockIdx.x == 0 && threadIdx.x == 0 && a.status)
      atomicOr(a.status, 2);
    if ((int)blockIdx.x >= n) return;
    tile = b.live[xcd_tile(blockIdx.x, n)];
  } else {
    if ((int64_t)blockIdx.x >= g.ntiles) return;
    tile = xcd_tile(blockIdx.x, g.ntiles);
  }
  sweep_tile<NV, DIR, BATCH, SPEC, TM, W>(a, b, g, mode, tile, smem);
}

// --------------------------------------------------------------- launchers --
static inline int64_t ceil_div64(int64_t x, int64_t y) { return (x + y - 1) / y; }

// Compiled tile shapes: x direction and batch tm in {128, 256}; y/z (tm, w)
// in {(16, 8), (32, 4), (32, 8), (64, 4), (128, 2), (256, 1)}.
bool sweep_shape_ok(int nv, int dir, int tm, int w) {
  if (dir == 0) return w == 1 && (tm == 128 || tm == 256);
  const bool known = (tm == 16 && w == 8) || (tm == 32 && w == 4) || (tm == 32 && w == 8) ||
                     (tm == 64 && w == 4) || (tm == 128 && w == 2) || (tm == 256 && w == 1);
  if (!known) return false;
  return sizeof(double) * sweep_lds_doubles(nv, tm, w) <= 64 * 1024;
}

template <int NV, int DIR, bool BATCH, int SPEC, int TM, int W>
static hipError_t sweep_launch(const SweepArgs& a, const BatchArgs& b, const TileGeom& g,
                               int mode, size_t lds, hipStream_t s) {
  const SweepKernArgs k{a, b, g, mode};
  hipLaunchKernelGGL((sweep_kernel<NV, DIR, BATCH, SPEC, TM, W>),
                     dim3((unsigned)(g.grid > 0 ? g.grid : g.ntiles)), dim3(256), lds, s, k);
  return hipGetLastError();
}

template <int NV, int DIR, bool BATCH, int TM, int W>
static hipError_t sweep_go(const SweepArgs& a, const BatchArgs& b, const TileGeom& g, int mode,
                           hipStream_t s) {
  const size_t lds = sizeof(double) * SweepLayout<NV, TM, W>::lds_doubles;
  const int spec = spec_of(a.ip);
  if (spec == SPEC_FE) return sweep_launch<NV, DIR, BATCH, SPEC_FE, TM, W>(a, b, g, mode, lds, s);
  if (spec == SPEC_FE_SAT)
    return sweep_launch<NV, DIR, BATCH, SPEC_FE_SAT, TM, W>(a, b, g, mode, lds, s);
  return sweep_launch<NV, DIR, BATCH, SPEC_GENERIC, TM, W>(a, b, g, mode, lds, s);
}

template <int NV, int DIR, bool BATCH>
static hipError_t sweep_shape(const SweepArgs& a, const BatchArgs& b, const TileGeom& g, int mode,
                              hipStream_t s) {
  if constexpr (DIR == 0) {
    if (g.tm == 128) return sweep_go<NV, DIR, BATCH, 128, 1>(a, b, g, mode, s);
    return sweep_go<NV, DIR, BATCH, 256, 1>(a, b, g, mode, s);
  } else {
    if (g.tm == 16) return sweep_go<NV, DIR, BATCH, 16, 8>(a, b, g, mode, s);
    if (g.w == 4 && g.tm == 32) return sweep_go<NV, DIR, BATCH, 32, 4>(a, b, g, mode, s);
    if (g.tm == 32) return sweep_go<NV, DIR, BATCH, 32, 8>(a, b, g, mode, s);
    if (g.tm == 128) return sweep_go<NV, DIR, BATCH, 128, 2>(a, b, g, mode, s);
    if (g.tm == 256) return sweep_go<NV, DIR, BATCH, 256, 1>(a, b, g, mode, s);
    return sweep_go<NV, DIR, BATCH, 64, 4>(a, b, g, mode, s);
  }
}

static TileGeom make_geom(int dir, const int64_t n[3], int diff, int tm, int w) {
  TileGeom g{};
  g.tm = tm;
  g.w = w;
  g.lw = 0;
  g.ltmw = 0;
  g.tl = tm - (diff ? 5 : 3);
  g.segs = ceil_div64(n[dir], g.tl);
  g.xgroups = dir == 0 ? 1 : ceil_div64(n[0], w);
  // (both below 2^31 whenever the tile count is, which the launch checks)
  g.dxg = fast_div((uint32_t)g.xgroups);
  g.dseg = fast_div((uint32_t)g.segs);
  const int64_t others = dir == 0 ? n[1] * n[2] : (dir == 1 ? n[2] : n[1]);
  g.ntiles = g.segs * g.xgroups * others;
  g.lines = 0;
  g.inv_line = 0.0;
  g.grid = 0;
  if (dir == 0) {  // packed x-lines
    const int64_t L = n[0] + 2 * (diff ? 5 : 4);
    g.lines = others;
    g.inv_line = 1.0 / (double)L;
    g.ntiles = ceil_div64(others * L, g.tl);
  }
  return g;
}

hipError_t launch_sweep(int nv, int dir, const SweepArgs& a, int mode, int tm, int w,
                        hipStream_t stream) {
  if (!sweep_shape_ok(nv, dir, tm, w)) return hipErrorInvalidConfiguration;
  const TileGeom g = make_geom(dir, a.n, a.diff, tm, w);
  if (g.ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  BatchArgs b{};
#define WCNS_S(NVV, DD) \
  if (nv == NVV && dir == DD) return sweep_shape<NVV, DD, false>(a, b, g, mode, stream);
  WCNS_S(1, 0) WCNS_S(1, 1) WCNS_S(1, 2)
  WCNS_S(3, 0)
  WCNS_S(4, 0) WCNS_S(4, 1)
  WCNS_S(5, 0) WCNS_S(5, 1) WCNS_S(5, 2)
#undef WCNS_S
  return hipErrorInvalidValue;
}

hipError_t launch_batch_sweep(const SweepArgs& a, const BatchArgs& b, int mode, int tm,
                              hipStream_t stream, int32_t cap) {
  if (!sweep_shape_ok(3, 0, tm, 1)) return hipErrorInvalidConfiguration;
  TileGeom g{};
  g.tm = tm;
  g.w = 1;
  g.lw = 0;
  g.ltmw = 0;
  g.tl = tm - (a.diff ? 5 : 3);
  g.segs = 1;
  g.xgroups = 1;
  g.ntiles = b.ntiles;
  g.lines = 0;
  g.inv_line = 0.0;
  g.grid = (cap > 0 && b.live && cap < b.ntiles) ? cap : 0;
  return sweep_shape<3, 0, true>(a, b, g, mode, stream);
}

}  // namespace wcns
