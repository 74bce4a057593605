// Internal (non-ABI) declarations shared by the kernel and API translation
// units of the WCNS-FE library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcns_device.hpp"

namespace wcns {

// MODE_RES: out = R; MODE_ACC: out = Rin + R; MODE_STAGE: out = ca*U0 +
// cb*(U + dt*R); MODE_LIN: out = ca*U0 + cb*U + cr*dt*R (R includes Rin).
enum SweepMode : int { MODE_RES = 0, MODE_ACC = 1, MODE_STAGE = 2, MODE_LIN = 3 };

// Which compiled specialisation of the interpolation serves these parameters.
inline int spec_of(const InterpParams& ip) {
  if (ip.weights != WFE || ip.zpow != 2) return SPEC_GENERIC;
  return ip.fast_fe ? SPEC_FE : (ip.shared_exp ? SPEC_GENERIC : SPEC_FE_SAT);
}

// Arguments of one directional sweep.
struct SweepArgs {
  const double* U;      // state under the stencil, U^(k)
  const double* U0;     // U^n (stage mode, ca != 0)
  const double* Rin;    // residual of earlier sweeps (acc/stage), may be null
  double* out;          // R (res/acc) or U^(k+1) (stage)
  const double* dt;     // device dt (stage mode, non-batch)
  int32_t* status;      // OR-ed bit 0 on a non-physical stage result (may be null)
  double ca, cb;        // stage: out = ca*U0 + cb*(U + dt*R)
  double cr;            // linear stage: out = ca*U0 + cb*U + cr*dt*R
  int64_t npts;         // stride between variables
  int64_t n[3];         // grid extents (x, y, z)
  int32_t bc;           // boundary type along the sweep direction
  int32_t diff;         // 0 = MND6, 1 = MD6
  double ih;            // 1/h along the sweep direction
  InterpParams ip;
  PhysParams pp;
  // batch stage only, may be null: per-problem maxima (bit patterns) of the
  // wave rate of the written state, for the next step's dt
  unsigned long long* wmax;
};

// Ragged batch description (device arrays).
// Batch tiles are packed: problem p occupies the slots [s_p, s_p + N_p + 2G)
// of a virtual index space, s_p = offset[p] + 2 G p (G ghost slots on each
// side of its nodes), and tile k outputs the slots [k TL, k TL + TL), so a
// tile may span the end of one problem and the start of the next.
// Stage launches may walk a list of live tiles instead of every tile: a
// persistent grid (resident workgroups only) takes the list positions, each
// XCD a contiguous range of them.
struct BatchArgs {
  const int64_t* offset;   // nprob+1 column offsets
  const double* ih;        // 1/h per problem
  double* dtp;             // per-problem dt of the current step (0 = inactive)
  const int32_t* tile_p0;  // first and last problem that the slots a tile
  const int32_t* tile_p1;  //   loads (outputs and halo) touch
  const int32_t* live;     // live tiles in increasing order by runs (null: all tiles)
  const int32_t* nlive;    // length of the live list (device)
  int32_t ntiles;
  int32_t nprob;
};

// Geometry of a sweep's tiles: tm midpoints along the sweep direction by w
// adjacent x-columns (w = 1 along x); tm*w is 128 or 256 (powers of two).
// Division of a tile index n < 2^31 by a divisor 1 <= d < 2^31 fixed for a
// launch, by a multiply and a shift (Granlund and Montgomery, PLDI 1994):
// with l = ceil(log2 d) and m = ceil(2^(31+l) / d) < 2^32, m d = 2^(31+l) + e
// with 0 <= e < d <= 2^l, so n m / 2^(31+l) exceeds n/d by less than 1/d
// and its floor is floor(n/d).  On the device this is a few scalar
// instructions where a 64-bit division is a long branchy sequence.
struct FastDiv {
  uint32_t m;
  int32_t sh;  // 31 + l
  __host__ __device__ uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)n * m) >> sh);
  }
};
inline FastDiv fast_div(uint32_t d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t num = 1ull << (31 + l);
  return FastDiv{(uint32_t)((num + d - 1) / d), 31 + l};
}

struct TileGeom {
  int tm, w, lw, ltmw;   // lw = log2 w, ltmw = log2 (tm w)
  int tl;                // nodes per tile and column: tm - 3 (MND6) or tm - 5 (MD6)
  int64_t segs;          // tiles along one line
  int64_t xgroups;       // column groups across x (1 along x)
  int64_t ntiles;
  // x sweep of the sweep kernel: the x-lines packed end to end like a batch
  // of equal problems (line r at slots [r L, (r+1) L), L = n[0] + 2G)
  int64_t lines;
  double inv_line;       // 1 / L
  int64_t grid;          // workgroups launched (0: ntiles)
  FastDiv dxg, dseg;     // division by xgroups and by segs (y and z sweeps)
};

// Launchers.  All enqueue on `stream` and return the hipError_t of the launch
// (hipErrorInvalidConfiguration for a tile shape that sweep_shape_ok rejects).
bool sweep_shape_ok(int nv, int dir, int tm, int w);
hipError_t launch_sweep(int nv, int dir, const SweepArgs& a, int mode, int tm, int w,
                        hipStream_t stream);
// cap > 0 (with a live list in b): launch min(cap, b.ntiles) workgroups,
// the caller's bound on the list's length (see wcns_batch_rk3_steps_capped).
hipError_t launch_batch_sweep(const SweepArgs& a, const BatchArgs& b, int mode, int tm,
                              hipStream_t stream, int32_t cap = 0);
hipError_t launch_cfl(int nv, int ndim, const double* U, int64_t npts, double gamma,
                      const double* ih, const double* adv, double cfl, double* partial,
                      int nblocks, double* dt_out, hipStream_t stream);
// The per-problem dt kernels.  A problem whose maximum wave rate is not a
// positive finite number gets dt = 0, keeps its time and sets bit 0 of
// *status (when given).  nlive, when given, is cleared for a rebuild of the
// live list (launch_batch_live) after the kernel.
hipError_t launch_batch_cfl(const double* U, int64_t total, const BatchArgs& b, double gamma,
                            double* t, double t_end, double cfl, unsigned long long* wmax,
                            int32_t* status, int32_t* nlive, hipStream_t stream);
hipError_t launch_batch_dt(const BatchArgs& b, double* t, double t_end, double cfl,
                           unsigned long long* wmax, int32_t* status, int32_t* nlive,
                           hipStream_t stream);
// The live-tile list: every tile with a problem of dt > 0, appended to
// live[] in runs of consecutive tiles (nlive must be 0 before).
hipError_t launch_batch_live(const BatchArgs& b, int32_t* live, int32_t* nlive,
                             hipStream_t stream);
hipError_t launch_axpy_state(double* y, const double* x, double a, int64_t n,
                             hipStream_t stream);
hipError_t launch_lincomb(double* out, const double* x, double ax, const double* y, double ay,
                          const double* dt, double ydt, int64_t n, hipStream_t stream);
// The filtered embedded WENO sweep of App. B (wcns_weno.hip).
hipError_t launch_weno_sweep(int nv, int dir, const SweepArgs& a, int mode, hipStream_t stream);
// Weight histograms of one direction's interpolations (wcns_stats.hip).
hipError_t launch_weight_hist(int nv, int dir, const SweepArgs& a, unsigned long long* hist,
                              int nbins, hipStream_t stream);

// Adjoint launchers (wcns_adjoint.hip).
struct AdjArgs {
  const double* U;      // state
  const double* Rbar;   // cotangent of the residual
  double* Ubar;         // cotangent of U (output)
  // Ubar = ca A + cb B + cc C + s (dL/dU)^T Rbar when A is set (B and C
  // optional; any of them may be Ubar itself), else Ubar += s (dL/dU)^T Rbar;
  // s = scale * (*dt) when dt is set, else scale
  double scale;
  const double* dt;
  const double* A;
  const double* B;
  const double* C;
  double ca, cb, cc;
  int64_t npts;
  int64_t n[3];
  int32_t bc;
  int32_t diff;
  double ih;
  InterpParams ip;
  PhysParams pp;
};
hipError_t launch_adjoint_dir(int nv, int dir, const AdjArgs& a, hipStream_t stream);

int cfl_blocks(int64_t npts);

hipError_t launch_probe_fma(double* out, int blocks, int iters, hipStream_t stream);
hipError_t launch_probe_copy(const double* src, double* dst, int64_t n, hipStream_t stream);
hipError_t launch_probe_math(const double* x, double* out, int64_t n, int fn, hipStream_t stream);

}  // namespace wcns
