// Device helpers shared by the sweep kernels: boundary index map, tile and
// slot maps of packed lines, LDS row addresses and the stencil projection,
// status flag and the per-node epilogue (R, R+= or the fused SSP-RK3 stage
// combine).
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

// Logical tile of workgroup b among nt: workgroups are dealt to the 8 XCDs
// in turn (b % 8), each with its own L2, so XCD x is given the contiguous
// logical range [x q + min(x, r), ...) (q = nt / 8, r = nt % 8) in launch
// order.  Neighbouring logical tiles, which share cache lines (halos, and
// the 128-byte lines that adjacent column groups of a y or z sweep split),
// then run on the same XCD at about the same time.  A bijection of [0, nt).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nt) {
  const int64_t q = nt >> 3, r = nt & 7, x = b & 7, y = b >> 3;
  return x * q + (x < r ? x : r) + y;
}

// Slot v of a packed batch (BatchArgs) as problem p, its first node o in the
// state arrays, its length n and the node index j = v - s_p - G (negative or
// >= n for a ghost slot).  p0 .. p1 bound the problems the caller's slots
// can touch; slots outside all ranges come out with j < -G or j >= n + G.
struct BatchSlot {
  int64_t o;
  int n, j, p;
};
__device__ __forceinline__ BatchSlot batch_slot(const BatchArgs& b, int p0, int p1, int G,
                                                int64_t v) {
  int p = p0;
  int64_t o = b.offset[p], e = b.offset[p + 1];
  while (p < p1 && v >= e + 2 * (int64_t)G * (p + 1)) {
    ++p;
    o = e;
    e = b.offset[p + 1];
  }
  return BatchSlot{o, (int)(e - o), (int)(v - o - 2 * (int64_t)G * p - G), p};
}

// A tile of a packed batch, from uniform reads: its problems p0 .. p1 and,
// for the common case p1 <= p0 + 1, what maps a tile-relative slot r (slot
// i0 + r, r in [-G, TL + G)) to its problem in 32-bit arithmetic.
struct BatchTile {
  int p0, p1;
  int64_t o0, o1;  // first nodes of p0 and p0 + 1
  int n0, n1;      // their lengths
  int c0, c1;      // node index of slot i0 + r: r + c0 in p0, r + c1 in p0 + 1
  int r1;          // first relative slot of p0 + 1 (beyond every r if p1 == p0)
};
__device__ __forceinline__ BatchTile batch_tile(const BatchArgs& b, int64_t tile, int64_t i0,
                                                int G) {
  BatchTile t;
  t.p0 = b.tile_p0[tile];
  t.p1 = b.tile_p1[tile];
  t.o0 = b.offset[t.p0];
  t.o1 = b.offset[t.p0 + 1];
  t.n0 = (int)(t.o1 - t.o0);
  // slot i0 - G lies in p0's range (or before the first problem), so
  // c0 = i0 - s0 - G is in [-G, n0 + 2G)
  t.c0 = (int)(i0 - (t.o0 + 2 * (int64_t)G * t.p0) - G);
  if (t.p1 > t.p0) {
    const int64_t o2 = b.offset[t.p0 + 2];
    t.n1 = (int)(o2 - t.o1);
    // p0 + 1 starts within the tile's slots: r1 in (-G, TL + G]
    t.r1 = (int)(t.o1 + 2 * (int64_t)G * (t.p0 + 1) - i0);
    t.c1 = -t.r1 - G;
  } else {
    t.n1 = t.n0;
    t.r1 = 1 << 30;
    t.c1 = t.c0;
  }
  return t;
}
__device__ __forceinline__ BatchSlot batch_slot_near(const BatchTile& t, int r) {
  const bool s = r >= t.r1;
  return BatchSlot{s ? t.o1 : t.o0, s ? t.n1 : t.n0, r + (s ? t.c1 : t.c0), t.p0 + (int)s};
}

// The line holding slot v >= 0 of x-lines packed with L slots each (the
// quotient from the double reciprocal is off by at most one below 2^52).
__device__ __forceinline__ int64_t line_of(int64_t v, int64_t L, double invL) {
  int64_t q = (int64_t)((double)v * invL);
  if (q * L > v) --q;
  if ((q + 1) * L <= v) ++q;
  return q;
}
// Slot v of the packed x-lines (lines of N nodes) as a BatchSlot; slots
// before the first line or after the last come out with j < -G or j >= N + G.
__device__ __forceinline__ BatchSlot line_slot(int64_t v, int64_t N, int64_t lines, int G,
                                               double invL) {
  const int64_t L = N + 2 * G;
  int64_t p = v < 0 ? 0 : line_of(v, L, invL);
  if (p > lines - 1) p = lines - 1;
  return BatchSlot{p * N, (int)N, (int)(v - p * L - G), (int)p};
}
// The tile of packed x-lines whose output slots start at i0 (as batch_tile).
__device__ __forceinline__ BatchTile line_tile(int64_t i0, int64_t N, int64_t lines, int G,
                                               int TL, double invL) {
  const int64_t L = N + 2 * G;
  const BatchSlot a = line_slot(i0 - G, N, lines, G, invL);
  const BatchSlot e = line_slot(i0 + TL + G - 1, N, lines, G, invL);
  BatchTile t;
  t.p0 = a.p;
  t.p1 = e.p;
  t.o0 = a.o;
  t.o1 = a.o + N;
  t.n0 = t.n1 = (int)N;
  t.c0 = a.j + G;  // node index of slot i0 (a is slot i0 - G)
  if (t.p1 > t.p0) {
    t.r1 = (int)((int64_t)(t.p0 + 1) * L - i0);
    t.c1 = -t.r1 - G;
  } else {
    t.r1 = 1 << 30;
    t.c1 = t.c0;
  }
  return t;
}

// bc_index for a node index within [-G, n + G) of a problem of n > G nodes
__device__ __forceinline__ int bc_index_near(int j, int n, int bc) {
  if (bc == 0) return j < 0 ? j + n : (j >= n ? j - n : j);
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// A row of a tile in LDS as its own address.  Paired LDS reads (two
// doubles, offsets up to 2040 bytes from one address) of rows that lie
// further apart than that would otherwise each get an address add; the
// empty asm hides that the row is a constant offset of another address, so
// all reads of the row share one.
using lds_cptr = const __attribute__((address_space(3))) double*;
__device__ __forceinline__ lds_cptr lds_row(const double* p) {
  lds_cptr r = (lds_cptr)p;
  asm volatile("" : "+v"(r));
  return r;
}

// w_j = sum_e l_e u[e SV + j W], j = 0..5: one field of the six stencil
// nodes from the tile's nodes in LDS (variable rows SV doubles apart), one
// LDS address per variable row.
template <int NV, int SV, int W>
__device__ __forceinline__ void project_stencil(const double* u, const double (&l)[NV],
                                                double (&w)[6]) {
  lds_cptr ur[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) ur[e] = e > 0 ? lds_row(u + e * SV) : (lds_cptr)u;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double acc = l[0] * ur[0][j * W];
#pragma unroll
    for (int e = 1; e < NV; ++e) acc = __builtin_fma(l[e], ur[e][j * W], acc);
    w[j] = acc;
  }
}

__device__ __forceinline__ void flag_status(int32_t* status) {
  if (status) atomicOr(status, 1);
}

// The fields of SweepArgs that writing a result needs (emit): a kernel may
// read them late, from its argument segment, instead of holding them in
// scalar registers through its main loop.
struct EmitArgs {
  const double* U0;
  const double* Rin;
  double* out;
  int32_t* status;
  double ca, cb, cr;
  PhysParams pp;
};

template <class A>
__device__ __forceinline__ EmitArgs emit_args(const A& a) {
  EmitArgs e;
  e.U0 = a.U0;
  e.Rin = a.Rin;
  e.out = a.out;
  e.status = a.status;
  e.ca = a.ca;
  e.cb = a.cb;
  e.cr = a.cr;
  e.pp.gamma = a.pp.gamma;
  e.pp.adv = a.pp.adv;
  e.pp.charproj = a.pp.charproj;
  return e;
}

// Writes one node's result according to the sweep mode (MODE_RES, MODE_ACC,
// MODE_STAGE or MODE_LIN; `mode` is uniform, so the switch costs a scalar
// branch).  A is SweepArgs or EmitArgs.
template <int NV, class A>
__device__ __forceinline__ void emit_rt(int mode, const A& a, int64_t gidx, int64_t vstride,
                                        const double (&res)[NV], const double (&Un)[NV],
                                        double dt, double* yout = nullptr);

// Writes one node's result according to the sweep mode.  Un is the state
// under the stencil at that node (needed by the stage combine).  The stage
// combines read every input value of the node before the arithmetic, so
// that the loads are in flight together.
template <int NV, int MODE, class A>
__device__ __forceinline__ void emit(const A& a, int64_t gidx, int64_t vstride,
                                     const double (&res)[NV], const double (&Un)[NV],
                                     double dt, double* yout = nullptr) {
  if constexpr (MODE == MODE_RES) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = res[v];
  } else if constexpr (MODE == MODE_ACC) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = a.Rin[v * vstride + gidx] + res[v];
  } else if constexpr (MODE == MODE_LIN) {
    double y[NV], rin[NV], u0[NV];
    const bool hr = a.Rin != nullptr, h0 = a.ca != 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      rin[v] = hr ? a.Rin[v * vstride + gidx] : 0.0;
      u0[v] = h0 ? a.U0[v * vstride + gidx] : 0.0;
    }
    const double crdt = a.cr * dt;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = res[v];
      if (hr) r += rin[v];
      double s = __builtin_fma(crdt, r, a.cb * Un[v]);
      // (with ca = 0, u0 is 0 and the term adds +0: no select; an exact
      // zero result then comes out as +0)
      y[v] = __builtin_fma(a.ca, u0[v], s);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = y[v];
    if (!physical<NV>(y, a.pp.gamma)) flag_status(a.status);
  } else {
    double y[NV], rin[NV], u0[NV];
    const bool hr = a.Rin != nullptr, h0 = a.ca != 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      rin[v] = hr ? a.Rin[v * vstride + gidx] : 0.0;
      u0[v] = h0 ? a.U0[v * vstride + gidx] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = res[v];
      if (hr) r += rin[v];
      const double s = a.cb * __builtin_fma(dt, r, Un[v]);
      // (with ca = 0, u0 is 0 and the term adds +0: no select; an exact
      // zero result then comes out as +0)
      y[v] = __builtin_fma(a.ca, u0[v], s);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) a.out[v * vstride + gidx] = y[v];
    if (!physical<NV>(y, a.pp.gamma)) flag_status(a.status);
    if (yout) {
#pragma unroll
      for (int v = 0; v < NV; ++v) yout[v] = y[v];
    }
  }
}

template <int NV, class A>
__device__ __forceinline__ void emit_rt(int mode, const A& a, int64_t gidx, int64_t vstride,
                                        const double (&res)[NV], const double (&Un)[NV],
                                        double dt, double* yout) {
  if (mode == MODE_RES)
    emit<NV, MODE_RES>(a, gidx, vstride, res, Un, dt);
  else if (mode == MODE_ACC)
    emit<NV, MODE_ACC>(a, gidx, vstride, res, Un, dt);
  else if (mode == MODE_STAGE)
    emit<NV, MODE_STAGE>(a, gidx, vstride, res, Un, dt, yout);
  else
    emit<NV, MODE_LIN>(a, gidx, vstride, res, Un, dt);
}

}  // namespace wcns
