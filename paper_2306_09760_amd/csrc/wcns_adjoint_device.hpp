// Reverse-mode (vector-Jacobian) versions of the device arithmetic in
// wcns_device.hpp, written by hand.  Each *_vjp recomputes the forward
// intermediates it needs and propagates a cotangent backwards through them.
// Conventions at non-smooth points: d|x|/dx = 0 at x = 0; the tie in
// max(a, b) goes to the first argument; the PFE switch differentiates the
// branch it takes.
#pragma once

#include "wcns_device.hpp"

namespace wcns {

// g_i(w) and g_i'(w) of eq. 20 (see fe_map; d tanh = 1 - tanh^2, exactly 0
// where tanh saturates to +-1).
template <int SPEC>
__device__ __forceinline__ double fe_g_d(int i, double w, const InterpParams& P, double* dg) {
  if (i == 0) return fe_g0<SPEC>(w, P, dg);
  if (i == 1) return fe_g1<SPEC>(w, P, dg);
  return fe_g2<SPEC>(w, P, dg);
}

// The FE weights' part of the VJP on the forward SPEC_FE arithmetic: from
// the indicators IS_k, the candidates c_k and the output cotangent yb, the
// cotangents of the candidates (the weights times yb) and of the indicators
// (interp5_grad takes yb = 1: then the first three are the weights).
// Z weights z_k = Z_k / sum Z with Z_k = d_k (q_k + tau^2) prod_{l != k} q_l,
// q_k = (IS_k + eps)^2 (polynomial in q and tau^2, so their cotangents need
// no reciprocal); per map, with i_j = 1 / D_j = o_j / e (o_j the product of
// the other D, e of all), g = w - 2 sum_j A_j i_j and
// g' = 1 - 2 sum_j b_j i_j + 4 xi sum_j A_j i_j (1 - i_j).  Five
// reciprocals: sum Z, one per map, sum g.
template <bool TAB>
__device__ __forceinline__ void fe_weights_vjp(const InterpParams& P, double c0, double c1,
                                               double c2, double IS0, double IS1, double IS2,
                                               double yb, double& c0b, double& c1b, double& c2b,
                                               double& ISb0, double& ISb1, double& ISb2,
                                               const double* xt) {
  const double tau = __builtin_fabs(IS0 - IS2);
  const double t2 = tau * tau;
  const double b0 = IS0 + P.eps, b1 = IS1 + P.eps, b2 = IS2 + P.eps;
  const double q0 = b0 * b0, q1 = b1 * b1, q2 = b2 * b2;
  const double p12 = q1 * q2, p02 = q0 * q2, p01 = q0 * q1;
  const double u0 = q0 + t2, u1 = q1 + t2, u2 = q2 + t2;
  const double Z0 = D0 * u0 * p12, Z1 = D1 * u1 * p02, Z2 = D2 * u2 * p01;
  const double zi = rcp(Z0 + Z1 + Z2);
  const double z[3] = {Z0 * zi, Z1 * zi, Z2 * zi};
  const double xi2 = 2.0 * P.xi, xi4 = 4.0 * P.xi;
  // E_k = exp(2 xi z_k - C2_k); the third from the other two as in weigh5
  // (the z_k sum to one: E_0 E_1 E_2 = Ke)
  const double zE0 = __builtin_fma(xi2, z[0], -P.C2[0]), zE1 = __builtin_fma(xi2, z[1], -P.C2[1]);
  const double E0 = TAB ? exp_tab(zE0, xt) : exp_cw(zE0);
  const double E1 = TAB ? exp_tab(zE1, xt) : exp_cw(zE1);
  // the reciprocals below that do not feed an exponential's argument take
  // one Newton step (rcp1), as in the forward fast path
  const double E2 = P.Ke * rcp1(E0 * E1);
  double g[3], gp[3];
  auto map = [&](auto ntc, int k, const double* av, const double* bv, const double* K, double E) {
    constexpr int NT = decltype(ntc)::value;
    const double w = z[k];
    double D[NT], o[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) D[j] = __builtin_fma(E, K[j], 1.0);
    const double d01 = D[0] * D[1];
    double e;
    if constexpr (NT == 3) {
      o[0] = D[1] * D[2];
      o[1] = D[0] * D[2];
      o[2] = d01;
      e = d01 * D[2];
    } else {
      const double d23 = D[2] * D[3];
      o[0] = D[1] * d23;
      o[1] = D[0] * d23;
      o[2] = d01 * D[3];
      o[3] = d01 * D[2];
      e = d01 * d23;
    }
    const double r = rcp1(e);
    double gk = w, dk = 1.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const double i = o[j] * r;
      const double Ai = (bv[j] == 0.0 ? av[j] : __builtin_fma(bv[j], w, av[j])) * i;
      gk = __builtin_fma(-2.0, Ai, gk);
      if (bv[j] != 0.0) dk = __builtin_fma(-2.0 * bv[j], i, dk);
      dk = __builtin_fma(xi4 * Ai, 1.0 - i, dk);
    }
    g[k] = gk;
    gp[k] = dk;
  };
  map(std::integral_constant<int, 3>{}, 0, kG0a, kG0b, P.K, E0);
  map(std::integral_constant<int, 4>{}, 1, kG1a, kG1b, P.K + 3, E1);
  map(std::integral_constant<int, 3>{}, 2, kG2a, kG2b, P.K + 7, E2);
  const double rg = rcp1(g[0] + g[1] + g[2]);
  const double w0 = g[0] * rg, w1 = g[1] * rg, w2 = g[2] * rg;
  c0b = w0 * yb;
  c1b = w1 * yb;
  c2b = w2 * yb;
  // w = g / sum g: gb_k = (wb_k - sum_l wb_l w_l) / sum g
  const double wb0 = yb * c0, wb1 = yb * c1, wb2 = yb * c2;
  const double sdot = wb0 * w0 + wb1 * w1 + wb2 * w2;
  const double wb[3] = {wb0, wb1, wb2};
  double zb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) zb[k] = (wb[k] - sdot) * rg * gp[k];
  // z = Z / sum Z
  const double zdot = zb[0] * z[0] + zb[1] * z[1] + zb[2] * z[2];
  const double Y0 = D0 * (zb[0] - zdot) * zi, Y1 = D1 * (zb[1] - zdot) * zi,
               Y2 = D2 * (zb[2] - zdot) * zi;
  const double qb0 = Y0 * p12 + (Y1 * u1) * q2 + (Y2 * u2) * q1;
  const double qb1 = Y1 * p02 + (Y0 * u0) * q2 + (Y2 * u2) * q0;
  const double qb2 = Y2 * p01 + (Y0 * u0) * q1 + (Y1 * u1) * q0;
  const double t2b = Y0 * p12 + Y1 * p02 + Y2 * p01;
  ISb0 = 2.0 * b0 * qb0;
  ISb1 = 2.0 * b1 * qb1;
  ISb2 = 2.0 * b2 * qb2;
  const double taub = 2.0 * tau * t2b;
  const double dd = IS0 - IS2;
  const double sg = dd > 0.0 ? 1.0 : (dd < 0.0 ? -1.0 : 0.0);
  ISb0 += taub * sg;
  ISb2 -= taub * sg;
}

// One nonlinear interpolation (the left-biased one of interp5_pair) of the
// stencil (a, b, c, e, f) = (u_{i-2} .. u_{i+2}) and its gradient: returns
// the interpolated value y and G[j] = dy/du_j.  The value and the gradient
// come from the same intermediates (the weights, the maps and their slopes),
// so the adjoint needs no second evaluation of the weights: the cotangent of
// the stencil for an output cotangent yb is yb G.  y equals the forward
// value of interp5_pair to rounding (the weights are normalised here map by
// map rather than over one common denominator).
// xt: the kExp2Tab64 table in LDS (TAB = true, FE specialisation only).
template <int SPEC = SPEC_GENERIC, bool TAB = false>
__device__ __forceinline__ double interp5_grad(const InterpParams& P, double a, double b, double c,
                                               double e, double f, double (&G)[5],
                                               const double* xt = nullptr) {
  constexpr bool FE = (SPEC == SPEC_FE);
  constexpr double yb = 1.0;
  double y;
  double ab = 0.0, bb = 0.0, cb = 0.0, eb = 0.0, fb = 0.0;
  const double c0 = 0.125 * (3.0 * a - 10.0 * b + 15.0 * c);
  const double c1 = 0.125 * (-b + 6.0 * c + 3.0 * e);
  const double c2 = 0.125 * (3.0 * c + 6.0 * e - f);
  double c0b, c1b, c2b;
  if (!FE && P.weights == WLIN) {
    c0b = D0 * yb;
    c1b = D1 * yb;
    c2b = D2 * yb;
    y = D0 * c0 + D1 * c1 + D2 * c2;
  } else {
    const double d0 = b - a, d1 = c - b, d2 = e - c, d3 = f - e;
    const double f0 = 0.5 * (3.0 * d1 - d0), s0 = d1 - d0;
    const double f1 = 0.5 * (d1 + d2), s1 = d2 - d1;
    const double f2 = 0.5 * (3.0 * d2 - d3), s2 = d3 - d2;
    const double IS0 = f0 * f0 + s0 * s0;
    const double IS1 = f1 * f1 + s1 * s1;
    const double IS2 = f2 * f2 + s2 * s2;
    double ISb0, ISb1, ISb2;
    if constexpr (FE) {
      fe_weights_vjp<TAB>(P, c0, c1, c2, IS0, IS1, IS2, yb, c0b, c1b, c2b, ISb0, ISb1, ISb2, xt);
      y = c0b * c0 + c1b * c1 + c2b * c2;  // (the weights, yb = 1)
    } else {
      const double r0 = rcp(IS0 + P.eps), r1 = rcp(IS1 + P.eps), r2 = rcp(IS2 + P.eps);
      double a0, a1, a2, w0, w1, w2, tau = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0;
      const int zpow = P.zpow;
      const bool js = P.weights == WJS;
      if (js) {
        a0 = D0 * r0 * r0;
        a1 = D1 * r1 * r1;
        a2 = D2 * r2 * r2;
      } else {
        tau = __builtin_fabs(IS0 - IS2);
        q0 = tau * r0;
        q1 = tau * r1;
        q2 = tau * r2;
        double p0 = q0, p1 = q1, p2 = q2;
        for (int k = 1; k < zpow; ++k) {
          p0 *= q0;
          p1 *= q1;
          p2 *= q2;
        }
        a0 = D0 * (1.0 + p0);
        a1 = D1 * (1.0 + p1);
        a2 = D2 * (1.0 + p2);
      }
      const double inv = rcp(a0 + a1 + a2);
      const double z0 = a0 * inv, z1 = a1 * inv, z2 = a2 * inv;
      bool map = P.weights == WFE;
      if (P.weights == WPFE) {
        const bool inside = __builtin_fabs(z0 - D0) <= P.cv && __builtin_fabs(z1 - D1) <= P.cv &&
                            __builtin_fabs(z2 - D2) <= P.cv;
        map = !inside;
      }
      double zb0, zb1, zb2;
      if (map) {
        double d0, d1, d2;
        const double g0 = fe_g_d<SPEC>(0, z0, P, &d0);
        const double g1 = fe_g_d<SPEC>(1, z1, P, &d1);
        const double g2 = fe_g_d<SPEC>(2, z2, P, &d2);
        const double ginv = rcp(g0 + g1 + g2);
        w0 = g0 * ginv;
        w1 = g1 * ginv;
        w2 = g2 * ginv;
        const double wb0 = yb * c0, wb1 = yb * c1, wb2 = yb * c2;
        const double sdot = wb0 * w0 + wb1 * w1 + wb2 * w2;
        zb0 = (wb0 - sdot) * ginv * d0;
        zb1 = (wb1 - sdot) * ginv * d1;
        zb2 = (wb2 - sdot) * ginv * d2;
      } else {
        w0 = z0;
        w1 = z1;
        w2 = z2;
        zb0 = yb * c0;
        zb1 = yb * c1;
        zb2 = yb * c2;
      }
      c0b = w0 * yb;
      c1b = w1 * yb;
      c2b = w2 * yb;
      y = w0 * c0 + w1 * c1 + w2 * c2;
      // z = alpha / sum(alpha)
      const double zdot = zb0 * z0 + zb1 * z1 + zb2 * z2;
      const double ab0 = (zb0 - zdot) * inv, ab1 = (zb1 - zdot) * inv, ab2 = (zb2 - zdot) * inv;
      if (js) {
        // alpha = d r^2, r = 1/(IS + eps): d alpha / d IS = -2 d r^3
        ISb0 = -2.0 * D0 * r0 * r0 * r0 * ab0;
        ISb1 = -2.0 * D1 * r1 * r1 * r1 * ab1;
        ISb2 = -2.0 * D2 * r2 * r2 * r2 * ab2;
      } else {
        // alpha = d (1 + q^p), q = tau r
        double dp0 = 1.0, dp1 = 1.0, dp2 = 1.0;  // d q^p / dq = p q^(p-1)
        for (int k = 1; k < zpow; ++k) {
          dp0 *= q0;
          dp1 *= q1;
          dp2 *= q2;
        }
        const double qb0 = D0 * ab0 * zpow * dp0;
        const double qb1 = D1 * ab1 * zpow * dp1;
        const double qb2 = D2 * ab2 * zpow * dp2;
        const double taub = qb0 * r0 + qb1 * r1 + qb2 * r2;
        ISb0 = -qb0 * tau * r0 * r0;
        ISb1 = -qb1 * tau * r1 * r1;
        ISb2 = -qb2 * tau * r2 * r2;
        const double dd = IS0 - IS2;
        const double sg = dd > 0.0 ? 1.0 : (dd < 0.0 ? -1.0 : 0.0);
        ISb0 += taub * sg;
        ISb2 -= taub * sg;
      }
    }
    const double f0b = 2.0 * f0 * ISb0, s0b = 2.0 * s0 * ISb0;
    const double f1b = 2.0 * f1 * ISb1, s1b = 2.0 * s1 * ISb1;
    const double f2b = 2.0 * f2 * ISb2, s2b = 2.0 * s2 * ISb2;
    // back through the first differences d0..d3
    const double db0 = -0.5 * f0b - s0b;
    const double db1 = 1.5 * f0b + s0b + 0.5 * f1b - s1b;
    const double db2 = 0.5 * f1b + s1b + 1.5 * f2b - s2b;
    const double db3 = -0.5 * f2b + s2b;
    ab -= db0;
    bb += db0 - db1;
    cb += db1 - db2;
    eb += db2 - db3;
    fb += db3;
  }
  ab += 0.375 * c0b;
  bb += -1.25 * c0b - 0.125 * c1b;
  cb += 1.875 * c0b + 0.75 * c1b + 0.375 * c2b;
  eb += 0.375 * c1b + 0.75 * c2b;
  fb += -0.125 * c2b;
  G[0] = ab;
  G[1] = bb;
  G[2] = cb;
  G[3] = eb;
  G[4] = fb;
  return y;
}

// Ub += (dF/dU)^T Fb + (d lam/dU)^T lamb for the Euler flux along DIR and the
// wave speed lam = |u_n| + c of one state.
template <int ND, int DIR>
__device__ __forceinline__ void flux_speed_vjp(const double* U, double gamma, const double* Fb,
                                               double lamb, double* Ub) {
  const double rho = U[0], E = U[ND + 1];
  const double ir = rcp(rho);
  double vel[ND], msq = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    vel[k] = U[1 + k] * ir;
    msq += U[1 + k] * U[1 + k];
  }
  const double mm = msq * ir;
  const double p = (gamma - 1.0) * (E - 0.5 * mm);
  const double vn = vel[DIR];
  double mb[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) mb[k] = 0.0;
  double vnb = 0.0, pb = 0.0, Eb = 0.0, irb = 0.0;
  mb[DIR] += Fb[0];
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    mb[k] += Fb[1 + k] * vn;
    vnb += Fb[1 + k] * U[1 + k];
  }
  pb += Fb[1 + DIR];
  Eb += Fb[ND + 1] * vn;
  pb += Fb[ND + 1] * vn;
  vnb += Fb[ND + 1] * (E + p);
  if (lamb != 0.0) {
    vnb += lamb * (vn > 0.0 ? 1.0 : (vn < 0.0 ? -1.0 : 0.0));
    const double X = gamma * p * ir;
    const double cs = sqrt_pos(X);
    const double Xb = 0.5 * lamb * rcp(cs);
    pb += Xb * gamma * ir;
    irb += Xb * gamma * p;
  }
  // p = (gamma-1)(E - mm/2), mm = |m|^2 ir
  Eb += (gamma - 1.0) * pb;
  const double mmb = -0.5 * (gamma - 1.0) * pb;
#pragma unroll
  for (int k = 0; k < ND; ++k) mb[k] += mmb * 2.0 * vel[k];
  irb += mmb * msq;
  // vn = m_n ir
  mb[DIR] += vnb * ir;
  irb += vnb * U[1 + DIR];
  Ub[0] += -irb * ir * ir;
#pragma unroll
  for (int k = 0; k < ND; ++k) Ub[1 + k] += mb[k];
  Ub[ND + 1] += Eb;
}

// Cotangent of the Roe-averaged quantities.
template <int ND>
struct RoeBar {
  double vel[ND];
  double H, c, ic, q2h, b1, b2;
};

// Propagates rb back to the two node states (accumulating into UbA, UbB).
template <int ND>
__device__ __forceinline__ void roe_vjp(const double* UA, const double* UB, double gamma,
                                        const RoeState<ND>& r, RoeBar<ND> rb, double* UbA,
                                        double* UbB) {
  // b2 = q2h b1 ; b1 = (g-1) ic^2 ; ic = 1/c
  rb.q2h += rb.b2 * r.b1;
  rb.b1 += rb.b2 * r.q2h;
  rb.ic += rb.b1 * 2.0 * (gamma - 1.0) * r.ic;
  rb.c += -rb.ic * r.ic * r.ic;
  // c = sqrt((g-1)(H - q2h))
  const double Yb = rb.c * 0.5 * r.ic;
  rb.H += Yb * (gamma - 1.0);
  rb.q2h -= Yb * (gamma - 1.0);
#pragma unroll
  for (int k = 0; k < ND; ++k) rb.vel[k] += rb.q2h * r.vel[k];
  // Forward pieces of the average.
  const Prim<ND> A = primitives<ND>(UA, gamma);
  const Prim<ND> B = primitives<ND>(UB, gamma);
  const double sA = sqrt_pos(UA[0]), sB = sqrt_pos(UB[0]);
  const double den = rcp(sA + sB);
  const double wA = sA * den, wB = sB * den;
  const double HA = (UA[ND + 1] + A.p) * A.ir;
  const double HB = (UB[ND + 1] + B.p) * B.ir;
  double wAb = rb.H * HA, wBb = rb.H * HB;
  const double HAb = rb.H * wA, HBb = rb.H * wB;
  double velAb[ND], velBb[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    wAb += rb.vel[k] * A.vel[k];
    wBb += rb.vel[k] * B.vel[k];
    velAb[k] = rb.vel[k] * wA;
    velBb[k] = rb.vel[k] * wB;
  }
  const double denb = wAb * sA + wBb * sB;
  const double Sb = -denb * den * den;
  const double sAb = wAb * den + Sb;
  const double sBb = wBb * den + Sb;
  // Node A: H = (E + p) ir, vel = m ir, p = (g-1)(E - |m|^2 ir / 2), ir = 1/rho, s = sqrt(rho)
  auto node = [&](const double* U, const Prim<ND>& Q, double s, double sb, double Hb,
                  const double* velb, double* Ub) {
    double irb = Hb * (U[ND + 1] + Q.p);
    double Eb = Hb * Q.ir;
    const double pb = Hb * Q.ir;
    Eb += (gamma - 1.0) * pb;
    const double mmb = -0.5 * (gamma - 1.0) * pb;
    double msq = 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) msq += U[1 + k] * U[1 + k];
    irb += mmb * msq;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      Ub[1 + k] += mmb * 2.0 * Q.vel[k] + velb[k] * Q.ir;
      irb += velb[k] * U[1 + k];
    }
    Ub[ND + 1] += Eb;
    Ub[0] += -irb * Q.ir * Q.ir + 0.5 * sb * rcp(s);
  };
  node(UA, A, sA, sAb, HAb, velAb, UbA);
  node(UB, B, sB, sBb, HBb, velBb, UbB);
}

// Local Lax-Friedrichs flux F = (F(UL) + F(UR)) / 2 - alpha (UR - UL) / 2,
// alpha = max(lam(UL), lam(UR)): sets ULb, URb = (dF/dUL)^T Fb, (dF/dUR)^T Fb.
template <int ND, int DIR>
__device__ __forceinline__ void llf_vjp(const double* UL, const double* UR, double gamma,
                                        const double* Fb, double* ULb, double* URb) {
  constexpr int NV = ND + 2;
  const Prim<ND> L = primitives<ND>(UL, gamma);
  const Prim<ND> R = primitives<ND>(UR, gamma);
  const double lamL = __builtin_fabs(L.vel[DIR]) + sqrt_pos(gamma * L.p * L.ir);
  const double lamR = __builtin_fabs(R.vel[DIR]) + sqrt_pos(gamma * R.p * R.ir);
  const bool takeL = lamL >= lamR;
  const double alpha = takeL ? lamL : lamR;
  double alphab = 0.0, Fh[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    alphab += -0.5 * (UR[v] - UL[v]) * Fb[v];
    ULb[v] = 0.5 * alpha * Fb[v];
    URb[v] = -0.5 * alpha * Fb[v];
    Fh[v] = 0.5 * Fb[v];
  }
  flux_speed_vjp<ND, DIR>(UL, gamma, Fh, takeL ? alphab : 0.0, ULb);
  flux_speed_vjp<ND, DIR>(UR, gamma, Fh, takeL ? 0.0 : alphab, URb);
}

// Back-projection U = R W (see unproject): sets Wb = R^T Ub and accumulates
// the cotangent of the Roe quantities R depends on into rb.
template <int ND, int DIR>
__device__ __forceinline__ void unproject_vjp(const RoeState<ND>& r, const double* W,
                                              const double* Ub, double* Wb, RoeBar<ND>& rb) {
  constexpr int NV = ND + 2;
  const double sum = W[0] + W[1] + W[ND + 1];
  const double dif = W[ND + 1] - W[0];
  double sumb = Ub[0], difb = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) Wb[v] = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    rb.vel[k] += Ub[1 + k] * sum;
    sumb += Ub[1 + k] * r.vel[k];
  }
  rb.c += Ub[1 + DIR] * dif;
  difb += Ub[1 + DIR] * r.c;
  const double Eb = Ub[ND + 1];
  rb.H += Eb * (W[0] + W[ND + 1]);
  Wb[0] += Eb * r.H;
  Wb[ND + 1] += Eb * r.H;
  rb.vel[DIR] += Eb * r.c * dif;
  rb.c += Eb * r.vel[DIR] * dif;
  difb += Eb * r.vel[DIR] * r.c;
  rb.q2h += Eb * W[1];
  Wb[1] += Eb * r.q2h;
#pragma unroll
  for (int t = 0; t < ND - 1; ++t) {
    const int ax = tangential_axis<ND, DIR>(t);
    Wb[2 + t] += Ub[1 + ax] + Eb * r.vel[ax];
    rb.vel[ax] += Eb * W[2 + t];
  }
  Wb[0] += sumb - difb;
  Wb[1] += sumb;
  Wb[ND + 1] += sumb + difb;
}

// Projection W = L U of one node (see project): accumulates Ub += L^T Wb
// and the cotangent of the Roe quantities L depends on into rb.
template <int ND, int DIR>
__device__ __forceinline__ void project_vjp(const RoeState<ND>& r, const double* U,
                                            const double* Wb, double* Ub, RoeBar<ND>& rb) {
  double um = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) um += r.vel[k] * U[1 + k];
  const double thb = 0.5 * Wb[0] - Wb[1] + 0.5 * Wb[ND + 1];
  const double anb = 0.5 * Wb[0] - 0.5 * Wb[ND + 1];
  Ub[0] += Wb[1];
#pragma unroll
  for (int t = 0; t < ND - 1; ++t) {
    const int ax = tangential_axis<ND, DIR>(t);
    Ub[1 + ax] += Wb[2 + t];
    rb.vel[ax] -= Wb[2 + t] * U[0];
    Ub[0] -= Wb[2 + t] * r.vel[ax];
  }
  // an = (vel_n rho - m_n) ic
  rb.vel[DIR] += anb * U[0] * r.ic;
  Ub[0] += anb * r.vel[DIR] * r.ic;
  Ub[1 + DIR] -= anb * r.ic;
  rb.ic += anb * (r.vel[DIR] * U[0] - U[1 + DIR]);
  // theta = b2 rho - b1 um + b1 E
  rb.b2 += thb * U[0];
  Ub[0] += thb * r.b2;
  rb.b1 += thb * (U[ND + 1] - um);
  Ub[ND + 1] += thb * r.b1;
  const double umb = -thb * r.b1;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    rb.vel[k] += umb * U[1 + k];
    Ub[1 + k] += umb * r.vel[k];
  }
}

// Ub += (dF/dU)^T Fb for the physical flux at a node.
template <int NV, int DIR>
__device__ __forceinline__ void node_flux_vjp(const PhysParams& PP, const double (&U)[NV],
                                              const double (&Fb)[NV], double (&Ub)[NV]) {
  if constexpr (NV == 1) {
    Ub[0] += PP.adv * Fb[0];
  } else {
    flux_speed_vjp<NV - 2, DIR>(U, PP.gamma, Fb, 0.0, Ub);
  }
}

}  // namespace wcns
