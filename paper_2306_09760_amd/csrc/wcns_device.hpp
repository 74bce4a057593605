// Device arithmetic of the WCNS-FE residual for gfx950 (FP64 VALU).
//
// Everything here is a __device__ inline function used by the sweep, batch
// and adjoint kernels.  The formulas follow arXiv 2306.09760:
//   smoothness indicators          eq. 9-10
//   JS weights                     eq. 11  (denominator (IS + eps)^2)
//   Z weights                      eq. 14-15 (integer exponent p)
//   FE mapping                     eq. 20-21 with the coefficient table of
//                                  Sec. 3.1, applied to the Z weights and
//                                  renormalised
//   PFE switch                     App. A (inclusive band)
//   candidate interpolations       eq. 5, combined per eq. 6
//   Euler flux                     eq. 32 (extended to 2D/3D)
// The characteristic projection (Roe-averaged eigenvectors of the
// direction-normal Jacobian) and the local Lax-Friedrichs midpoint flux are
// the readings chosen where the paper only says "approximate Riemann
// solution".
//
// Cost notes (the path is bound by FP64 VALU issue, not by HBM):
//  * the projection uses the sparsity of the Euler eigenvectors: one shared
//    scalar theta = b2*rho - b1*(u.m) + b1*E per node instead of a dense
//    nv x nv product;
//  * reciprocals are v_rcp_f64 refined by two Newton steps;
//  * tanh returns +-1 without evaluation once |x| >= 20 (tanh(x) rounds to
//    +-1 in FP64 for |x| > 19.06), which at large steepness xi covers almost
//    every call.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wcns {

// Weight choice codes (same values as wcns_weights in wcns.h).
enum : int { WJS = 0, WZ = 1, WFE = 2, WPFE = 3, WLIN = 4 };

// Compile-time specialisation of the interpolation.  SPEC_FE is the paper's
// configuration (FE weights on Z weights with p = 2, one shared exponential
// per map); SPEC_GENERIC switches on the runtime parameters.
// SPEC_FE: FE weights on p = 2 Z weights with one exponential per map
// (fast_fe); SPEC_FE_SAT: the same weights where every term takes its own
// saturating tanh (large xi, shared_exp = 0); SPEC_GENERIC: every choice.
enum : int { SPEC_GENERIC = 0, SPEC_FE = 1, SPEC_FE_SAT = 2 };

// Uniform parameters of the interpolation, passed by value to kernels.
struct InterpParams {
  double eps;       // eq. 11 / eq. 14
  double xi;        // steepness of eq. 20
  double cv;        // PFE band (App. A)
  // Per term j of the three maps (g0: 0..2, g1: 3..6, g2: 7..9), with the null
  // points nu_j = kappa*(psi_{i,j} + psi_{i,j-1}) and a reference point c_i per
  // map (the mean of its null points):
  //   shared_exp = 1:  K[j] = exp(2 xi (c_i - nu_j)),  C2[i] = 2 xi c_i
  //   shared_exp = 0:  K[j] = nu_j                      (C2 unused)
  double K[10];
  double C2[3];
  double Ke;        // exp(2 xi - C2[0] - C2[1] - C2[2]) (shared_exp; weigh5)
  // fe_map_poly (shared_exp): per map m with NT_m terms, prod_j D_j and the
  // two parts of sum_j -2 A_j(w) prod_{l != j} D_l, alpha (constant in w)
  // and beta (times w), D_j = 1 + E K_j, as polynomials in E divided by the
  // leading coefficient prod_j K_j (= 1 up to rounding: c_m is the mean of
  // the map's null points), so that the denominator is monic:
  //   Pd = [c_1 .. c_{NT-1}, c_0] for E^NT + c_{NT-1} E^{NT-1} + .. + c_0,
  //   Pa, Pb = the coefficients of E^1 .. E^{NT-1} (the constants vanish);
  // maps at offsets 0, 3, 7 of Pd and 0, 2, 5 of Pa and Pb
  double Pd[10], Pa[7], Pb[7];
  int weights;      // WJS .. WLIN
  int zpow;         // exponent p of eq. 14 (1..4)
  int shared_exp;   // 1: one exponential per map (xi * max|nu - c| < 300)
  int weno;         // 1: K, C2 hold the Table B.2 maps (WENO family)
  int fast_fe;      // 1: shared_exp and the unclamped products of the
                    //    SPEC_FE path stay below e^600 (see fe_map_poly)
};

// Physics parameters of one sweep.
struct PhysParams {
  double gamma;     // Euler
  double adv;       // advection speed along the sweep direction
  int charproj;     // 1 = characteristic projection
};

__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  return r;
}
// 1/x with one Newton step: the seed's relative error (at most 2^-24.4)
// squared, 2^-48.8 (about 10 ulp), for reciprocals whose error reaches the
// result only in proportion (a final normalisation), never through an
// exponential's argument.
__device__ __forceinline__ double rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// sqrt(x) for x = 0 or 2^-760 <= x < inf (densities, pressures, sound speeds
// squared): v_rsq_f64 seed, one Goldschmidt step for sqrt and 1/(2 sqrt),
// two Newton corrections of the root (about 1 ulp); NaN for x < -2^-1000.
// Without the rescaling that a full-range square root needs for tiny
// arguments.  The seed is taken at x + 2^-1000, which is x itself from
// 2^-760 up and keeps x = 0 off the seed's pole: there every step below
// gives g = 0 exactly, with no select.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x + 0x1p-1000);
  double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  return g;
}

// e^z for |z| <= 708 (Cody-Waite reduction z = n ln2 + r, |r| <= ln2/2, then
// the Taylor polynomial of e^r to degree 13: truncation below 5e-18).
__device__ __forceinline__ double exp_cw(double z) {
  constexpr double kLog2e = 0x1.71547652b82fep+0;
  constexpr double kLn2Hi = 0x1.62e42ff000000p-1;   // ln 2 to 32 bits: n*hi is exact
  constexpr double kLn2Lo = -0x1.718432a1b0e26p-35; // ln 2 - hi
  const double n = __builtin_rint(z * kLog2e);
  double r = __builtin_fma(-n, kLn2Hi, z);
  r = __builtin_fma(-n, kLn2Lo, r);
  double p = 1.6059043836821613e-10;            // 1/13!
  p = __builtin_fma(p, r, 2.08767569878681e-09);  // 1/12!
  p = __builtin_fma(p, r, 2.505210838544172e-08);
  p = __builtin_fma(p, r, 2.755731922398589e-07);
  p = __builtin_fma(p, r, 2.7557319223985893e-06);
  p = __builtin_fma(p, r, 2.48015873015873e-05);
  p = __builtin_fma(p, r, 0.0001984126984126984);
  p = __builtin_fma(p, r, 0.001388888888888889);
  p = __builtin_fma(p, r, 0.008333333333333333);
  p = __builtin_fma(p, r, 0.041666666666666664);
  p = __builtin_fma(p, r, 0.16666666666666666);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_ldexp(p, (int)n);
}

// 2^(k/64), k = 0..63, each correctly rounded (generated in 60-digit decimal
// arithmetic).  Kernels that call exp_tab copy it into LDS first.
__device__ constexpr double kExp2Tab64[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};

// e^z for |z| <= 708 through the table above (Tang's method, ACM TOMS 15
// (1989)): z = (64 m + k) ln2/64 + r with |r| <= ln2/128, reduced with a
// 36-bit head of ln2/64 (exact for |64 m + k| < 2^17) and its tail; e^r - 1
// from the degree-5 Taylor polynomial (truncation r^6 / 720 < 3.6e-17, a
// third of an ulp of 1); the result is 2^m (T_k + T_k (e^r - 1)).  T points
// to the table in LDS.
__device__ __forceinline__ double exp_tab(double z, const double* T) {
  constexpr double kInv = 0x1.71547652b82fep+6;       // 64 / ln 2
  constexpr double kHi = 0x1.62e42fefa0000p-7;        // ln2/64, 36 significant bits
  constexpr double kLo = 0x1.cf79abc9e3b3ap-46;       // ln2/64 - kHi
  // z * 64/ln2 rounded to an integer by adding 1.5 * 2^52: the sum's low 32
  // bits hold it in two's complement (|z| <= 708 keeps it below 2^17)
  constexpr double kShift = 0x1.8p52;
  const double sh = __builtin_fma(z, kInv, kShift);
  const double n = sh - kShift;
  double r = __builtin_fma(-n, kHi, z);
  r = __builtin_fma(-n, kLo, r);
  const int ni = (int)(unsigned)__builtin_bit_cast(unsigned long long, sh);
  const double t = T[ni & 63];
  double p = 1.0 / 120.0;
  p = __builtin_fma(p, r, 1.0 / 24.0);
  p = __builtin_fma(p, r, 1.0 / 6.0);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p *= r;
  return __builtin_ldexp(__builtin_fma(t, p, t), ni >> 6);
}

// tanh(x) = sign(x) (1 - e^{-2|x|}) / (1 + e^{-2|x|}); +-1 for |x| >= 20.
__device__ __forceinline__ double tanh_sat(double x) {
  const double ax = __builtin_fabs(x);
  double r = 1.0;
  if (ax < 20.0) {
    const double e = exp_cw(-2.0 * ax);
    r = (1.0 - e) * rcp(1.0 + e);
  }
  return __builtin_copysign(r, x);
}

// Ideal weights d_k (Sec. 2).
constexpr double D0 = 1.0 / 16.0, D1 = 10.0 / 16.0, D2 = 5.0 / 16.0;

// g_i of eq. 20 for one map with NT terms:
//   g(w) = w + sum_j A_j(w) tanh(xi (w - nu_j)),  A_j(w) = a_j + b_j w.
// phi(i,j) * tanh(xi * phi(i,j) * x) = tanh(xi * x) because tanh is odd and
// phi = +-1, so the sign table of eq. 21 folds away; the amplitudes
// (omega_{i,j} - omega_{i,j-1}) / 2 come from the coefficient table, and an
// entry equal to the argument makes b_j = +-1/2.
// All terms of one map share w, so with E = exp(2 xi w - 2 xi c) every term is
// tanh(xi (w - nu_j)) = (q_j - 1) / (q_j + 1), q_j = E K_j = exp(2 xi (w -
// nu_j)): one exponential per map instead of one per term.  A term is
// saturated (tanh = +-1 in FP64) exactly when q_j is outside (e^-40, e^40).
// E and E K_j stay finite and normal whenever a term is unsaturated as long
// as xi |nu_j - c| < 300 (shared_exp); beyond that each unsaturated term
// takes its own exponential.  If dg is not null it receives g'(w).
template <int NT, int SPEC>
__device__ __forceinline__ double fe_map(double w, const double (&a)[NT], const double (&b)[NT],
                                         const double* K, double C2, const InterpParams& P,
                                         double* dg) {
  constexpr double kQlo = 4.248354255291589e-18;  // e^-40
  constexpr double kQhi = 2.3538526683702e+17;    // e^40
  const bool shared = (SPEC == SPEC_FE) || P.shared_exp;
  double g = w, d = 1.0;
  double E = 0.0;
  if (shared) E = exp_cw(__builtin_fma(2.0 * P.xi, w, -C2));
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    double t;
    if (shared) {
      const double q = E * K[j];
      t = (q > 1.0) ? 1.0 : -1.0;
      if (q > kQlo && q < kQhi) t = (q - 1.0) * rcp(q + 1.0);
    } else {
      t = tanh_sat(P.xi * (w - K[j]));
    }
    const double A = b[j] == 0.0 ? a[j] : __builtin_fma(b[j], w, a[j]);
    g = __builtin_fma(A, t, g);
    if (dg) d += b[j] * t + A * P.xi * (1.0 - t * t);
  }
  if (dg) *dg = d;
  return g;
}

// A_j = a_j + b_j w of the three maps.
constexpr double kG0a[3] = {0.5 * D0, 0.5 * (1.0 / 6.0 - D0), -0.5 / 6.0};
constexpr double kG0b[3] = {-0.5, 0.0, 0.5};
constexpr double kG1a[4] = {0.5 * D1, 0.5 * (0.5 - D1), 0.5 * (5.0 / 6.0 - 0.5), -0.5 * 5.0 / 6.0};
constexpr double kG1b[4] = {-0.5, 0.0, 0.0, 0.5};
constexpr double kG2a[3] = {0.5 * D2, 0.5 * (0.5 - D2), -0.25};
constexpr double kG2b[3] = {-0.5, 0.0, 0.5};

// Each map is the identity below its first null point, where every t_j is -1
// in the limit: g = w - sum_j A_j(w) there, so the a_j and the b_j of a map
// sum to zero and sum_j A_j(w) = 0 for every w.
constexpr bool map_sums_vanish(const double* a, const double* b, int n) {
  double sa = 0.0, sb = 0.0, m = 0.0;
  for (int j = 0; j < n; ++j) {
    sa += a[j];
    sb += b[j];
    m = (a[j] < 0 ? -a[j] : a[j]) > m ? (a[j] < 0 ? -a[j] : a[j]) : m;
  }
  return sb == 0.0 && (sa < 0 ? -sa : sa) <= 1e-15 * m;
}
constexpr bool kMapSumsVanish = map_sums_vanish(kG0a, kG0b, 3) &&
                                map_sums_vanish(kG1a, kG1b, 4) &&
                                map_sums_vanish(kG2a, kG2b, 3);
static_assert(kMapSumsVanish, "the FE maps' A_j must sum to zero");

template <int SPEC = SPEC_GENERIC>
__device__ __forceinline__ double fe_g0(double w, const InterpParams& P, double* dg = nullptr) {
  return fe_map<3, SPEC>(w, kG0a, kG0b, P.K, P.C2[0], P, dg);
}
template <int SPEC = SPEC_GENERIC>
__device__ __forceinline__ double fe_g1(double w, const InterpParams& P, double* dg = nullptr) {
  return fe_map<4, SPEC>(w, kG1a, kG1b, P.K + 3, P.C2[1], P, dg);
}
template <int SPEC = SPEC_GENERIC>
__device__ __forceinline__ double fe_g2(double w, const InterpParams& P, double* dg = nullptr) {
  return fe_map<3, SPEC>(w, kG2a, kG2b, P.K + 7, P.C2[2], P, dg);
}

// g(w) of one map in the form used by the forward SPEC_FE path.  With
// t_j = tanh(xi (w - nu_j)) = 1 - 2 / D_j, D_j = 1 + q_j, q_j = E K_j:
//   g(w) = w + sum_j A_j(w) - 2 sum_j A_j(w) / D_j,
// taken over the common denominator prod_j D_j: the map returns the
// numerator and leaves the denominator in *den, so that the caller can
// normalise the three maps with one reciprocal.  The D_j are not clamped:
// ln prod_j D_j is convex in w, so over the simplex of (w_0, w_1, w_2) the
// product of all three maps' denominators peaks at a vertex, at
// B = max_i [sum_j softplus(2 xi (1 - nu_ij)) + sum_{l != i, j} softplus(-2 xi nu_lj)]
// (469 at xi = 100, kappa = 0.5).  The host selects this path only while
// B < 600 (fast_fe), which leaves e^100 of headroom for the candidate values
// that multiply the products; below e^-45 a q_j rounds away against 1.
// E = exp(2 xi w - C2) is the caller's (weigh5).  The numerator and the
// denominator are polynomials in E whose coefficients are constants of the
// plan (InterpParams::Pd, Pa, Pb): Horner's rule in E takes 8 (NT = 3) or
// 11 (NT = 4) operations instead of 12 and 16 for the products of the D_j.
// The denominator's coefficients are positive, so it has no cancellation;
// with the plan's maps the polynomial form rounds g(w) within 3.4e-16 of
// its exact value over w in [0, 1], as the product form does within 1.4e-16.
// The denominator is monic, so its Horner chain starts from E + c_{NT-1}
// (no instruction with two constant operands, which the vector ALU cannot
// read in one operation).
template <int NT>
__device__ __forceinline__ double fe_map_poly(double w, double E, const double* pd,
                                              const double* pa, const double* pb, double* den) {
  static_assert(NT == 3 || NT == 4, "maps have three or four terms");
  double t = E + pd[NT - 2];
#pragma unroll
  for (int r = NT - 3; r >= 0; --r) t = __builtin_fma(t, E, pd[r]);
  *den = __builtin_fma(t, E, pd[NT - 1]);
  double ta = pa[NT - 2], tb = pb[NT - 2];
#pragma unroll
  for (int r = NT - 3; r >= 0; --r) {
    ta = __builtin_fma(ta, E, pa[r]);
    tb = __builtin_fma(tb, E, pb[r]);
  }
  // sum_j A_j(w) = 0 for every map (kMapSumsVanish), so g = w - 2 sum_j A_j / D_j.
  return __builtin_fma(w, *den, E * __builtin_fma(w, tb, ta));
}

// Constants of one scheme family in the FE fast path of weigh5: the ideal
// weights, the A_j = a_j + b_j w of its three maps, and the factor the
// candidates passed to weigh5 are scaled by (1/8 for the WCNS candidates of
// eq. 5, 1/6 for the WENO5 ones).
struct FamWcns {
  static constexpr double d0 = D0, d1 = D1, d2 = D2, scale = 0.125;
  static constexpr double dr1 = 10.0, dr2 = 5.0;  // d_1 / d_0, d_2 / d_0
  static constexpr const double (&m0a)[3] = kG0a;
  static constexpr const double (&m0b)[3] = kG0b;
  static constexpr const double (&m1a)[4] = kG1a;
  static constexpr const double (&m1b)[4] = kG1b;
  static constexpr const double (&m2a)[3] = kG2a;
  static constexpr const double (&m2b)[3] = kG2b;
};

// The nonlinear weights of eq. 11 / 14 (+ FE map, eq. 20; PFE switch) from
// the regularised smoothness indicators b_k = IS_k + eps (so that
// tau = |IS_0 - IS_2| = |b_0 - b_2|), applied to the candidates of eq. 5; (c0, c1, c2)
// are eight times the candidates (the 1/8 is applied once, to the sum).  The
// FE branch serves either family (FAM); the generic branch is the WCNS one.
// xt: the kExp2Tab64 table in LDS (TAB = true), else unused.
template <int SPEC = SPEC_GENERIC, bool TAB = false, class FAM = FamWcns>
__device__ __forceinline__ double weigh5(const InterpParams& P, double c0, double c1, double c2,
                                         double b0, double b1, double b2,
                                         const double* xt = nullptr) {
  constexpr bool FE = (SPEC == SPEC_FE);
  if constexpr (FE) {
    // Z weights (p = 2) over the common denominator: alpha_k b_0^2 b_1^2 b_2^2
    // = d_k (b_k^2 + tau^2) times the other two squares, here divided by d_0
    // (the ratios d_k / d_0 are small integers; the normalisation removes
    // the common factor); one reciprocal normalises them.  The smallest
    // product, eps^6 = 1e-240, is still a normal number.
    const double tau = __builtin_fabs(b0 - b2);
    const double t2 = tau * tau;
    const double q0 = b0 * b0, q1 = b1 * b1, q2 = b2 * b2;
    const double z0 = (q0 + t2) * (q1 * q2);
    const double z1 = FAM::dr1 * (q1 + t2) * (q0 * q2);
    const double z2 = FAM::dr2 * (q2 + t2) * (q0 * q1);
    const double zi = rcp(z0 + z1 + z2);
    const double xi2 = 2.0 * P.xi;
    const double w0 = z0 * zi, w1 = z1 * zi, w2 = z2 * zi;
    // E_k = exp(2 xi w_k - C2_k).  The Z weights sum to one, so E_0 E_1 E_2 =
    // exp(2 xi - C2_0 - C2_1 - C2_2) = Ke and the third exponential is
    // Ke / (E_0 E_1); E_0 E_1 lies within [e^(-2 xi (c_0 + c_1)),
    // e^(2 xi (1 - c_0 - c_1))], normal numbers wherever the host selects
    // this path (fast_fe).
    const double zE0 = __builtin_fma(xi2, w0, -P.C2[0]), zE1 = __builtin_fma(xi2, w1, -P.C2[1]);
    const double Ex0 = TAB ? exp_tab(zE0, xt) : exp_cw(zE0);
    const double Ex1 = TAB ? exp_tab(zE1, xt) : exp_cw(zE1);
    // (E_2 enters only the third map's polynomials, so a relative error
    // of 2^-48.8 moves g_2 by at most about twice that: rcp1)
    const double Ex2 = P.Ke * rcp1(Ex0 * Ex1);
    // g_k = n_k / e_k; the normalised weights g_k / sum_l g_l over the
    // common denominator e_0 e_1 e_2 (below e^B, fe_map_poly): one reciprocal.
    double e0, e1, e2;
    const double n0 = fe_map_poly<3>(w0, Ex0, P.Pd, P.Pa, P.Pb, &e0);
    const double n1 = fe_map_poly<4>(w1, Ex1, P.Pd + 3, P.Pa + 2, P.Pb + 2, &e1);
    const double n2 = fe_map_poly<3>(w2, Ex2, P.Pd + 7, P.Pa + 5, P.Pb + 5, &e2);
    // T_k = n_k prod_{l != k} e_l: T_0 = A e_2, T_1 = B e_2, T_2 = C
    const double A = n0 * e1, B = n1 * e0, C = n2 * (e0 * e1);
    const double num = __builtin_fma(e2, __builtin_fma(A, c0, B * c1), C * c2);
    return (FAM::scale * num) * rcp1(__builtin_fma(e2, A + B, C));
  }
  if constexpr (SPEC == SPEC_FE_SAT) {
    // Z weights (p = 2) over the common denominator as above, then each map
    // term by term (tanh_sat: +-1 without an exponential once saturated).
    const double tau = __builtin_fabs(b0 - b2);
    const double t2 = tau * tau;
    const double q0 = b0 * b0, q1 = b1 * b1, q2 = b2 * b2;
    const double z0 = D0 * (q0 + t2) * (q1 * q2);
    const double z1 = D1 * (q1 + t2) * (q0 * q2);
    const double z2 = D2 * (q2 + t2) * (q0 * q1);
    const double zi = rcp(z0 + z1 + z2);
    const double g0 = fe_g0<SPEC_GENERIC>(z0 * zi, P), g1 = fe_g1<SPEC_GENERIC>(z1 * zi, P),
                 g2 = fe_g2<SPEC_GENERIC>(z2 * zi, P);
    const double ginv = rcp(g0 + g1 + g2);
    return 0.125 * ((g0 * ginv) * c0 + (g1 * ginv) * c1 + (g2 * ginv) * c2);
  }
  double a0, a1, a2;
  if (!FE && P.weights == WJS) {
    const double r0 = rcp(b0), r1 = rcp(b1), r2 = rcp(b2);
    a0 = D0 * r0 * r0;
    a1 = D1 * r1 * r1;
    a2 = D2 * r2 * r2;
  } else {
    const double tau = __builtin_fabs(b0 - b2);
    double q0 = tau * rcp(b0), q1 = tau * rcp(b1), q2 = tau * rcp(b2);
    double p0 = q0, p1 = q1, p2 = q2;
    const int zpow = FE ? 2 : P.zpow;
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
  double w0 = a0 * inv, w1 = a1 * inv, w2 = a2 * inv;

  bool map = FE || (P.weights == WFE);
  if (!FE && P.weights == WPFE) {
    const bool inside = __builtin_fabs(w0 - D0) <= P.cv && __builtin_fabs(w1 - D1) <= P.cv &&
                        __builtin_fabs(w2 - D2) <= P.cv;
    map = !inside;
  }
  if (map) {
    const double g0 = fe_g0<SPEC>(w0, P), g1 = fe_g1<SPEC>(w1, P), g2 = fe_g2<SPEC>(w2, P);
    const double ginv = rcp(g0 + g1 + g2);
    w0 = g0 * ginv;
    w1 = g1 * ginv;
    w2 = g2 * ginv;
  }
  return 0.125 * (w0 * c0 + w1 * c1 + w2 * c2);
}

// Both nonlinear interpolations (eq. 5-6) of one field at x_{m+1/2} from the
// six values u[j] = u_{m-2+j}: the left-biased one from (u_0 .. u_4) and the
// right-biased one from the mirrored stencil (u_5, u_4, u_3, u_2, u_1).
// Smoothness indicators (eq. 9-10) are written through the first differences
// of the stencil so that a sub-stencil of equal values gives IS = 0 exactly
// (with FMA contraction too): at steepness xi ~ 100 the FE map keeps a small
// weight g_0(0) on a stencil across a jump, and how that weight is
// renormalised depends on the ratio of the two flat stencils' weights, so
// flat stencils must not see rounding noise.  The mirrored stencil's first
// differences are the negated left ones (plus u_5 - u_4), so its second
// differences s'_1, s'_2 are the left s_2, s_1.
template <int SPEC = SPEC_GENERIC, bool TAB = false>
__device__ __forceinline__ void interp5_pair(const InterpParams& P, const double (&u)[6],
                                             double* left, double* right,
                                             const double* xt = nullptr) {
  constexpr bool FE = (SPEC == SPEC_FE);
  // candidates of eq. 5 (times 8) of both stencils
  const double c0 = 3.0 * u[0] - 10.0 * u[1] + 15.0 * u[2];
  const double c1 = -u[1] + 6.0 * u[2] + 3.0 * u[3];
  const double c2 = 3.0 * u[2] + 6.0 * u[3] - u[4];
  const double r0 = 3.0 * u[5] - 10.0 * u[4] + 15.0 * u[3];
  const double r1 = -u[4] + 6.0 * u[3] + 3.0 * u[2];
  const double r2 = 3.0 * u[3] + 6.0 * u[2] - u[1];
  if (!FE && P.weights == WLIN) {
    *left = 0.125 * (D0 * c0 + D1 * c1 + D2 * c2);
    *right = 0.125 * (D0 * r0 + D1 * r1 + D2 * r2);
    return;
  }
  const double d0 = u[1] - u[0], d1 = u[2] - u[1], d2 = u[3] - u[2], d3 = u[4] - u[3],
               d4 = u[5] - u[4];
  const double s0 = d1 - d0, s1 = d2 - d1, s2 = d3 - d2, s3 = d4 - d3;
  // IS_k + eps = f_k^2 + (s_k^2 + eps)
  const double q1 = __builtin_fma(s1, s1, P.eps), q2 = __builtin_fma(s2, s2, P.eps);
  const double f0 = 0.5 * (3.0 * d1 - d0), f1 = 0.5 * (d1 + d2), f2 = 0.5 * (3.0 * d2 - d3);
  const double g0 = 0.5 * (3.0 * d3 - d4), g1 = 0.5 * (d2 + d3), g2 = 0.5 * (3.0 * d2 - d1);
  *left = weigh5<SPEC, TAB>(P, c0, c1, c2, __builtin_fma(f0, f0, __builtin_fma(s0, s0, P.eps)),
                            __builtin_fma(f1, f1, q1), __builtin_fma(f2, f2, q2), xt);
  *right = weigh5<SPEC, TAB>(P, r0, r1, r2, __builtin_fma(g0, g0, __builtin_fma(s3, s3, P.eps)),
                             __builtin_fma(g1, g1, q2), __builtin_fma(g2, g2, q1), xt);
}

// ----------------------------------------- WENO5 reconstruction (App. B) --
// Ideal weights of Table B.1 and the A_j = a_j + b_j w of the three maps of
// Table B.2 (same construction as kG0a .. kG2b).
constexpr double E0 = 1.0 / 10.0, E1 = 6.0 / 10.0, E2 = 3.0 / 10.0;
constexpr double kV0a[3] = {0.5 * E0, 0.5 * (0.25 - E0), -0.5 * 0.25};
constexpr double kV0b[3] = {-0.5, 0.0, 0.5};
constexpr double kV1a[4] = {0.5 * E1, 0.5 * (0.5 - E1), 0.5 * (0.75 - 0.5), -0.5 * 0.75};
constexpr double kV1b[4] = {-0.5, 0.0, 0.0, 0.5};
constexpr double kV2a[3] = {0.5 * E2, 0.5 * (0.5 - E2), -0.25};
constexpr double kV2b[3] = {-0.5, 0.0, 0.5};
static_assert(map_sums_vanish(kV0a, kV0b, 3) && map_sums_vanish(kV1a, kV1b, 4) &&
                  map_sums_vanish(kV2a, kV2b, 3),
              "the WENO FE maps' A_j must sum to zero");

struct FamWeno {
  static constexpr double d0 = E0, d1 = E1, d2 = E2, scale = 1.0 / 6.0;
  static constexpr double dr1 = 6.0, dr2 = 3.0;  // d_1 / d_0, d_2 / d_0
  static constexpr const double (&m0a)[3] = kV0a;
  static constexpr const double (&m0b)[3] = kV0b;
  static constexpr const double (&m1a)[4] = kV1a;
  static constexpr const double (&m1b)[4] = kV1b;
  static constexpr const double (&m2a)[3] = kV2a;
  static constexpr const double (&m2b)[3] = kV2b;
};

// weno5 with FE weights on p = 2 Z weights through the fast path of weigh5
// (Table B.1 ideal weights, Table B.2 maps); xt: the kExp2Tab64 table in LDS.
template <bool TAB>
__device__ __forceinline__ double weno5_fe(const InterpParams& P, double a, double b, double c,
                                           double e, double f, const double* xt) {
  const double d0 = b - a, d1 = c - b, d2 = e - c, d3 = f - e;
  const double s20 = d1 - d0, s10 = 3.0 * d1 - d0;
  const double s21 = d2 - d1, s11 = d1 + d2;
  const double s22 = d3 - d2, s12 = 3.0 * d2 - d3;
  const double B0 = (13.0 / 12.0) * s20 * s20 + 0.25 * s10 * s10;
  const double B1 = (13.0 / 12.0) * s21 * s21 + 0.25 * s11 * s11;
  const double B2 = (13.0 / 12.0) * s22 * s22 + 0.25 * s12 * s12;
  return weigh5<SPEC_FE, TAB, FamWeno>(P, 2.0 * a - 7.0 * b + 11.0 * c, -b + 5.0 * c + 2.0 * e,
                                       2.0 * c + 5.0 * e - f, B0 + P.eps, B1 + P.eps,
                                       B2 + P.eps, xt);
}

// Finite-difference WENO5 reconstruction at x_{i+1/2} from the point values
// (f_{i-2}, ..., f_{i+2}) = (a, b, c, e, f): Jiang-Shu smoothness indicators
// (through first differences, as for the WCNS indicators), JS / Z weights
// with the ideal weights of Table B.1, the FE map of Table B.2 (P.K and P.C2
// hold its null points), PFE switch.
__device__ __forceinline__ double weno5(const InterpParams& P, double a, double b, double c,
                                        double e, double f) {
  const double q0 = (1.0 / 6.0) * (2.0 * a - 7.0 * b + 11.0 * c);
  const double q1 = (1.0 / 6.0) * (-b + 5.0 * c + 2.0 * e);
  const double q2 = (1.0 / 6.0) * (2.0 * c + 5.0 * e - f);
  if (P.weights == WLIN) return E0 * q0 + E1 * q1 + E2 * q2;
  const double d0 = b - a, d1 = c - b, d2 = e - c, d3 = f - e;
  const double s20 = d1 - d0, s10 = 3.0 * d1 - d0;
  const double s21 = d2 - d1, s11 = d1 + d2;
  const double s22 = d3 - d2, s12 = 3.0 * d2 - d3;
  const double B0 = (13.0 / 12.0) * s20 * s20 + 0.25 * s10 * s10;
  const double B1 = (13.0 / 12.0) * s21 * s21 + 0.25 * s11 * s11;
  const double B2 = (13.0 / 12.0) * s22 * s22 + 0.25 * s12 * s12;
  double a0, a1, a2;
  if (P.weights == WJS) {
    const double r0 = rcp(B0 + P.eps), r1 = rcp(B1 + P.eps), r2 = rcp(B2 + P.eps);
    a0 = E0 * r0 * r0;
    a1 = E1 * r1 * r1;
    a2 = E2 * r2 * r2;
  } else {
    const double tau = __builtin_fabs(B0 - B2);
    const double t0 = tau * rcp(B0 + P.eps), t1 = tau * rcp(B1 + P.eps), t2 = tau * rcp(B2 + P.eps);
    double p0 = t0, p1 = t1, p2 = t2;
    for (int k = 1; k < P.zpow; ++k) {
      p0 *= t0;
      p1 *= t1;
      p2 *= t2;
    }
    a0 = E0 * (1.0 + p0);
    a1 = E1 * (1.0 + p1);
    a2 = E2 * (1.0 + p2);
  }
  const double inv = rcp(a0 + a1 + a2);
  double w0 = a0 * inv, w1 = a1 * inv, w2 = a2 * inv;
  bool map = P.weights == WFE;
  if (P.weights == WPFE)
    map = !(__builtin_fabs(w0 - E0) <= P.cv && __builtin_fabs(w1 - E1) <= P.cv &&
            __builtin_fabs(w2 - E2) <= P.cv);
  if (map) {
    const double g0 = fe_map<3, SPEC_GENERIC>(w0, kV0a, kV0b, P.K, P.C2[0], P, nullptr);
    const double g1 = fe_map<4, SPEC_GENERIC>(w1, kV1a, kV1b, P.K + 3, P.C2[1], P, nullptr);
    const double g2 = fe_map<3, SPEC_GENERIC>(w2, kV2a, kV2b, P.K + 7, P.C2[2], P, nullptr);
    const double gi = rcp(g0 + g1 + g2);
    w0 = g0 * gi;
    w1 = g1 * gi;
    w2 = g2 * gi;
  }
  return w0 * q0 + w1 * q1 + w2 * q2;
}

// ------------------------------------------------------------------ Euler --
// State layout in registers: [rho, m_0 .. m_{ND-1}, E].

template <int ND>
struct Prim {
  double ir;        // 1/rho
  double vel[ND];
  double p;
};

template <int ND>
__device__ __forceinline__ Prim<ND> primitives(const double* U, double gamma) {
  Prim<ND> q;
  q.ir = rcp(U[0]);
  double mm = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    q.vel[k] = U[1 + k] * q.ir;
    mm += U[1 + k] * q.vel[k];
  }
  q.p = (gamma - 1.0) * (U[ND + 1] - 0.5 * mm);
  return q;
}

// Physical flux along DIR (eq. 32).
template <int ND, int DIR>
__device__ __forceinline__ void euler_flux(const double* U, double gamma, double* F) {
  const Prim<ND> q = primitives<ND>(U, gamma);
  const double vn = q.vel[DIR];
  F[0] = U[1 + DIR];
#pragma unroll
  for (int k = 0; k < ND; ++k) F[1 + k] = U[1 + k] * vn + (k == DIR ? q.p : 0.0);
  F[ND + 1] = (U[ND + 1] + q.p) * vn;
}

// Roe-averaged quantities that define the eigenvectors between two nodes.
template <int ND>
struct RoeState {
  double vel[ND];
  double H, c, ic, q2h, b1, b2;   // q2h = |u|^2 / 2
};

// Fills q2h, b1 and b2 of a Roe state from vel and ic, by the same operations
// as roe_average (so tiles may keep only vel, H, c and ic).
template <int ND>
__device__ __forceinline__ void roe_derived(RoeState<ND>& r, double gamma) {
  double q2 = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) q2 += r.vel[k] * r.vel[k];
  r.q2h = 0.5 * q2;
  r.b1 = (gamma - 1.0) * r.ic * r.ic;
  r.b2 = r.q2h * r.b1;
}

template <int ND>
__device__ __forceinline__ RoeState<ND> roe_average(const double* UA, const double* UB,
                                                    double gamma) {
  const Prim<ND> A = primitives<ND>(UA, gamma);
  const Prim<ND> B = primitives<ND>(UB, gamma);
  // weights sqrt(rho_A) / (sqrt(rho_A) + sqrt(rho_B)) and the same for B,
  // through s = sqrt(rho_B / rho_A)
  const double s = sqrt_pos(UB[0] * A.ir);
  const double wA = rcp(1.0 + s), wB = s * wA;
  RoeState<ND> r;
  double q2 = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    r.vel[k] = wA * A.vel[k] + wB * B.vel[k];
    q2 += r.vel[k] * r.vel[k];
  }
  const double HA = (UA[ND + 1] + A.p) * A.ir;
  const double HB = (UB[ND + 1] + B.p) * B.ir;
  r.H = wA * HA + wB * HB;
  r.q2h = 0.5 * q2;
  r.c = sqrt_pos((gamma - 1.0) * (r.H - r.q2h));
  r.ic = rcp(r.c);
  r.b1 = (gamma - 1.0) * r.ic * r.ic;
  r.b2 = r.q2h * r.b1;
  return r;
}

// Characteristic field order: 0 = (u_n - c), 1 = entropy, 2 .. ND = shear
// along the tangential axes in increasing order, ND + 1 = (u_n + c).
template <int ND, int DIR>
__device__ __forceinline__ int tangential_axis(int t) {
  // t-th axis other than DIR
  return (t < DIR) ? t : t + 1;
}

// Left eigenvectors applied to one node U: W = L U.
template <int ND, int DIR>
__device__ __forceinline__ void project(const RoeState<ND>& r, const double* U, double* W) {
  double um = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) um += r.vel[k] * U[1 + k];
  const double theta = r.b2 * U[0] - r.b1 * um + r.b1 * U[ND + 1];
  const double an = (r.vel[DIR] * U[0] - U[1 + DIR]) * r.ic;
  W[0] = 0.5 * (theta + an);
  W[1] = U[0] - theta;
#pragma unroll
  for (int t = 0; t < ND - 1; ++t) {
    const int ax = tangential_axis<ND, DIR>(t);
    W[2 + t] = U[1 + ax] - r.vel[ax] * U[0];
  }
  W[ND + 1] = 0.5 * (theta - an);
}

// Right eigenvectors applied to characteristic values: U = R W.
// Row v of the left eigenvector matrix L, for a field that is not a shear
// field (v = 0, 1 or NV-1): W_v = l . U.  Same quantity as project_field,
// written as a dot product so that a stencil costs NV operations per node.
template <int ND, int DIR>
__device__ __forceinline__ void field_row(const RoeState<ND>& r, int v, double (&l)[ND + 2]) {
  if (v == 1) {  // entropy: rho - theta
    l[0] = 1.0 - r.b2;
#pragma unroll
    for (int k = 0; k < ND; ++k) l[1 + k] = r.b1 * r.vel[k];
    l[ND + 1] = -r.b1;
    return;
  }
  // acoustic: (theta +- an) / 2, an = (vel_n rho - m_n) / c
  const double s = (v == 0) ? 0.5 : -0.5;
  const double hb1 = 0.5 * r.b1;
  l[0] = __builtin_fma(s * r.vel[DIR], r.ic, 0.5 * r.b2);
#pragma unroll
  for (int k = 0; k < ND; ++k) l[1 + k] = -hb1 * r.vel[k];
  l[1 + DIR] -= s * r.ic;
  l[ND + 1] = hb1;
}

template <int ND, int DIR>
__device__ __forceinline__ void unproject(const RoeState<ND>& r, const double* W, double* U) {
  const double sum = W[0] + W[1] + W[ND + 1];
  const double dif = W[ND + 1] - W[0];
  U[0] = sum;
  double E = r.H * (W[0] + W[ND + 1]) + r.vel[DIR] * r.c * dif + r.q2h * W[1];
#pragma unroll
  for (int k = 0; k < ND; ++k) U[1 + k] = r.vel[k] * sum;
  U[1 + DIR] += r.c * dif;
#pragma unroll
  for (int t = 0; t < ND - 1; ++t) {
    const int ax = tangential_axis<ND, DIR>(t);
    U[1 + ax] += W[2 + t];
    E += r.vel[ax] * W[2 + t];
  }
  U[ND + 1] = E;
}

// Local Lax-Friedrichs flux between the interpolated states UL and UR.
template <int ND, int DIR>
__device__ __forceinline__ void llf_flux(const double* UL, const double* UR, double gamma,
                                         double* F) {
  constexpr int NV = ND + 2;
  double FL[NV], FR[NV];
  const Prim<ND> L = primitives<ND>(UL, gamma);
  const Prim<ND> R = primitives<ND>(UR, gamma);
  const double cL = sqrt_pos(gamma * L.p * L.ir);
  const double cR = sqrt_pos(gamma * R.p * R.ir);
  const double lamL = __builtin_fabs(L.vel[DIR]) + cL;
  const double lamR = __builtin_fabs(R.vel[DIR]) + cR;
  const double alpha = __builtin_fmax(lamL, lamR);  // (the larger; a NaN only if both are)
  FL[0] = UL[1 + DIR];
  FR[0] = UR[1 + DIR];
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    FL[1 + k] = UL[1 + k] * L.vel[DIR] + (k == DIR ? L.p : 0.0);
    FR[1 + k] = UR[1 + k] * R.vel[DIR] + (k == DIR ? R.p : 0.0);
  }
  FL[ND + 1] = (UL[ND + 1] + L.p) * L.vel[DIR];
  FR[ND + 1] = (UR[ND + 1] + R.p) * R.vel[DIR];
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * alpha * (UR[v] - UL[v]);
}

// Physical flux at one node along DIR.
template <int NV, int DIR>
__device__ __forceinline__ void node_flux(const PhysParams& PP, const double (&U)[NV],
                                          double (&F)[NV]) {
  if constexpr (NV == 1) {
    F[0] = PP.adv * U[0];
  } else {
    euler_flux<NV - 2, DIR>(U, PP.gamma, F);
  }
}

// Sum over directions of (|u_d| + c) / h_d at one node (advection: the
// caller adds |a_d| / h_d).
template <int ND>
__device__ __forceinline__ double wave_rate(const double* U, double gamma, const double* ih) {
  const Prim<ND> q = primitives<ND>(U, gamma);
  const double c = sqrt_pos(gamma * q.p * q.ir);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) s += (__builtin_fabs(q.vel[k]) + c) * ih[k];
  return s;
}

// Maxima of wave rates are taken on their bit patterns as unsigned integers:
// for non-negative doubles that is the order of the values, and a NaN (of
// either sign) exceeds every finite rate, so it always reaches dt.  Maximum
// over the 64 lanes of a wavefront (all lanes active), by DPP lane moves
// (vector-ALU operations, where each step of a lane-permute exchange would
// be a round trip through the LDS crossbar): the maximum within quads, rows
// of 16 by two right shifts, then rows 0 -> 1, 2 -> 3 and the first half ->
// the second by row broadcasts, which leaves the wavefront's maximum in
// lane 63.  Lanes that a move leaves out read 0, the neutral value.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, ROWS, 0xf, true);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, ROWS, 0xf, true);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return b > a ? b : a;
}
__device__ __forceinline__ unsigned long long wave_max_bits(unsigned long long v) {
  v = umax64(v, dpp_u64<0xb1, 0xf>(v));   // quad_perm [1, 0, 3, 2]
  v = umax64(v, dpp_u64<0x4e, 0xf>(v));   // quad_perm [2, 3, 0, 1]
  v = umax64(v, dpp_u64<0x114, 0xf>(v));  // row_shr:4
  v = umax64(v, dpp_u64<0x118, 0xf>(v));  // row_shr:8
  v = umax64(v, dpp_u64<0x142, 0xa>(v));  // row_bcast:15 into rows 1 and 3
  v = umax64(v, dpp_u64<0x143, 0xc>(v));  // row_bcast:31 into rows 2 and 3
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Wave speed |u_DIR| + c of one state along DIR.
template <int ND, int DIR>
__device__ __forceinline__ double dir_speed(const double* U, double gamma) {
  const Prim<ND> q = primitives<ND>(U, gamma);
  return __builtin_fabs(q.vel[DIR]) + sqrt_pos(gamma * q.p * q.ir);
}

// True if the state is finite and (Euler) rho > 0 and p > 0.
template <int NV>
__device__ __forceinline__ bool physical(const double (&U)[NV], double gamma) {
  bool ok = true;
#pragma unroll
  for (int v = 0; v < NV; ++v) ok = ok && __builtin_isfinite(U[v]);
  if constexpr (NV > 1) {
    constexpr int ND = NV - 2;
    double mm = 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) mm += U[1 + k] * U[1 + k];
    // with rho > 0 and gamma > 1: p = (gamma - 1)(E - |m|^2 / (2 rho)) > 0
    // exactly when 2 E rho - |m|^2 > 0
    ok = ok && (U[0] > 0.0) && (__builtin_fma(2.0 * U[ND + 1], U[0], -mm) > 0.0);
  }
  return ok;
}

}  // namespace wcns
