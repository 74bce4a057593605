// Plain FP64 CPU oracle of the WCNS-FE semi-discrete residual and its SSP-RK3
// time step (Liu, Min, Cai, Ma, Yan: "A filtered embedded weighted compact
// nonlinear scheme for hyperbolic conservation law", arXiv 2306.09760).
//
// TEST INFRASTRUCTURE ONLY.  It is loaded by the test-suite, by the smoke
// check and by the CPU-baseline leg of the benchmark, never by the GPU
// product path, and it shares no source with the HIP library.
//
// It is written to be read against the paper, not to be fast: every line of
// every direction is copied into a padded line with ghost nodes, every
// midpoint flux is computed from scratch with full nv x nv eigenvector
// matrices, and every weight goes through the formulas in the paper's order.
//
// Every routine is templated on the scalar type T.  T = double gives values;
// T = Dual (forward-mode dual number) gives exact directional derivatives
// (Jacobian-vector products) of the same arithmetic, used to check the
// hand-written adjoint of the GPU path.  T = Counted tallies the arithmetic.
//
// Readings of points the paper leaves open (the GPU path takes the same):
//  * weights: JS per eq. 11 with (IS+eps)^2; Z per eq. 14-15 with integer
//    exponent p (default 2); FE = the mapping of eq. 20-21 and the coefficient
//    table of Sec. 3.1 applied to the normalised Z weights, followed by a
//    renormalisation (as eq. 12 renormalises the mapped M weights); PFE per
//    App. A with an inclusive band.
//  * the right-biased midpoint state is the same interpolation applied to
//    the mirrored stencil.
//  * characteristic projection uses Roe-averaged eigenvectors of the
//    direction-normal Euler Jacobian, frozen per midpoint.
//  * the midpoint flux is local Lax-Friedrichs (Rusanov) at the two
//    interpolated states, alpha = max(|u_n|+c) of the two states.
//  * the flux difference is the sixth-order midpoint-and-node operator
//    (3/2, -3/10, 1/30) or eq. 3's midpoint-only operator (MD6).
//  * time integration is the three-stage SSP Runge-Kutta scheme.

#include <omp.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace ora {

// ---------------------------------------------------------------- scalars --
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double sqrt_(double x) { return std::sqrt(x); }
inline Dual sqrt_(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline double tanh_(double x) { return std::tanh(x); }
inline Dual tanh_(Dual a) {
  double t = std::tanh(a.v);
  return Dual(t, a.d * (1.0 - t * t));
}
// |x| with derivative sign(x), and 0 at x = 0.
inline double abs_(double x) { return std::fabs(x); }
inline Dual abs_(Dual a) {
  if (a.v > 0.0) return a;
  if (a.v < 0.0) return -a;
  return Dual(0.0, 0.0);
}
// max with ties resolved to the first argument.
template <class T> inline T max_(T a, T b) { return (a >= b) ? a : b; }

// Operation counter: a double that tallies the arithmetic done on it.
struct OpCount {
  long long add = 0, mul = 0, div = 0, sqrt = 0, tanh = 0;
};
static OpCount g_ops;
struct Counted {
  double v;
  Counted() : v(0.0) {}
  Counted(double x) : v(x) {}
};
inline Counted operator+(Counted a, Counted b) { g_ops.add++; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { g_ops.add++; return Counted(a.v - b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline Counted operator*(Counted a, Counted b) { g_ops.mul++; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { g_ops.div++; return Counted(a.v / b.v); }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline Counted& operator*=(Counted& a, Counted b) { a = a * b; return a; }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
inline double val(Counted x) { return x.v; }
inline Counted sqrt_(Counted a) { g_ops.sqrt++; return Counted(std::sqrt(a.v)); }
inline Counted tanh_(Counted a) { g_ops.tanh++; return Counted(std::tanh(a.v)); }
inline Counted abs_(Counted a) { return Counted(std::fabs(a.v)); }

// Whether the lines of a residual may run on several threads: not for the
// counting scalar, whose tally is one global.
template <class T> constexpr bool kThreaded = true;
template <> constexpr bool kThreaded<Counted> = false;

// ------------------------------------------------------------- descriptor --
// The oracle's own problem descriptor (filled by oracle/oracle.py).
struct Desc {
  int64_t n[3];     // nodes per axis (unused axes = 1)
  double h[3];      // grid spacing per axis
  double adv[3];    // advection speed per axis (scalar advection only)
  double gamma;     // ratio of specific heats (Euler only)
  double eps;       // epsilon of eq. 11 / eq. 14
  double xi;        // steepness parameter of eq. 20
  double kappa;     // null-point parameter of eq. 20
  double cv;        // PFE switch value (App. A)
  int32_t system;   // 0 = scalar advection, 1 = Euler
  int32_t ndim;     // 1, 2 or 3
  int32_t bc[3];    // per axis: 0 = periodic, 1 = transmissive
  int32_t weights;  // 0 JS, 1 Z, 2 FE, 3 PFE, 4 linear (ideal weights)
  int32_t zpow;     // exponent p of eq. 14
  int32_t diff;     // 0 = MND6, 1 = MD6 (eq. 3)
  int32_t charproj; // 1 = characteristic projection, 0 = component-wise
  int32_t family;   // 0 = WCNS (interpolation + LLF + MND6/MD6),
                    // 1 = finite-difference WENO5 of App. B (flux splitting)
};

enum { W_JS = 0, W_Z = 1, W_FE = 2, W_PFE = 3, W_LINEAR = 4 };
enum { DIFF_MND6 = 0, DIFF_MD6 = 1 };
enum { FAMILY_WCNS = 0, FAMILY_WENO = 1 };

inline int nvars(const Desc& D) { return D.system == 0 ? 1 : D.ndim + 2; }
inline int64_t npoints(const Desc& D) { return D.n[0] * D.n[1] * D.n[2]; }
inline int ghosts(const Desc& D) { return D.diff == DIFF_MD6 ? 5 : 4; }

// ----------------------------------------------- ideal weights (Sec. 2) ----
static const double d_ideal[3] = {1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0};

// ------------------------------------------- FE mapping (eq. 20, eq. 21) ----
// Coefficient table of Sec. 3.1: omega_{i,j} and psi_{i,j}.  An entry marked
// "self" stands for the weight omega_i being mapped.  i = 0 and i = 2 use
// j = 0..3, i = 1 uses j = 0..4.
struct MapRow {
  int J;                 // last j of the row
  bool self[5];          // omega_{i,j} is the argument itself
  double omega[5];       // constant omega_{i,j} otherwise
  double psi[5];
};
static const MapRow map_table[3] = {
    {3, {true, false, false, true, false},
     {0.0, 1.0 / 16.0, 1.0 / 6.0, 0.0, 0.0},
     {0.0, 1.0 / 16.0, 1.0 / 11.0, 1.0, 0.0}},
    {4, {true, false, false, false, true},
     {0.0, 10.0 / 16.0, 1.0 / 2.0, 5.0 / 6.0, 0.0},
     {0.0, 10.0 / 16.0, 2.0 / 3.0, 10.0 / 11.0, 1.0}},
    {3, {true, false, false, true, false},
     {0.0, 5.0 / 16.0, 1.0 / 2.0, 0.0, 0.0},
     {0.0, 5.0 / 16.0, 1.0 / 3.0, 1.0, 0.0}},
};
// Table B.2 (App. B): the same construction for the embedded fifth-order WENO
// scheme, whose ideal weights are (1/10, 6/10, 3/10) (Table B.1).
static const MapRow map_table_weno[3] = {
    {3, {true, false, false, true, false},
     {0.0, 1.0 / 10.0, 1.0 / 4.0, 0.0, 0.0},
     {0.0, 1.0 / 10.0, 1.0 / 7.0, 1.0, 0.0}},
    {4, {true, false, false, false, true},
     {0.0, 6.0 / 10.0, 1.0 / 2.0, 3.0 / 4.0, 0.0},
     {0.0, 6.0 / 10.0, 2.0 / 3.0, 6.0 / 7.0, 1.0}},
    {3, {true, false, false, true, false},
     {0.0, 3.0 / 10.0, 1.0 / 2.0, 0.0, 0.0},
     {0.0, 3.0 / 10.0, 1.0 / 3.0, 1.0, 0.0}},
};
static const double d_ideal_weno[3] = {1.0 / 10.0, 6.0 / 10.0, 3.0 / 10.0};

// Sign table phi(i,j) of eq. 21.
inline double phi(int i, int j) {
  if ((i == 0 && j == 3) || (i == 2 && j == 3) || (i == 1 && j == 4)) return -1.0;
  return 1.0;
}

// g_i(omega) of eq. 20 with the coefficient table of Sec. 3.1 (family 0) or
// Table B.2 (family 1).
template <class T>
T fe_map(int i, T w, double xi, double kappa, int family = FAMILY_WCNS) {
  const MapRow& row = family == FAMILY_WENO ? map_table_weno[i] : map_table[i];
  T g = w;
  for (int j = 1; j <= row.J; ++j) {
    T wj = row.self[j] ? w : T(row.omega[j]);
    T wjm1 = row.self[j - 1] ? w : T(row.omega[j - 1]);
    double ph = phi(i, j);
    double null_point = kappa * (row.psi[j] + row.psi[j - 1]);
    g = g + T(ph) * (wj - wjm1) / T(2.0) * tanh_(T(xi * ph) * (w - T(null_point)));
  }
  return g;
}

// -------------------------------- nonlinear interpolation (eq. 5 - eq. 15) --
// Interpolates to x_{i+1/2} from the five-point stencil u = (u_{i-2}, ...,
// u_{i+2}).  w_base receives the normalised JS/Z weights, w_out the weights
// actually used.
template <class T>
T interpolate(const Desc& D, const T u[5], T* w_base = nullptr, T* w_out = nullptr) {
  // Smoothness indicators, eq. 9-10 (the powers of h cancel).  The one-sided
  // first and second differences of eq. 10 are evaluated through the first
  // differences du_j = u_{j+1} - u_j of the stencil, e.g.
  //   u_{i-2} - 4u_{i-1} + 3u_i = 3 du_{i-1} - du_{i-2},
  // which is the same polynomial in u but makes a sub-stencil of equal values
  // give IS = 0 exactly, whatever the rounding of the products.
  T du[4];
  for (int j = 0; j < 4; ++j) du[j] = u[j + 1] - u[j];
  T hf[3], hs[3], IS[3];
  hf[0] = T(0.5) * (T(3.0) * du[1] - du[0]);   // (u_{i-2} - 4u_{i-1} + 3u_i) / 2
  hs[0] = du[1] - du[0];                       //  u_{i-2} - 2u_{i-1} + u_i
  hf[1] = T(0.5) * (du[1] + du[2]);            // (u_{i+1} - u_{i-1}) / 2
  hs[1] = du[2] - du[1];                       //  u_{i-1} - 2u_i + u_{i+1}
  hf[2] = T(0.5) * (T(3.0) * du[2] - du[3]);   // (-3u_i + 4u_{i+1} - u_{i+2}) / 2
  hs[2] = du[3] - du[2];                       //  u_i - 2u_{i+1} + u_{i+2}
  for (int k = 0; k < 3; ++k) IS[k] = hf[k] * hf[k] + hs[k] * hs[k];

  T w[3];
  if (D.weights == W_LINEAR) {
    for (int k = 0; k < 3; ++k) w[k] = T(d_ideal[k]);
  } else if (D.weights == W_JS) {
    // eq. 11
    T alpha[3], sum = T(0.0);
    for (int k = 0; k < 3; ++k) {
      T den = IS[k] + T(D.eps);
      alpha[k] = T(d_ideal[k]) / (den * den);
      sum = sum + alpha[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = alpha[k] / sum;
  } else {
    // eq. 14-15
    T tau = abs_(IS[0] - IS[2]);
    T alpha[3], sum = T(0.0);
    for (int k = 0; k < 3; ++k) {
      T ratio = tau / (IS[k] + T(D.eps));
      T powr = T(1.0);
      for (int q = 0; q < D.zpow; ++q) powr = powr * ratio;
      alpha[k] = T(d_ideal[k]) * (T(1.0) + powr);
      sum = sum + alpha[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = alpha[k] / sum;
  }
  if (w_base)
    for (int k = 0; k < 3; ++k) w_base[k] = w[k];

  bool map = (D.weights == W_FE);
  if (D.weights == W_PFE) {
    // App. A: keep the Z weights when all three lie in [d_k - c_v, d_k + c_v].
    bool inside = true;
    for (int k = 0; k < 3; ++k)
      if (!(val(w[k]) >= d_ideal[k] - D.cv && val(w[k]) <= d_ideal[k] + D.cv)) inside = false;
    map = !inside;
  }
  if (map) {
    T g[3], sum = T(0.0);
    for (int k = 0; k < 3; ++k) {
      g[k] = fe_map(k, w[k], D.xi, D.kappa);
      sum = sum + g[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = g[k] / sum;
  }
  if (w_out)
    for (int k = 0; k < 3; ++k) w_out[k] = w[k];

  // Candidate interpolations, eq. 5.
  T c0 = (T(3.0) * u[0] - T(10.0) * u[1] + T(15.0) * u[2]) / T(8.0);
  T c1 = (T(-1.0) * u[1] + T(6.0) * u[2] + T(3.0) * u[3]) / T(8.0);
  T c2 = (T(3.0) * u[2] + T(6.0) * u[3] - u[4]) / T(8.0);
  // eq. 6
  return w[0] * c0 + w[1] * c1 + w[2] * c2;
}

// ------------------------------------------------------------ Euler (eq. 32)
// Conservative variables U = (rho, rho u_1..rho u_nd, E).
template <class T>
void euler_flux(int nd, int d, double gamma, const T* U, T* F) {
  T rho = U[0];
  T vel[3], q2 = T(0.0);
  for (int k = 0; k < nd; ++k) {
    vel[k] = U[1 + k] / rho;
    q2 = q2 + vel[k] * vel[k];
  }
  T E = U[nd + 1];
  T p = T(gamma - 1.0) * (E - T(0.5) * rho * q2);
  F[0] = U[1 + d];
  for (int k = 0; k < nd; ++k) F[1 + k] = U[1 + k] * vel[d] + (k == d ? p : T(0.0));
  F[nd + 1] = (E + p) * vel[d];
}

// |u_d| + c of one state.
template <class T>
T euler_speed(int nd, int d, double gamma, const T* U) {
  T rho = U[0];
  T q2 = T(0.0);
  for (int k = 0; k < nd; ++k) q2 = q2 + (U[1 + k] / rho) * (U[1 + k] / rho);
  T p = T(gamma - 1.0) * (U[nd + 1] - T(0.5) * rho * q2);
  T c = sqrt_(T(gamma) * p / rho);
  return abs_(U[1 + d] / rho) + c;
}

// Roe-averaged left (Lm, rows) and right (Rm, columns) eigenvectors of the
// direction-d flux Jacobian, between states Ua and Ub.  Field order:
// u_d - c, entropy, shear (tangential axes in increasing order), u_d + c.
template <class T>
void euler_eigenvectors(int nd, int d, double gamma, const T* Ua, const T* Ub, T Lm[5][5],
                        T Rm[5][5]) {
  const int nv = nd + 2;
  T ra = sqrt_(Ua[0]), rb = sqrt_(Ub[0]);
  T pa, pb;
  {
    T q2a = T(0.0), q2b = T(0.0);
    for (int k = 0; k < nd; ++k) {
      q2a = q2a + Ua[1 + k] * Ua[1 + k] / (Ua[0] * Ua[0]);
      q2b = q2b + Ub[1 + k] * Ub[1 + k] / (Ub[0] * Ub[0]);
    }
    pa = T(gamma - 1.0) * (Ua[nd + 1] - T(0.5) * Ua[0] * q2a);
    pb = T(gamma - 1.0) * (Ub[nd + 1] - T(0.5) * Ub[0] * q2b);
  }
  T u[3], q2 = T(0.0);
  for (int k = 0; k < nd; ++k) {
    u[k] = (ra * (Ua[1 + k] / Ua[0]) + rb * (Ub[1 + k] / Ub[0])) / (ra + rb);
    q2 = q2 + u[k] * u[k];
  }
  T Ha = (Ua[nd + 1] + pa) / Ua[0];
  T Hb = (Ub[nd + 1] + pb) / Ub[0];
  T H = (ra * Ha + rb * Hb) / (ra + rb);
  T c = sqrt_(T(gamma - 1.0) * (H - T(0.5) * q2));
  T b1 = T(gamma - 1.0) / (c * c);
  T b2 = T(0.5) * q2 * b1;

  for (int r = 0; r < 5; ++r)
    for (int s = 0; s < 5; ++s) {
      Lm[r][s] = T(0.0);
      Rm[r][s] = T(0.0);
    }
  // Tangential axes in increasing order.
  int tang[2], nt = 0;
  for (int k = 0; k < nd; ++k)
    if (k != d) tang[nt++] = k;

  // Right eigenvectors (columns).
  Rm[0][0] = T(1.0);
  Rm[0][1] = T(1.0);
  Rm[0][nv - 1] = T(1.0);
  for (int k = 0; k < nd; ++k) {
    Rm[1 + k][0] = u[k] - (k == d ? c : T(0.0));
    Rm[1 + k][1] = u[k];
    Rm[1 + k][nv - 1] = u[k] + (k == d ? c : T(0.0));
  }
  Rm[nd + 1][0] = H - u[d] * c;
  Rm[nd + 1][1] = T(0.5) * q2;
  Rm[nd + 1][nv - 1] = H + u[d] * c;
  for (int t = 0; t < nt; ++t) {
    Rm[1 + tang[t]][2 + t] = T(1.0);
    Rm[nd + 1][2 + t] = u[tang[t]];
  }
  // Left eigenvectors (rows).
  Lm[0][0] = T(0.5) * (b2 + u[d] / c);
  Lm[1][0] = T(1.0) - b2;
  Lm[nv - 1][0] = T(0.5) * (b2 - u[d] / c);
  for (int k = 0; k < nd; ++k) {
    T dk = (k == d) ? T(1.0) / c : T(0.0);
    Lm[0][1 + k] = T(0.5) * (T(-1.0) * b1 * u[k] - dk);
    Lm[1][1 + k] = b1 * u[k];
    Lm[nv - 1][1 + k] = T(0.5) * (T(-1.0) * b1 * u[k] + dk);
  }
  Lm[0][nd + 1] = T(0.5) * b1;
  Lm[1][nd + 1] = T(-1.0) * b1;
  Lm[nv - 1][nd + 1] = T(0.5) * b1;
  for (int t = 0; t < nt; ++t) {
    Lm[2 + t][0] = T(-1.0) * u[tang[t]];
    Lm[2 + t][1 + tang[t]] = T(1.0);
  }
}

// ------------------------- WENO5 reconstruction (App. B, Jiang and Shu) --
// Reconstructs the split flux at x_{i+1/2} from its point values f =
// (f_{i-2}, ..., f_{i+2}): candidates of the three sub-stencils, Jiang-Shu
// smoothness indicators, JS / Z weights with the ideal weights of Table B.1,
// the FE mapping with Table B.2, PFE switch.  As for the WCNS indicators, the
// one-sided differences are taken through the first differences of f.
template <class T>
T reconstruct_weno(const Desc& D, const T f[5], T* w_base = nullptr, T* w_out = nullptr) {
  T df[4];
  for (int j = 0; j < 4; ++j) df[j] = f[j + 1] - f[j];
  // second differences and one-sided first differences of each sub-stencil
  T s2[3], s1[3], beta[3];
  s2[0] = df[1] - df[0];                      // f_{i-2} - 2f_{i-1} + f_i
  s1[0] = T(3.0) * df[1] - df[0];             // f_{i-2} - 4f_{i-1} + 3f_i
  s2[1] = df[2] - df[1];                      // f_{i-1} - 2f_i + f_{i+1}
  s1[1] = df[1] + df[2];                      // f_{i+1} - f_{i-1}
  s2[2] = df[3] - df[2];                      // f_i - 2f_{i+1} + f_{i+2}
  s1[2] = T(3.0) * df[2] - df[3];             // -3f_i + 4f_{i+1} - f_{i+2}
  for (int k = 0; k < 3; ++k)
    beta[k] = T(13.0 / 12.0) * s2[k] * s2[k] + T(0.25) * s1[k] * s1[k];
  T w[3];
  if (D.weights == W_LINEAR) {
    for (int k = 0; k < 3; ++k) w[k] = T(d_ideal_weno[k]);
  } else if (D.weights == W_JS) {
    T alpha[3], sum = T(0.0);
    for (int k = 0; k < 3; ++k) {
      T den = beta[k] + T(D.eps);
      alpha[k] = T(d_ideal_weno[k]) / (den * den);
      sum = sum + alpha[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = alpha[k] / sum;
  } else {
    T tau = abs_(beta[0] - beta[2]);
    T alpha[3], sum = T(0.0);
    for (int k = 0; k < 3; ++k) {
      T ratio = tau / (beta[k] + T(D.eps));
      T powr = T(1.0);
      for (int q = 0; q < D.zpow; ++q) powr = powr * ratio;
      alpha[k] = T(d_ideal_weno[k]) * (T(1.0) + powr);
      sum = sum + alpha[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = alpha[k] / sum;
  }
  if (w_base)
    for (int k = 0; k < 3; ++k) w_base[k] = w[k];
  bool map = (D.weights == W_FE);
  if (D.weights == W_PFE) {
    bool inside = true;
    for (int k = 0; k < 3; ++k)
      if (!(val(w[k]) >= d_ideal_weno[k] - D.cv && val(w[k]) <= d_ideal_weno[k] + D.cv)) inside = false;
    map = !inside;
  }
  if (map) {
    T g[3], sum = T(0.0);
    for (int k = 0; k < 3; ++k) {
      g[k] = fe_map(k, w[k], D.xi, D.kappa, FAMILY_WENO);
      sum = sum + g[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = g[k] / sum;
  }
  if (w_out)
    for (int k = 0; k < 3; ++k) w_out[k] = w[k];
  T q0 = (T(2.0) * f[0] - T(7.0) * f[1] + T(11.0) * f[2]) / T(6.0);
  T q1 = (T(-1.0) * f[1] + T(5.0) * f[2] + T(2.0) * f[3]) / T(6.0);
  T q2 = (T(2.0) * f[2] + T(5.0) * f[3] - f[4]) / T(6.0);
  return w[0] * q0 + w[1] * q1 + w[2] * q2;
}

// ------------------------------------------------------- midpoint flux -----
// Numerical flux at the midpoint between nodes m and m+1 of a line in
// direction d.  st[k] points to the nv values of node m-2+k, k = 0..5.
template <class T>
void midpoint_flux(const Desc& D, int d, const T* const st[6], T* Fhat) {
  const int nd = D.ndim;
  const int nv = nvars(D);
  if (D.system == 0) {
    // Scalar advection u_t + a u_x = 0.
    T uL, uR;
    {
      T s[5] = {st[0][0], st[1][0], st[2][0], st[3][0], st[4][0]};
      uL = interpolate(D, s);
      T r[5] = {st[5][0], st[4][0], st[3][0], st[2][0], st[1][0]};
      uR = interpolate(D, r);
    }
    double a = D.adv[d];
    // Local Lax-Friedrichs with alpha = |a|.
    Fhat[0] = T(0.5) * (T(a) * uL + T(a) * uR) - T(0.5 * std::fabs(a)) * (uR - uL);
    return;
  }
  T Lm[5][5], Rm[5][5];
  if (D.charproj) {
    euler_eigenvectors(nd, d, D.gamma, st[2], st[3], Lm, Rm);
  } else {
    for (int r = 0; r < 5; ++r)
      for (int s = 0; s < 5; ++s) {
        Lm[r][s] = T(r == s ? 1.0 : 0.0);
        Rm[r][s] = T(r == s ? 1.0 : 0.0);
      }
  }
  // Project the six nodes: W_j = L U_j.
  T W[6][5];
  for (int j = 0; j < 6; ++j)
    for (int r = 0; r < nv; ++r) {
      T acc = T(0.0);
      for (int s = 0; s < nv; ++s) acc = acc + Lm[r][s] * st[j][s];
      W[j][r] = acc;
    }
  // Interpolate each characteristic field from the left and (mirrored) right.
  T WL[5], WR[5];
  for (int r = 0; r < nv; ++r) {
    T s[5] = {W[0][r], W[1][r], W[2][r], W[3][r], W[4][r]};
    WL[r] = interpolate(D, s);
    T m[5] = {W[5][r], W[4][r], W[3][r], W[2][r], W[1][r]};
    WR[r] = interpolate(D, m);
  }
  // Back to conservative variables.
  T UL[5], UR[5];
  for (int r = 0; r < nv; ++r) {
    T aL = T(0.0), aR = T(0.0);
    for (int s = 0; s < nv; ++s) {
      aL = aL + Rm[r][s] * WL[s];
      aR = aR + Rm[r][s] * WR[s];
    }
    UL[r] = aL;
    UR[r] = aR;
  }
  // Local Lax-Friedrichs flux at the midpoint.
  T FL[5], FR[5];
  euler_flux(nd, d, D.gamma, UL, FL);
  euler_flux(nd, d, D.gamma, UR, FR);
  T alpha = max_(euler_speed(nd, d, D.gamma, UL), euler_speed(nd, d, D.gamma, UR));
  for (int r = 0; r < nv; ++r)
    Fhat[r] = T(0.5) * (FL[r] + FR[r]) - T(0.5) * alpha * (UR[r] - UL[r]);
}

// Numerical flux of the finite-difference WENO scheme (App. B) at the
// midpoint between nodes m and m+1: Lax-Friedrichs splitting f+- = (F(U) +-
// alpha U)/2 with alpha the largest wave speed over the six stencil nodes
// (|c| for advection), characteristic projection with the Roe eigenvectors of
// nodes m, m+1, f+ reconstructed from the left-biased stencil and f- from the
// mirrored one, F = R (f+ + f-).
template <class T>
void midpoint_flux_weno(const Desc& D, int d, const T* const st[6], T* Fhat) {
  const int nd = D.ndim;
  const int nv = nvars(D);
  if (D.system == 0) {
    const double a = D.adv[d];
    T fp[5], fm[5];
    for (int k = 0; k < 5; ++k) {
      fp[k] = T(0.5 * (a + std::fabs(a))) * st[k][0];
      fm[k] = T(0.5 * (a - std::fabs(a))) * st[5 - k][0];
    }
    Fhat[0] = reconstruct_weno(D, fp) + reconstruct_weno(D, fm);
    return;
  }
  T alpha = T(0.0);
  for (int j = 0; j < 6; ++j) alpha = max_(alpha, euler_speed(nd, d, D.gamma, st[j]));
  T Lm[5][5], Rm[5][5];
  if (D.charproj) {
    euler_eigenvectors(nd, d, D.gamma, st[2], st[3], Lm, Rm);
  } else {
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) {
        Lm[r][c] = T(r == c ? 1.0 : 0.0);
        Rm[r][c] = T(r == c ? 1.0 : 0.0);
      }
  }
  T P[6][5], M[6][5];  // projected f+ and f- at the six nodes
  for (int j = 0; j < 6; ++j) {
    T F[5];
    euler_flux(nd, d, D.gamma, st[j], F);
    for (int r = 0; r < nv; ++r) {
      T ap = T(0.0), am = T(0.0);
      for (int c = 0; c < nv; ++c) {
        ap = ap + Lm[r][c] * (F[c] + alpha * st[j][c]);
        am = am + Lm[r][c] * (F[c] - alpha * st[j][c]);
      }
      P[j][r] = T(0.5) * ap;
      M[j][r] = T(0.5) * am;
    }
  }
  T G[5];
  for (int r = 0; r < nv; ++r) {
    T fp[5] = {P[0][r], P[1][r], P[2][r], P[3][r], P[4][r]};
    T fm[5] = {M[5][r], M[4][r], M[3][r], M[2][r], M[1][r]};
    G[r] = reconstruct_weno(D, fp) + reconstruct_weno(D, fm);
  }
  for (int r = 0; r < nv; ++r) {
    T acc = T(0.0);
    for (int c = 0; c < nv; ++c) acc = acc + Rm[r][c] * G[c];
    Fhat[r] = acc;
  }
}

// Physical flux at a node.
template <class T>
void node_flux(const Desc& D, int d, const T* U, T* F) {
  if (D.system == 0) {
    F[0] = T(D.adv[d]) * U[0];
    return;
  }
  euler_flux(D.ndim, d, D.gamma, U, F);
}

// ------------------------------------------------------ residual L(U) ------
// R = -sum_d dF_d/dx_d at every node (eq. 2), one line at a time.  The state
// U is stored variable-major: U[v*npts + x + n0*(y + n1*z)].
template <class T>
void residual(const Desc& D, const T* U, T* R) {
  const int nv = nvars(D);
  const int64_t np = npoints(D);
  const int G = ghosts(D);
  for (int64_t i = 0; i < nv * np; ++i) R[i] = T(0.0);

  for (int d = 0; d < D.ndim; ++d) {
    const int64_t N = D.n[d];
    const int64_t stride = (d == 0) ? 1 : (d == 1) ? D.n[0] : D.n[0] * D.n[1];
    // The two axes other than d.
    int a1 = (d == 0) ? 1 : 0;
    int a2 = (d == 2) ? 1 : 2;
    const int64_t s1 = (a1 == 0) ? 1 : (a1 == 1) ? D.n[0] : D.n[0] * D.n[1];
    const int64_t s2 = (a2 == 0) ? 1 : (a2 == 1) ? D.n[0] : D.n[0] * D.n[1];
    const double h = D.h[d];

    // The lines of one direction are independent (each writes only its own
    // nodes of R), so they may be shared among threads: every line is
    // computed by the same arithmetic whichever thread takes it.
    const int64_t nlines = D.n[a1] * D.n[a2];
#pragma omp parallel if (kThreaded<T> && nlines > 1)
    {
    // Padded line: node j (j = -G .. N-1+G) at line[(j+G)*nv + v].
    std::vector<T> line((N + 2 * G) * nv);
    // Midpoint j+1/2 stored at fhat[(j+G)*nv + v] for j = -G+2 .. N+G-4.
    std::vector<T> fhat((N + 2 * G) * nv);
    std::vector<T> fnode((N + 2 * G) * nv);

#pragma omp for schedule(static)
    for (int64_t li = 0; li < nlines; ++li) {
      {
        const int64_t i1 = li % D.n[a1], i2 = li / D.n[a1];
        const int64_t base = i1 * s1 + i2 * s2;
        // Ghost nodes: periodic wrap or transmissive (zeroth-order) copy.
        for (int64_t j = -G; j < N + G; ++j) {
          int64_t src;
          if (D.bc[d] == 0)
            src = ((j % N) + N) % N;
          else
            src = (j < 0) ? 0 : (j >= N ? N - 1 : j);
          for (int v = 0; v < nv; ++v) line[(j + G) * nv + v] = U[v * np + base + src * stride];
        }
        // Midpoint fluxes.
        const int64_t mlo = -G + 2, mhi = N + G - 4;
        for (int64_t m = mlo; m <= mhi; ++m) {
          const T* st[6];
          for (int k = 0; k < 6; ++k) st[k] = &line[(m - 2 + k + G) * nv];
          if (D.family == FAMILY_WENO)
            midpoint_flux_weno(D, d, st, &fhat[(m + G) * nv]);
          else
            midpoint_flux(D, d, st, &fhat[(m + G) * nv]);
        }
        // Node fluxes (needed by MND6 at i-1 .. i+1).
        for (int64_t j = -1; j <= N; ++j) node_flux(D, d, &line[(j + G) * nv], &fnode[(j + G) * nv]);
        // Flux difference.
        for (int64_t i = 0; i < N; ++i)
          for (int v = 0; v < nv; ++v) {
            auto FH = [&](int64_t m) { return fhat[(m + G) * nv + v]; };  // F~_{m+1/2}
            auto FN = [&](int64_t j) { return fnode[(j + G) * nv + v]; };
            T dfdx;
            if (D.family == FAMILY_WENO) {
              // conservative finite difference of the WENO flux
              dfdx = (FH(i) - FH(i - 1)) / T(h);
            } else if (D.diff == DIFF_MD6) {
              // eq. 3
              dfdx = (T(75.0 / 64.0) * (FH(i) - FH(i - 1)) + T(-25.0 / 384.0) * (FH(i + 1) - FH(i - 2)) +
                      T(3.0 / 640.0) * (FH(i + 2) - FH(i - 3))) /
                     T(h);
            } else {
              // Sixth-order midpoint-and-node difference.
              dfdx = (T(1.5) * (FH(i) - FH(i - 1)) - T(0.3) * (FN(i + 1) - FN(i - 1)) +
                      T(1.0 / 30.0) * (FH(i + 1) - FH(i - 2))) /
                     T(h);
            }
            R[v * np + base + i * stride] = R[v * np + base + i * stride] - dfdx;
          }
      }
    }
    }  // omp parallel
  }
}

// ------------------------------------------------- weight statistics -------
// Every interpolation one residual evaluation performs (App. A statistics):
// for each direction, line, distinct midpoint (periodic: N per line;
// transmissive: the N + 2G - 5 the difference reads), field and side (left,
// then mirrored right), nine values: the normalised JS/Z weights, their FE
// images g_k(omega_k) / sum_l g_l(omega_l), and the weights the configured
// scheme uses.  Returns the number of interpolations written (at most cap).
inline int64_t interpolation_weights(const Desc& D, const double* U, double* out, int64_t cap) {
  if (D.family != FAMILY_WCNS) return -1;  // statistics of the WCNS interpolation only
  const int nv = nvars(D);
  const int64_t np = npoints(D);
  const int G = ghosts(D);
  int64_t count = 0;
  for (int d = 0; d < D.ndim; ++d) {
    const int64_t N = D.n[d];
    const int64_t stride = (d == 0) ? 1 : (d == 1) ? D.n[0] : D.n[0] * D.n[1];
    int a1 = (d == 0) ? 1 : 0;
    int a2 = (d == 2) ? 1 : 2;
    const int64_t s1 = (a1 == 0) ? 1 : (a1 == 1) ? D.n[0] : D.n[0] * D.n[1];
    const int64_t s2 = (a2 == 0) ? 1 : (a2 == 1) ? D.n[0] : D.n[0] * D.n[1];
    std::vector<double> line((N + 2 * G) * nv);
    for (int64_t i2 = 0; i2 < D.n[a2]; ++i2)
      for (int64_t i1 = 0; i1 < D.n[a1]; ++i1) {
        const int64_t base = i1 * s1 + i2 * s2;
        for (int64_t j = -G; j < N + G; ++j) {
          int64_t src = (D.bc[d] == 0) ? ((j % N) + N) % N : ((j < 0) ? 0 : (j >= N ? N - 1 : j));
          for (int v = 0; v < nv; ++v) line[(j + G) * nv + v] = U[v * np + base + src * stride];
        }
        const int64_t mlo = (D.bc[d] == 0) ? 0 : -G + 2;
        const int64_t mhi = (D.bc[d] == 0) ? N - 1 : N + G - 4;
        for (int64_t m = mlo; m <= mhi; ++m) {
          const double* st[6];
          for (int k = 0; k < 6; ++k) st[k] = &line[(m - 2 + k + G) * nv];
          double W[6][5];
          if (D.system == 1 && D.charproj) {
            double Lm[5][5], Rm[5][5];
            euler_eigenvectors(D.ndim, d, D.gamma, st[2], st[3], Lm, Rm);
            for (int j = 0; j < 6; ++j)
              for (int r = 0; r < nv; ++r) {
                double acc = 0.0;
                for (int c = 0; c < nv; ++c) acc = acc + Lm[r][c] * st[j][c];
                W[j][r] = acc;
              }
          } else {
            for (int j = 0; j < 6; ++j)
              for (int r = 0; r < nv; ++r) W[j][r] = st[j][r];
          }
          for (int r = 0; r < nv; ++r)
            for (int side = 0; side < 2; ++side) {
              double sten[5];
              for (int k = 0; k < 5; ++k) sten[k] = side == 0 ? W[k][r] : W[5 - k][r];
              double wb[3], wo[3], g[3], gs = 0.0;
              interpolate(D, sten, wb, wo);
              for (int k = 0; k < 3; ++k) {
                g[k] = fe_map(k, wb[k], D.xi, D.kappa);
                gs = gs + g[k];
              }
              if (count < cap) {
                double* o = out + 9 * count;
                for (int k = 0; k < 3; ++k) {
                  o[k] = wb[k];
                  o[3 + k] = g[k] / gs;
                  o[6 + k] = wo[k];
                }
              }
              ++count;
            }
        }
      }
  }
  return count;
}

// -------------------------------------------------------------- time step --
// Largest stable step dt = CFL / max_i sum_d (|u_d| + c) / h_d.
inline double cfl_dt(const Desc& D, const double* U, double cfl) {
  const int64_t np = npoints(D);
  double smax = 0.0;
  for (int64_t i = 0; i < np; ++i) {
    double s = 0.0;
    if (D.system == 0) {
      for (int d = 0; d < D.ndim; ++d) s += std::fabs(D.adv[d]) / D.h[d];
    } else {
      double st[5];
      for (int v = 0; v < D.ndim + 2; ++v) st[v] = U[v * np + i];
      for (int d = 0; d < D.ndim; ++d) s += euler_speed(D.ndim, d, D.gamma, st) / D.h[d];
    }
    if (s > smax) smax = s;
  }
  return cfl / smax;
}

// 0 if every value is finite and (Euler) rho > 0 and p > 0, else 1.
template <class T>
int check_state(const Desc& D, const T* U) {
  const int nv = nvars(D);
  const int64_t np = npoints(D);
  for (int64_t i = 0; i < nv * np; ++i)
    if (!std::isfinite(val(U[i]))) return 1;
  if (D.system == 1)
    for (int64_t i = 0; i < np; ++i) {
      double rho = val(U[i]);
      double q2 = 0.0;
      for (int k = 0; k < D.ndim; ++k) q2 += val(U[(1 + k) * np + i]) * val(U[(1 + k) * np + i]);
      double p = (D.gamma - 1.0) * (val(U[(D.ndim + 1) * np + i]) - 0.5 * q2 / rho);
      if (!(rho > 0.0) || !(p > 0.0)) return 1;
    }
  return 0;
}

// One SSP-RK3 step of size dt, in place.  Returns the state check of the
// three stage results (0 = all physical).
template <class T>
int rk3_step(const Desc& D, T* U, double dt) {
  const int64_t len = nvars(D) * npoints(D);
  std::vector<T> U1(len), U2(len), L(len);
  int bad = 0;
  residual(D, U, L.data());
  for (int64_t i = 0; i < len; ++i) U1[i] = U[i] + T(dt) * L[i];
  bad |= check_state(D, U1.data());
  residual(D, U1.data(), L.data());
  for (int64_t i = 0; i < len; ++i) U2[i] = T(0.75) * U[i] + T(0.25) * (U1[i] + T(dt) * L[i]);
  bad |= check_state(D, U2.data());
  residual(D, U2.data(), L.data());
  for (int64_t i = 0; i < len; ++i) U[i] = T(1.0 / 3.0) * U[i] + T(2.0 / 3.0) * (U2[i] + T(dt) * L[i]);
  bad |= check_state(D, U);
  return bad;
}

// One step of the four-stage Runge-Kutta scheme of eq. 16, in place:
//   u1 = u + dt/2 L(u),  u2 = u + dt/2 L(u1),  u3 = u + dt L(u2),
//   u_new = -u/3 + u1/3 + 2 u2/3 + u3/3 + dt/6 L(u3).
// Returns the state check of the four stage results (0 = all physical).
template <class T>
int rk4_step(const Desc& D, T* U, double dt) {
  const int64_t len = nvars(D) * npoints(D);
  std::vector<T> U1(len), U2(len), U3(len), L(len);
  int bad = 0;
  residual(D, U, L.data());
  for (int64_t i = 0; i < len; ++i) U1[i] = U[i] + T(0.5 * dt) * L[i];
  bad |= check_state(D, U1.data());
  residual(D, U1.data(), L.data());
  for (int64_t i = 0; i < len; ++i) U2[i] = U[i] + T(0.5 * dt) * L[i];
  bad |= check_state(D, U2.data());
  residual(D, U2.data(), L.data());
  for (int64_t i = 0; i < len; ++i) U3[i] = U[i] + T(dt) * L[i];
  bad |= check_state(D, U3.data());
  residual(D, U3.data(), L.data());
  for (int64_t i = 0; i < len; ++i)
    U[i] = T(-1.0 / 3.0) * U[i] + T(1.0 / 3.0) * U1[i] + T(2.0 / 3.0) * U2[i] +
           T(1.0 / 3.0) * U3[i] + T(dt / 6.0) * L[i];
  bad |= check_state(D, U);
  return bad;
}

}  // namespace ora

// ================================================================ C ABI ====
using ora::Desc;
using ora::Dual;

extern "C" {

int ora_nvars(const Desc* D) { return ora::nvars(*D); }

// Threads that share the lines of a residual (0: the OpenMP default).
void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }

int ora_residual(const Desc* D, const double* U, double* R) {
  ora::residual(*D, U, R);
  return 0;
}

// R = L(U) and JV = (dL/dU) V, exactly, by forward-mode dual numbers.
int ora_residual_jvp(const Desc* D, const double* U, const double* V, double* R, double* JV) {
  const int64_t len = ora::nvars(*D) * ora::npoints(*D);
  std::vector<Dual> u(len), r(len);
  for (int64_t i = 0; i < len; ++i) u[i] = Dual(U[i], V[i]);
  ora::residual(*D, u.data(), r.data());
  for (int64_t i = 0; i < len; ++i) {
    R[i] = r[i].v;
    JV[i] = r[i].d;
  }
  return 0;
}

double ora_cfl_dt(const Desc* D, const double* U, double cfl) { return ora::cfl_dt(*D, U, cfl); }

int ora_check_state(const Desc* D, const double* U) { return ora::check_state(*D, U); }

int ora_rk3_step(const Desc* D, double* U, double dt) { return ora::rk3_step(*D, U, dt); }

// One step applied to U and to a tangent V (exact derivative of the step
// with dt held fixed).
int ora_rk3_step_jvp(const Desc* D, double* U, double* V, double dt) {
  const int64_t len = ora::nvars(*D) * ora::npoints(*D);
  std::vector<Dual> u(len);
  for (int64_t i = 0; i < len; ++i) u[i] = Dual(U[i], V[i]);
  int bad = ora::rk3_step(*D, u.data(), dt);
  for (int64_t i = 0; i < len; ++i) {
    U[i] = u[i].v;
    V[i] = u[i].d;
  }
  return bad;
}

// nsteps SSP-RK3 steps.  dt_fixed > 0: that step every time; otherwise the
// CFL step is recomputed from the state before each step.
int ora_run_steps(const Desc* D, double* U, double cfl, double dt_fixed, int64_t nsteps) {
  int bad = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    double dt = dt_fixed > 0.0 ? dt_fixed : ora::cfl_dt(*D, U, cfl);
    bad |= ora::rk3_step(*D, U, dt);
  }
  return bad;
}

// SSP-RK3 steps of the given sizes dts[0 .. n-1] (steps of size 0 are
// skipped): the same run as another integrator that took those steps.
int ora_run_dt_sequence(const Desc* D, double* U, const double* dts, int64_t n) {
  int bad = 0;
  for (int64_t k = 0; k < n; ++k)
    if (dts[k] > 0.0) bad |= ora::rk3_step(*D, U, dts[k]);
  return bad;
}

// March to t_end with the CFL step, the last step clipped to land on t_end.
int ora_run_to_time(const Desc* D, double* U, double cfl, double t_end, int64_t max_steps,
                    int64_t* steps_done, double* t_done) {
  double t = 0.0;
  int64_t s = 0;
  int bad = 0;
  while (t < t_end && s < max_steps) {
    double dt = ora::cfl_dt(*D, U, cfl);
    if (t + dt > t_end) dt = t_end - t;
    bad |= ora::rk3_step(*D, U, dt);
    t += dt;
    ++s;
  }
  *steps_done = s;
  *t_done = t;
  return bad;
}

int ora_rk4_step(const Desc* D, double* U, double dt) { return ora::rk4_step(*D, U, dt); }

int64_t ora_interpolation_weights(const Desc* D, const double* U, double* out, int64_t cap) {
  return ora::interpolation_weights(*D, U, out, cap);
}

// March to t_end with the CFL step (last step clipped) by SSP-RK3 (method 3)
// or the four-stage scheme of eq. 16 (method 4).
int ora_run_to_time_rk(const Desc* D, double* U, double cfl, double t_end, int64_t max_steps,
                       int method, int64_t* steps_done, double* t_done) {
  double t = 0.0;
  int64_t s = 0;
  int bad = 0;
  while (t < t_end && s < max_steps) {
    double dt = ora::cfl_dt(*D, U, cfl);
    if (t + dt > t_end) dt = t_end - t;
    bad |= method == 4 ? ora::rk4_step(*D, U, dt) : ora::rk3_step(*D, U, dt);
    t += dt;
    ++s;
  }
  *steps_done = s;
  *t_done = t;
  return bad;
}

// Interpolation of one stencil (u_{i-2..i+2}) to x_{i+1/2}, with the weights
// before (w_base) and after (w_out) mapping.
double ora_interpolate(const Desc* D, const double* u, double* w_base, double* w_out) {
  return ora::interpolate(*D, u, w_base, w_out);
}

// The same, with the derivative along du.
double ora_interpolate_jvp(const Desc* D, const double* u, const double* du, double* dout) {
  Dual s[5];
  for (int k = 0; k < 5; ++k) s[k] = Dual(u[k], du[k]);
  Dual r = ora::interpolate(*D, s);
  *dout = r.d;
  return r.v;
}

double ora_fe_map(int i, double w, double xi, double kappa) { return ora::fe_map(i, w, xi, kappa); }

double ora_fe_map_family(int i, double w, double xi, double kappa, int family) {
  return ora::fe_map(i, w, xi, kappa, family);
}

// One WENO5 reconstruction of App. B from the point values f (f_{i-2..i+2}).
double ora_reconstruct_weno(const Desc* D, const double* f, double* w_base, double* w_out) {
  return ora::reconstruct_weno(*D, f, w_base, w_out);
}

// Roe-averaged eigenvectors (row-major 5x5 each) and flux of one state.
void ora_eigenvectors(int nd, int d, double gamma, const double* Ua, const double* Ub, double* L,
                      double* R) {
  double Lm[5][5], Rm[5][5];
  ora::euler_eigenvectors(nd, d, gamma, Ua, Ub, Lm, Rm);
  for (int r = 0; r < 5; ++r)
    for (int s = 0; s < 5; ++s) {
      L[r * 5 + s] = Lm[r][s];
      R[r * 5 + s] = Rm[r][s];
    }
}

void ora_euler_flux(int nd, int d, double gamma, const double* U, double* F) {
  ora::euler_flux(nd, d, gamma, U, F);
}

// Midpoint flux from six nodes (AoS, 6*nv values).
void ora_midpoint_flux(const Desc* D, int d, const double* nodes, double* F) {
  const int nv = ora::nvars(*D);
  const double* st[6];
  for (int k = 0; k < 6; ++k) st[k] = nodes + k * nv;
  ora::midpoint_flux(*D, d, st, F);
}

// Arithmetic tally of one residual evaluation (add/sub, mul, div, sqrt, tanh).
void ora_count_residual_ops(const Desc* D, const double* U, long long* counts) {
  const int64_t len = ora::nvars(*D) * ora::npoints(*D);
  std::vector<ora::Counted> u(len), r(len);
  for (int64_t i = 0; i < len; ++i) u[i] = ora::Counted(U[i]);
  ora::g_ops = ora::OpCount();
  ora::residual(*D, u.data(), r.data());
  counts[0] = ora::g_ops.add;
  counts[1] = ora::g_ops.mul;
  counts[2] = ora::g_ops.div;
  counts[3] = ora::g_ops.sqrt;
  counts[4] = ora::g_ops.tanh;
}

// Arithmetic tally of one interpolation (eq. 5-15, 20-21) of the stencil u.
void ora_count_interpolate_ops(const Desc* D, const double* u, long long* counts) {
  ora::Counted s[5];
  for (int k = 0; k < 5; ++k) s[k] = ora::Counted(u[k]);
  ora::g_ops = ora::OpCount();
  ora::interpolate(*D, s);
  counts[0] = ora::g_ops.add;
  counts[1] = ora::g_ops.mul;
  counts[2] = ora::g_ops.div;
  counts[3] = ora::g_ops.sqrt;
  counts[4] = ora::g_ops.tanh;
}

// Arithmetic tally of one midpoint flux (direction d) from six nodes (AoS).
void ora_count_midpoint_flux_ops(const Desc* D, int d, const double* nodes, long long* counts) {
  const int nv = ora::nvars(*D);
  std::vector<ora::Counted> c(6 * nv);
  for (int k = 0; k < 6 * nv; ++k) c[k] = ora::Counted(nodes[k]);
  const ora::Counted* st[6];
  for (int k = 0; k < 6; ++k) st[k] = c.data() + k * nv;
  ora::Counted F[5];
  ora::g_ops = ora::OpCount();
  ora::midpoint_flux(*D, d, st, F);
  counts[0] = ora::g_ops.add;
  counts[1] = ora::g_ops.mul;
  counts[2] = ora::g_ops.div;
  counts[3] = ora::g_ops.sqrt;
  counts[4] = ora::g_ops.tanh;
}

}  // extern "C"
