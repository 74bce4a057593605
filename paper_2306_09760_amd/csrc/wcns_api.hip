// C ABI of the WCNS-FE library: plan management, host-side validation,
// workspace layout, SSP-RK3 orchestration, the ragged batch with its
// graph-captured step, and the tile autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>
#include <algorithm>

#include "../../include/wcns.h"
#include "wcns_internal.hpp"

using namespace wcns;

namespace {

thread_local std::string g_err;

wcns_status fail(wcns_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wcns_status fail(wcns_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

wcns_status hip_fail(hipError_t e, const char* what) {
  return fail(WCNS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define WCNS_HIP(call, what)                         \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Tile candidates: x sweeps (and the batch) take tm midpoints per tile; y/z
// sweeps take (tm, w) = midpoints along the line by adjacent x-columns.
const int kTmCandidates[] = {128, 256};
const int kYzCandidates[][2] = {{16, 8}, {32, 4}, {32, 8}, {64, 4}, {128, 2}, {256, 1}};
const int kNumYz = 6;

bool in_list(int v, const int* l, int n) {
  for (int i = 0; i < n; ++i)
    if (l[i] == v) return true;
  return false;
}

// Null points kappa*(psi_{i,j} + psi_{i,j-1}) of eq. 20 from the coefficient
// table of Sec. 3.1.
// Null points kappa (psi_{i,j} + psi_{i,j-1}) of the three maps: the psi of
// the coefficient table of Sec. 3.1 (WCNS) or of Table B.2 (WENO).
void fill_null_points(double kappa, int scheme, double* nu) {
  const bool weno = scheme == WCNS_SCHEME_WENO;
  const double psi0[4] = {0.0, weno ? 1.0 / 10.0 : 1.0 / 16.0, weno ? 1.0 / 7.0 : 1.0 / 11.0, 1.0};
  const double psi1[5] = {0.0, weno ? 6.0 / 10.0 : 10.0 / 16.0, 2.0 / 3.0,
                          weno ? 6.0 / 7.0 : 10.0 / 11.0, 1.0};
  const double psi2[4] = {0.0, weno ? 3.0 / 10.0 : 5.0 / 16.0, 1.0 / 3.0, 1.0};
  int k = 0;
  for (int j = 1; j <= 3; ++j) nu[k++] = kappa * (psi0[j] + psi0[j - 1]);
  for (int j = 1; j <= 4; ++j) nu[k++] = kappa * (psi1[j] + psi1[j - 1]);
  for (int j = 1; j <= 3; ++j) nu[k++] = kappa * (psi2[j] + psi2[j - 1]);
}

wcns_status validate(const wcns_desc* d, bool batch) {
  if (!d) return fail(WCNS_EINVAL, "desc is NULL");
  if (d->struct_size != (int32_t)sizeof(wcns_desc))
    return fail(WCNS_EINVAL, "desc.struct_size %d != sizeof(wcns_desc) %d", d->struct_size,
                (int)sizeof(wcns_desc));
  if (d->system != WCNS_SYS_ADVECTION && d->system != WCNS_SYS_EULER)
    return fail(WCNS_EINVAL, "unknown system %d", d->system);
  if (d->ndim < 1 || d->ndim > 3) return fail(WCNS_EINVAL, "ndim %d not in 1..3", d->ndim);
  if (batch && d->ndim != 1) return fail(WCNS_EINVAL, "a batch prototype must be 1D");
  if (batch && d->system != WCNS_SYS_EULER)
    return fail(WCNS_EUNSUPPORTED, "the batch supports the 1D Euler system");
  if (d->weights < WCNS_W_JS || d->weights > WCNS_W_LINEAR)
    return fail(WCNS_EINVAL, "unknown weights %d", d->weights);
  if (d->diff != WCNS_DIFF_MND6 && d->diff != WCNS_DIFF_MD6)
    return fail(WCNS_EINVAL, "unknown difference operator %d", d->diff);
  if (d->z_power < 1 || d->z_power > 4) return fail(WCNS_EINVAL, "z_power %d not in 1..4", d->z_power);
  if (!(d->eps >= 0.0) || !std::isfinite(d->eps)) return fail(WCNS_EINVAL, "eps must be >= 0");
  if (!(d->xi > 0.0) || !std::isfinite(d->xi)) return fail(WCNS_EINVAL, "xi must be > 0");
  if (!std::isfinite(d->kappa)) return fail(WCNS_EINVAL, "kappa must be finite");
  if (!(d->cv >= 0.0)) return fail(WCNS_EINVAL, "cv must be >= 0");
  if (d->system == WCNS_SYS_EULER && !(d->gamma > 1.0))
    return fail(WCNS_EINVAL, "gamma must be > 1");
  if (d->char_proj != 0 && d->char_proj != 1) return fail(WCNS_EINVAL, "char_proj must be 0 or 1");
  if (d->scheme != WCNS_SCHEME_WCNS && d->scheme != WCNS_SCHEME_WENO)
    return fail(WCNS_EINVAL, "unknown scheme %d", d->scheme);
  if (batch && d->scheme != WCNS_SCHEME_WCNS)
    return fail(WCNS_EUNSUPPORTED, "the batch supports the WCNS scheme");
  for (int k = 0; k < 3; ++k) {
    if (k < d->ndim) {
      if (!batch && d->n[k] < 9) return fail(WCNS_EINVAL, "n[%d] = %lld < 9", k, (long long)d->n[k]);
      if (!batch && !(d->h[k] > 0.0)) return fail(WCNS_EINVAL, "h[%d] must be > 0", k);
      if (d->bc[k] != WCNS_BC_PERIODIC && d->bc[k] != WCNS_BC_TRANSMISSIVE)
        return fail(WCNS_EINVAL, "unknown bc[%d] %d", k, d->bc[k]);
      if (!std::isfinite(d->adv_speed[k])) return fail(WCNS_EINVAL, "adv_speed[%d] not finite", k);
    } else if (!batch && d->n[k] != 1) {
      return fail(WCNS_EINVAL, "n[%d] must be 1 for ndim %d", k, d->ndim);
    }
  }
  if (!batch) {
    const double np = (double)d->n[0] * (double)d->n[1] * (double)d->n[2];
    if (np * (d->ndim + 2) > 4.0e9) return fail(WCNS_EINVAL, "grid too large");
  }
  return WCNS_OK;
}

void interp_params(const wcns_desc* d, InterpParams* ip) {
  ip->eps = d->eps;
  ip->xi = d->xi;
  ip->cv = d->cv;
  double nu[10];
  fill_null_points(d->kappa, d->scheme, nu);
  ip->weno = d->scheme == WCNS_SCHEME_WENO ? 1 : 0;
  ip->weights = d->weights;
  ip->zpow = d->z_power;
  // One exponential per map: reference point c_i = mean of the map's null
  // points, K_j = exp(2 xi (c_i - nu_j)).  Usable while xi |nu_j - c_i| < 300
  // (then E = exp(2 xi (w - c_i)) and E K_j stay finite and normal whenever
  // a term is unsaturated, |xi (w - nu_j)| < 20); otherwise K_j = nu_j and
  // every unsaturated term takes its own exponential.
  const int first[3] = {0, 3, 7}, count[3] = {3, 4, 3};
  double spread = 0.0, c[3];
  for (int m = 0; m < 3; ++m) {
    c[m] = 0.0;
    for (int j = 0; j < count[m]; ++j) c[m] += nu[first[m] + j];
    c[m] /= count[m];
    for (int j = 0; j < count[m]; ++j) spread = std::max(spread, std::fabs(c[m] - nu[first[m] + j]));
  }
  ip->shared_exp = (d->xi * spread < 300.0) ? 1 : 0;
  // Bound on ln of the product of the three maps' denominators in the
  // unclamped SPEC_FE path: its largest value over the simplex of weights,
  // taken at a vertex (w_i = 1, the other two 0).
  auto softplus = [](double x) { return x > 30.0 ? x + std::log1p(std::exp(-x)) : std::log1p(std::exp(x)); };
  double B = 0.0;
  for (int i = 0; i < 3; ++i) {
    double b = 0.0;
    for (int m = 0; m < 3; ++m)
      for (int j = 0; j < count[m]; ++j)
        b += softplus(2.0 * d->xi * ((m == i ? 1.0 : 0.0) - nu[first[m] + j]));
    B = std::max(B, b);
  }
  // The fast path also takes the third map's exponential as
  // Ke / (E_0 E_1): E_0 E_1 = exp(2 xi (w_0 + w_1 - c_0 - c_1)) must stay a
  // normal number for w_0 + w_1 in [0, 1].
  const bool prod_ok = 2.0 * d->xi < 650.0 && 2.0 * d->xi * (c[0] + c[1]) < 650.0 &&
                       std::fabs(2.0 * d->xi * (1.0 - c[0] - c[1] - c[2])) < 650.0;
  ip->fast_fe = (ip->shared_exp && B < 600.0 && prod_ok) ? 1 : 0;
  for (int m = 0; m < 3; ++m) {
    ip->C2[m] = ip->shared_exp ? 2.0 * d->xi * c[m] : 0.0;
    for (int j = 0; j < count[m]; ++j) {
      const int k = first[m] + j;
      ip->K[k] = ip->shared_exp ? std::exp(2.0 * d->xi * (c[m] - nu[k])) : nu[k];
    }
  }
  ip->Ke = ip->shared_exp ? std::exp(2.0 * d->xi - ip->C2[0] - ip->C2[1] - ip->C2[2]) : 0.0;
  // Polynomial coefficients of the maps in E (fe_map_poly), in long double
  // from the K_j: elementary symmetric polynomials e_r of the map's K_j for
  // the denominator prod_j (1 + E K_j), and of the K_l, l != j, weighted by
  // -2 a_j and -2 b_j for the numerator.
  const double* fa[3] = {ip->weno ? kV0a : kG0a, ip->weno ? kV1a : kG1a, ip->weno ? kV2a : kG2a};
  const double* fb[3] = {ip->weno ? kV0b : kG0b, ip->weno ? kV1b : kG1b, ip->weno ? kV2b : kG2b};
  const int offd[3] = {0, 3, 7}, offp[3] = {0, 2, 5};
  auto esym = [](const long double* x, int n, long double* e) {  // e[0..n]
    e[0] = 1.0L;
    for (int r = 1; r <= n; ++r) e[r] = 0.0L;
    for (int i = 0; i < n; ++i)
      for (int r = i + 1; r >= 1; --r) e[r] += x[i] * e[r - 1];
  };
  for (int m = 0; m < 3; ++m) {
    const int nt = count[m];
    long double K[4], e[5], ex[5], pa[4] = {0, 0, 0, 0}, pb[4] = {0, 0, 0, 0};
    for (int j = 0; j < nt; ++j) K[j] = ip->shared_exp ? (long double)ip->K[first[m] + j] : 0.0L;
    esym(K, nt, e);
    // monic: divided by the leading coefficient prod_j K_j (1 up to rounding)
    const long double lead = ip->shared_exp ? e[nt] : 1.0L;
    for (int r = 1; r < nt; ++r) ip->Pd[offd[m] + r - 1] = (double)(e[r] / lead);
    ip->Pd[offd[m] + nt - 1] = (double)(1.0L / lead);
    for (int j = 0; j < nt; ++j) {
      long double rest[3];
      int n = 0;
      for (int l = 0; l < nt; ++l)
        if (l != j) rest[n++] = K[l];
      esym(rest, n, ex);
      for (int r = 1; r < nt; ++r) {
        pa[r] += -2.0L * fa[m][j] * ex[r];
        pb[r] += -2.0L * fb[m][j] * ex[r];
      }
    }
    for (int r = 1; r < nt; ++r) {
      ip->Pa[offp[m] + r - 1] = (double)(pa[r] / lead);
      ip->Pb[offp[m] + r - 1] = (double)(pb[r] / lead);
    }
  }
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

struct TuneKey {
  int ndim, nv, weights, diff, charproj;
  int64_t n0, n1, n2;
  bool operator<(const TuneKey& o) const {
    return std::tie(ndim, nv, weights, diff, charproj, n0, n1, n2) <
           std::tie(o.ndim, o.nv, o.weights, o.diff, o.charproj, o.n0, o.n1, o.n2);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::tuple<int, int, int>> g_tune_cache;

}  // namespace

struct wcns_plan {
  wcns_desc d;
  int nv;
  int64_t npts;
  int tm, seg, bw;
  InterpParams ip;
  double ih[3];
  int ncfl;
  size_t off_W1, off_W2, off_R, off_partial, off_dt, off_A1, off_A2, bytes;
};

struct wcns_batch_plan {
  wcns_desc d;
  int64_t nprob, total;
  std::vector<int64_t> h_offset;
  std::vector<double> h_ih;
  int64_t* d_offset = nullptr;
  double* d_ih = nullptr;
  int32_t* d_tile_p0 = nullptr;
  int32_t* d_tile_p1 = nullptr;
  int32_t ntiles = 0;
  int tm = 128;
  int grid = 0;
  int cus = 256;
  InterpParams ip;
  int64_t max_tiles = 0;  // tiles of the smallest tile candidate (sizes the live list)
  // workspace and tile size of the last live-list rebuild (wcns_batch_stage
  // uses the list only if both still hold)
  const void* list_work = nullptr;
  int list_tm = 0;
  size_t off_W1, off_W2, off_dtp, off_wmax, off_live, off_nlive, bytes;
  // graph-captured step
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  std::tuple<const void*, const void*, const void*, double, double, const void*, int> key;
};

namespace {

wcns_status sweep_common(const wcns_plan* P, int d, SweepArgs* a) {
  std::memset(a, 0, sizeof *a);
  a->npts = P->npts;
  for (int k = 0; k < 3; ++k) a->n[k] = P->d.n[k];
  a->bc = P->d.bc[d];
  a->diff = P->d.diff;
  a->ih = P->ih[d];
  a->ip = P->ip;
  a->pp.gamma = P->d.gamma;
  a->pp.adv = P->d.adv_speed[d];
  a->pp.charproj = P->d.char_proj;
  return WCNS_OK;
}

hipError_t run_sweep(const wcns_plan* P, int d, SweepArgs& a, int mode, hipStream_t s) {
  if (P->d.scheme == WCNS_SCHEME_WENO) return launch_weno_sweep(P->nv, d, a, mode, s);
  if (d == 0) return launch_sweep(P->nv, 0, a, mode, P->tm, 1, s);
  return launch_sweep(P->nv, d, a, mode, P->seg, P->bw, s);
}

// R = L(U) into R.
wcns_status residual_into(const wcns_plan* P, const double* U, double* R, hipStream_t s) {
  for (int d = 0; d < P->d.ndim; ++d) {
    SweepArgs a;
    sweep_common(P, d, &a);
    a.U = U;
    a.out = R;
    a.Rin = R;
    WCNS_HIP(run_sweep(P, d, a, d == 0 ? MODE_RES : MODE_ACC, s), "residual sweep launch");
  }
  return WCNS_OK;
}

// out = ca*U0 + cb*(Uk + dt*L(Uk)).
wcns_status stage(const wcns_plan* P, const double* Uk, const double* U0, double* out, double ca,
                  double cb, const double* dt, double* Racc, int32_t* status, hipStream_t s) {
  const int nd = P->d.ndim;
  for (int d = 0; d < nd; ++d) {
    SweepArgs a;
    sweep_common(P, d, &a);
    a.U = Uk;
    const bool last = (d == nd - 1);
    int mode;
    if (last) {
      mode = MODE_STAGE;
      a.U0 = U0;
      a.out = out;
      a.Rin = (nd > 1) ? Racc : nullptr;
      a.dt = dt;
      a.status = status;
      a.ca = ca;
      a.cb = cb;
    } else {
      mode = (d == 0) ? MODE_RES : MODE_ACC;
      a.out = Racc;
      a.Rin = Racc;
    }
    WCNS_HIP(run_sweep(P, d, a, mode, s), "stage sweep launch");
  }
  return WCNS_OK;
}

// out = ca*U0 + cb*Uk + cr*dt*L(Uk).
wcns_status stage_lin(const wcns_plan* P, const double* Uk, const double* U0, double* out,
                      double ca, double cb, double cr, const double* dt, double* Racc,
                      int32_t* status, hipStream_t s) {
  const int nd = P->d.ndim;
  for (int d = 0; d < nd; ++d) {
    SweepArgs a;
    sweep_common(P, d, &a);
    a.U = Uk;
    const bool last = (d == nd - 1);
    int mode;
    if (last) {
      mode = MODE_LIN;
      a.U0 = U0;
      a.out = out;
      a.Rin = (nd > 1) ? Racc : nullptr;
      a.dt = dt;
      a.status = status;
      a.ca = ca;
      a.cb = cb;
      a.cr = cr;
    } else {
      mode = (d == 0) ? MODE_RES : MODE_ACC;
      a.out = Racc;
      a.Rin = Racc;
    }
    WCNS_HIP(run_sweep(P, d, a, mode, s), "stage sweep launch");
  }
  return WCNS_OK;
}

}  // namespace

extern "C" {

void wcns_desc_init(wcns_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof *d);
  d->struct_size = sizeof(wcns_desc);
  d->system = WCNS_SYS_EULER;
  d->ndim = 1;
  d->weights = WCNS_W_FE;
  d->n[0] = d->n[1] = d->n[2] = 1;
  d->h[0] = d->h[1] = d->h[2] = 1.0;
  d->adv_speed[0] = d->adv_speed[1] = d->adv_speed[2] = 1.0;
  d->bc[0] = d->bc[1] = d->bc[2] = WCNS_BC_PERIODIC;
  d->diff = WCNS_DIFF_MND6;
  d->gamma = 1.4;
  d->eps = 1e-40;
  d->xi = 100.0;
  d->kappa = 0.5;
  d->cv = 1e-3;
  d->z_power = 2;
  d->char_proj = 1;
}

wcns_status wcns_plan_create(const wcns_desc* desc, wcns_plan** plan) {
  g_err.clear();
  if (!plan) return fail(WCNS_EINVAL, "plan is NULL");
  *plan = nullptr;
  wcns_status st = validate(desc, false);
  if (st != WCNS_OK) return st;
  wcns_plan* P = new (std::nothrow) wcns_plan();
  if (!P) return fail(WCNS_ENOMEM, "host allocation failed");
  P->d = *desc;
  P->nv = desc->system == WCNS_SYS_ADVECTION ? 1 : desc->ndim + 2;
  if (P->nv == 3 && desc->ndim != 1) {
    delete P;
    return fail(WCNS_EINVAL, "inconsistent nv");
  }
  P->npts = desc->n[0] * desc->n[1] * desc->n[2];
  for (int k = 0; k < 3; ++k) P->ih[k] = k < desc->ndim ? 1.0 / desc->h[k] : 0.0;
  interp_params(desc, &P->ip);
  P->tm = 128;
  P->seg = 32;
  P->bw = 4;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    TuneKey k{desc->ndim, P->nv, desc->weights, desc->diff, desc->char_proj, desc->n[0], desc->n[1], desc->n[2]};
    auto it = g_tune_cache.find(k);
    if (it != g_tune_cache.end()) std::tie(P->tm, P->seg, P->bw) = it->second;
  }
  P->ncfl = cfl_blocks(P->npts);
  const size_t state = sizeof(double) * P->nv * P->npts;
  size_t o = 0;
  P->off_W1 = o; o += align256(state);
  P->off_W2 = o; o += align256(state);
  P->off_R = o; o += align256(state);
  P->off_A1 = o; o += align256(state);
  P->off_A2 = o; o += align256(state);
  P->off_partial = o; o += align256(sizeof(double) * P->ncfl);
  P->off_dt = o; o += 256;
  P->bytes = o;
  *plan = P;
  return WCNS_OK;
}

wcns_status wcns_plan_destroy(wcns_plan* plan) {
  delete plan;
  return WCNS_OK;
}

int64_t wcns_state_elems(const wcns_plan* plan) { return plan ? plan->nv * plan->npts : 0; }
size_t wcns_workspace_bytes(const wcns_plan* plan) { return plan ? plan->bytes : 0; }

void wcns_plan_get_tiles(const wcns_plan* plan, int32_t tiles[3]) {
  if (!plan || !tiles) return;
  tiles[0] = plan->tm;
  tiles[1] = plan->seg;
  tiles[2] = plan->bw;
}

wcns_status wcns_plan_set_tiles(wcns_plan* plan, const int32_t tiles[3]) {
  g_err.clear();
  if (!plan || !tiles) return fail(WCNS_EINVAL, "NULL argument");
  bool yz_ok = false;
  for (int k = 0; k < kNumYz; ++k)
    if (kYzCandidates[k][0] == tiles[1] && kYzCandidates[k][1] == tiles[2]) yz_ok = true;
  if (!in_list(tiles[0], kTmCandidates, 2) || !sweep_shape_ok(plan->nv, 0, tiles[0], 1) ||
      !yz_ok || !sweep_shape_ok(plan->nv, 1, tiles[1], tiles[2]))
    return fail(WCNS_EINVAL, "tile shape (%d, %d, %d) not among the candidates", tiles[0], tiles[1],
                tiles[2]);
  plan->tm = tiles[0];
  plan->seg = tiles[1];
  plan->bw = tiles[2];
  return WCNS_OK;
}

wcns_status wcns_residual(wcns_plan* plan, const double* U, double* R, void* work, void* stream) {
  g_err.clear();
  (void)work;
  if (!plan || !U || !R) return fail(WCNS_EINVAL, "NULL argument");
  if (U == R) return fail(WCNS_EINVAL, "U and R must not overlap");
  return residual_into(plan, U, R, (hipStream_t)stream);
}

wcns_status wcns_cfl_dt(wcns_plan* plan, const double* U, double cfl, double* dt_dev, void* work,
                        void* stream) {
  g_err.clear();
  if (!plan || !U || !dt_dev || !work) return fail(WCNS_EINVAL, "NULL argument");
  if (!(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0");
  char* w = (char*)work;
  WCNS_HIP(launch_cfl(plan->nv, plan->d.ndim, U, plan->npts, plan->d.gamma, plan->ih,
                      plan->d.adv_speed, cfl, (double*)(w + plan->off_partial), plan->ncfl,
                      dt_dev, (hipStream_t)stream),
           "cfl launch");
  return WCNS_OK;
}

namespace {
// One SSP-RK3 step of U in place with the stage states in W1, W2, the
// residual accumulator of the 2D/3D sweeps in Racc, and (for a cfl-limited
// step) the block maxima in partial and dt in dtw.
wcns_status rk3_step_bufs(wcns_plan* plan, double* U, double* W1, double* W2, double* Racc,
                          double* partial, double* dtw, const double* dt_dev, double cfl,
                          int32_t* status_dev, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const double* dt = dt_dev;
  if (!dt) {
    if (!(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0 when dt_dev is NULL");
    WCNS_HIP(launch_cfl(plan->nv, plan->d.ndim, U, plan->npts, plan->d.gamma, plan->ih,
                        plan->d.adv_speed, cfl, partial, plan->ncfl, dtw, s),
             "cfl launch");
    dt = dtw;
  }
  wcns_status st;
  if ((st = stage(plan, U, U, W1, 0.0, 1.0, dt, Racc, status_dev, s)) != WCNS_OK) return st;
  if ((st = stage(plan, W1, U, W2, 0.75, 0.25, dt, Racc, status_dev, s)) != WCNS_OK) return st;
  if ((st = stage(plan, W2, U, U, 1.0 / 3.0, 2.0 / 3.0, dt, Racc, status_dev, s)) != WCNS_OK) return st;
  return WCNS_OK;
}

// rk3_step_bufs with the buffers in the caller's workspace.
wcns_status rk3_step_into(wcns_plan* plan, double* U, double* W1, double* W2, void* work,
                          const double* dt_dev, double cfl, int32_t* status_dev, void* stream) {
  char* w = (char*)work;
  return rk3_step_bufs(plan, U, W1, W2, (double*)(w + plan->off_R),
                       (double*)(w + plan->off_partial), (double*)(w + plan->off_dt), dt_dev, cfl,
                       status_dev, stream);
}

// The device array behind wcns_rk3_step_noalloc (each GPU holds its own copy
// until the process ends).  In host code `scratch` names a host-side stand-in;
// its device address on each GPU is taken once, with that GPU current.
constexpr size_t kScratchBytes = size_t(48) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
wcns_status scratch_address(void** out) {
  int dev = 0;
  WCNS_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(WCNS_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    WCNS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(WCNS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WCNS_OK;
}

// Bytes of scratch a step of this plan needs: the two stage states, the
// residual accumulator (2D/3D only), the CFL block maxima and dt.
size_t noalloc_bytes(const wcns_plan* P) {
  const size_t state = align256(sizeof(double) * P->nv * P->npts);
  return 2 * state + (P->d.ndim > 1 ? state : 0) + align256(sizeof(double) * P->ncfl) + 256;
}
}  // namespace

wcns_status wcns_rk3_step(wcns_plan* plan, double* U, void* work, const double* dt_dev, double cfl,
                          int32_t* status_dev, void* stream) {
  g_err.clear();
  if (!plan || !U || !work) return fail(WCNS_EINVAL, "NULL argument");
  char* w = (char*)work;
  return rk3_step_into(plan, U, (double*)(w + plan->off_W1), (double*)(w + plan->off_W2), work,
                       dt_dev, cfl, status_dev, stream);
}

wcns_status wcns_rk3_step_noalloc(wcns_plan* plan, double* U, const double* dt_dev, double cfl,
                                  int32_t* status_dev, void* stream) {
  g_err.clear();
  if (!plan || !U) return fail(WCNS_EINVAL, "NULL argument");
  const size_t need = noalloc_bytes(plan);
  if (need > kScratchBytes)
    return fail(WCNS_EINVAL,
                "wcns_rk3_step_noalloc needs %zu bytes of scratch for this plan, above its "
                "maximum of %zu (states of at most about %zu doubles); use wcns_rk3_step",
                need, kScratchBytes, (kScratchBytes - 65536) / (plan->d.ndim > 1 ? 3 : 2) / 8);
  if (!dt_dev && !(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0 when dt_dev is NULL");
  void* base = nullptr;
  const wcns_status st = scratch_address(&base);
  if (st != WCNS_OK) return st;
  char* w = (char*)base;
  const size_t state = align256(sizeof(double) * plan->nv * plan->npts);
  double* W1 = (double*)w;
  double* W2 = (double*)(w + state);
  size_t o = 2 * state;
  double* Racc = nullptr;
  if (plan->d.ndim > 1) {
    Racc = (double*)(w + o);
    o += state;
  }
  double* partial = (double*)(w + o);
  o += align256(sizeof(double) * plan->ncfl);
  double* dtw = (double*)(w + o);
  return rk3_step_bufs(plan, U, W1, W2, Racc, partial, dtw, dt_dev, cfl, status_dev, stream);
}

wcns_status wcns_rk3_step_stages(wcns_plan* plan, double* U, double* U1, double* U2, void* work,
                                 const double* dt_dev, double cfl, int32_t* status_dev,
                                 void* stream) {
  g_err.clear();
  if (!plan || !U || !U1 || !U2 || !work) return fail(WCNS_EINVAL, "NULL argument");
  if (U1 == U || U2 == U || U1 == U2) return fail(WCNS_EINVAL, "U, U1 and U2 must be distinct");
  return rk3_step_into(plan, U, U1, U2, work, dt_dev, cfl, status_dev, stream);
}

wcns_status wcns_rk4_step(wcns_plan* plan, double* U, void* work, const double* dt_dev, double cfl,
                          int32_t* status_dev, void* stream) {
  g_err.clear();
  if (!plan || !U || !work) return fail(WCNS_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)work;
  double* U1 = (double*)(w + plan->off_W1);
  double* U2 = (double*)(w + plan->off_W2);
  double* U3 = (double*)(w + plan->off_A1);
  double* A = (double*)(w + plan->off_A2);
  double* Racc = (double*)(w + plan->off_R);
  const int64_t len = plan->nv * plan->npts;
  const double* dt = dt_dev;
  if (!dt) {
    if (!(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0 when dt_dev is NULL");
    double* dtw = (double*)(w + plan->off_dt);
    WCNS_HIP(launch_cfl(plan->nv, plan->d.ndim, U, plan->npts, plan->d.gamma, plan->ih,
                        plan->d.adv_speed, cfl, (double*)(w + plan->off_partial), plan->ncfl, dtw, s),
             "cfl launch");
    dt = dtw;
  }
  wcns_status st;
  // u1 = u + dt/2 L(u); u2 = u + dt/2 L(u1); u3 = u + dt L(u2)
  if ((st = stage_lin(plan, U, U, U1, 0.0, 1.0, 0.5, dt, Racc, status_dev, s)) != WCNS_OK) return st;
  if ((st = stage_lin(plan, U1, U, U2, 1.0, 0.0, 0.5, dt, Racc, status_dev, s)) != WCNS_OK) return st;
  if ((st = stage_lin(plan, U2, U, U3, 1.0, 0.0, 1.0, dt, Racc, status_dev, s)) != WCNS_OK) return st;
  // u_new = (-u + u1 + 2 u2)/3 + u3/3 + dt/6 L(u3)
  WCNS_HIP(launch_lincomb(A, U, -1.0 / 3.0, U1, 1.0 / 3.0, nullptr, 0.0, len, s), "lincomb");
  WCNS_HIP(launch_axpy_state(A, U2, 2.0 / 3.0, len, s), "axpy");
  return stage_lin(plan, U3, A, U, 1.0, 1.0 / 3.0, 1.0 / 6.0, dt, Racc, status_dev, s);
}

wcns_status wcns_weight_histogram(wcns_plan* plan, const double* U, uint64_t* hist, int32_t nbins,
                                  void* stream) {
  g_err.clear();
  if (!plan || !U || !hist) return fail(WCNS_EINVAL, "NULL argument");
  if (nbins < 1 || nbins > (1 << 24)) return fail(WCNS_EINVAL, "nbins must be in [1, 2^24]");
  if (plan->d.scheme != WCNS_SCHEME_WCNS)
    return fail(WCNS_EUNSUPPORTED, "weight statistics cover the WCNS scheme");
  for (int d = 0; d < plan->d.ndim; ++d) {
    SweepArgs a;
    sweep_common(plan, d, &a);
    a.U = U;
    WCNS_HIP(launch_weight_hist(plan->nv, d, a, (unsigned long long*)hist, nbins,
                                (hipStream_t)stream),
             "weight histogram launch");
  }
  return WCNS_OK;
}

namespace {
// Ubar = ca A + cb B + scale dt (dL/dU)^T Rbar (A set; the first direction
// writes, the others accumulate) or Ubar += scale dt (dL/dU)^T Rbar (A null);
// dt_dev may be null (factor 1).
wcns_status adjoint_into(wcns_plan* plan, const double* U, const double* Rbar, double* Ubar,
                         double scale, const double* dt_dev, const double* A, double ca,
                         const double* B, double cb, void* stream, const double* C = nullptr,
                         double cc = 0.0) {
  for (int d = 0; d < plan->d.ndim; ++d) {
    AdjArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = U;
    a.Rbar = Rbar;
    a.Ubar = Ubar;
    a.scale = scale;
    a.dt = dt_dev;
    if (d == 0) {
      a.A = A;
      a.ca = ca;
      a.B = B;
      a.cb = cb;
      a.C = C;
      a.cc = cc;
    }
    a.npts = plan->npts;
    for (int k = 0; k < 3; ++k) a.n[k] = plan->d.n[k];
    a.bc = plan->d.bc[d];
    a.diff = plan->d.diff;
    a.ih = plan->ih[d];
    a.ip = plan->ip;
    a.pp.gamma = plan->d.gamma;
    a.pp.adv = plan->d.adv_speed[d];
    a.pp.charproj = plan->d.char_proj;
    WCNS_HIP(launch_adjoint_dir(plan->nv, d, a, (hipStream_t)stream), "adjoint launch");
  }
  return WCNS_OK;
}
}  // namespace

wcns_status wcns_residual_adjoint(wcns_plan* plan, const double* U, const double* Rbar,
                                  double* Ubar, void* work, void* stream) {
  g_err.clear();
  if (!plan || !U || !Rbar || !Ubar || !work) return fail(WCNS_EINVAL, "NULL argument");
  if (Ubar == U || Ubar == Rbar) return fail(WCNS_EINVAL, "Ubar must not alias U or Rbar");
  if (plan->d.scheme != WCNS_SCHEME_WCNS)
    return fail(WCNS_EUNSUPPORTED, "the adjoint covers the WCNS scheme");
  return adjoint_into(plan, U, Rbar, Ubar, 1.0, nullptr, nullptr, 0.0, nullptr, 0.0, stream);
}

namespace {
// Arrays [p, p + bytes) and [q, q + bytes) overlap.
bool overlaps(const void* p, size_t pb, const void* q, size_t qb) {
  const char* a = (const char*)p;
  const char* b = (const char*)q;
  return a < b + qb && b < a + pb;
}

// The reverse step writes lambda in place while neighbouring tiles still read
// the states under the stencil, and keeps its stage cotangents in the
// workspace: lambda must not overlap Un, U1, U2 or the workspace, and the
// states must not overlap the workspace's cotangent buffers.
wcns_status adjoint_aliasing(const wcns_plan* P, const double* Un, const double* U1,
                             const double* U2, const double* lambda, const void* work) {
  const size_t sb = sizeof(double) * P->nv * P->npts;
  const double* st[3] = {Un, U1, U2};
  for (const double* x : st)
    if (x && overlaps(lambda, sb, x, sb))
      return fail(WCNS_EINVAL, "lambda must not overlap Un, U1 or U2");
  if (overlaps(lambda, sb, work, P->bytes)) return fail(WCNS_EINVAL, "lambda must not overlap work");
  const char* w = (const char*)work;
  for (const double* x : st)
    if (x && (overlaps(x, sb, w + P->off_A1, sb) || overlaps(x, sb, w + P->off_A2, sb)))
      return fail(WCNS_EINVAL, "a state overlaps the workspace's cotangent buffers");
  return WCNS_OK;
}

// Reverse of one SSP-RK3 step given its stage states U1, U2.
wcns_status rk3_adjoint_from_stages(wcns_plan* plan, const double* Un, const double* U1,
                                    const double* U2, double* lambda, void* work,
                                    const double* dt_dev, void* stream) {
  char* w = (char*)work;
  double* l2 = (double*)(w + plan->off_A1);
  double* l1 = (double*)(w + plan->off_A2);
  wcns_status st;
  // Stage 3: U3 = 1/3 Un + 2/3 U2 + 2/3 dt L(U2), lambda = adjoint of U3:
  //   l2 = 2/3 lambda + 2/3 dt J(U2)^T lambda
  if ((st = adjoint_into(plan, U2, lambda, l2, 2.0 / 3.0, dt_dev, lambda, 2.0 / 3.0, nullptr, 0.0,
                         stream)) != WCNS_OK)
    return st;
  // Stage 2: U2 = 3/4 Un + 1/4 U1 + 1/4 dt L(U1):
  //   l1 = 1/4 l2 + 1/4 dt J(U1)^T l2
  if ((st = adjoint_into(plan, U1, l2, l1, 0.25, dt_dev, l2, 0.25, nullptr, 0.0, stream)) !=
      WCNS_OK)
    return st;
  // Stage 1: U1 = Un + dt L(Un).  lambda_n = 1/3 lambda (stage 3) + 3/4 l2
  // (stage 2) + l1 + dt J(Un)^T l1, in the epilogue of one launch
  return adjoint_into(plan, Un, l1, lambda, 1.0, dt_dev, lambda, 1.0 / 3.0, l2, 0.75, stream, l1,
                      1.0);
}
}  // namespace

wcns_status wcns_rk3_step_adjoint(wcns_plan* plan, const double* Un, double* lambda, void* work,
                                  const double* dt_dev, void* stream) {
  g_err.clear();
  if (!plan || !Un || !lambda || !work || !dt_dev) return fail(WCNS_EINVAL, "NULL argument");
  if (plan->d.scheme != WCNS_SCHEME_WCNS)
    return fail(WCNS_EUNSUPPORTED, "the adjoint covers the WCNS scheme");
  {
    const wcns_status st = adjoint_aliasing(plan, Un, nullptr, nullptr, lambda, work);
    if (st != WCNS_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)work;
  double* U1 = (double*)(w + plan->off_W1);
  double* U2 = (double*)(w + plan->off_W2);
  double* Racc = (double*)(w + plan->off_R);
  wcns_status st;
  // Recompute the stage states U1 = Un + dt L(Un), U2 = 3/4 Un + 1/4 (U1 +
  // dt L(U1)) with the forward step's own stage launches (bitwise the same).
  if ((st = stage(plan, Un, Un, U1, 0.0, 1.0, dt_dev, Racc, nullptr, s)) != WCNS_OK) return st;
  if ((st = stage(plan, U1, Un, U2, 0.75, 0.25, dt_dev, Racc, nullptr, s)) != WCNS_OK) return st;
  return rk3_adjoint_from_stages(plan, Un, U1, U2, lambda, work, dt_dev, stream);
}

wcns_status wcns_rk3_step_adjoint_stages(wcns_plan* plan, const double* Un, const double* U1,
                                         const double* U2, double* lambda, void* work,
                                         const double* dt_dev, void* stream) {
  g_err.clear();
  if (!plan || !Un || !U1 || !U2 || !lambda || !work || !dt_dev)
    return fail(WCNS_EINVAL, "NULL argument");
  if (plan->d.scheme != WCNS_SCHEME_WCNS)
    return fail(WCNS_EUNSUPPORTED, "the adjoint covers the WCNS scheme");
  {
    const wcns_status st = adjoint_aliasing(plan, Un, U1, U2, lambda, work);
    if (st != WCNS_OK) return st;
  }
  return rk3_adjoint_from_stages(plan, Un, U1, U2, lambda, work, dt_dev, stream);
}

wcns_status wcns_plan_autotune(wcns_plan* plan, const double* U, void* work, void* stream) {
  g_err.clear();
  if (!plan || !U || !work) return fail(WCNS_EINVAL, "NULL argument");
  if (plan->d.scheme == WCNS_SCHEME_WENO) return WCNS_OK;  // one compiled tile shape
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)work;
  double* out = (double*)(w + plan->off_W1);
  hipEvent_t e0, e1;
  WCNS_HIP(hipEventCreate(&e0), "event");
  WCNS_HIP(hipEventCreate(&e1), "event");
  auto time_sweep = [&](int d, float* ms) -> wcns_status {
    SweepArgs a;
    sweep_common(plan, d, &a);
    a.U = U;
    a.out = out;
    a.Rin = out;
    // one warm-up, then three timed launches
    for (int r = 0; r < 4; ++r) {
      if (r == 1) WCNS_HIP(hipEventRecord(e0, s), "event record");
      WCNS_HIP(run_sweep(plan, d, a, MODE_RES, s), "autotune launch");
    }
    WCNS_HIP(hipEventRecord(e1, s), "event record");
    WCNS_HIP(hipEventSynchronize(e1), "event sync");
    WCNS_HIP(hipEventElapsedTime(ms, e0, e1), "event time");
    return WCNS_OK;
  };
  wcns_status st = WCNS_OK;
  float best = 1e30f;
  int best_tm = plan->tm;
  for (int tm : kTmCandidates) {
    if (!sweep_shape_ok(plan->nv, 0, tm, 1)) continue;
    plan->tm = tm;
    float ms;
    if ((st = time_sweep(0, &ms)) != WCNS_OK) break;
    if (ms < best) {
      best = ms;
      best_tm = tm;
    }
  }
  plan->tm = best_tm;
  if (st == WCNS_OK && plan->d.ndim > 1) {
    best = 1e30f;
    int bs = plan->seg, bb = plan->bw;
    for (int k = 0; k < kNumYz; ++k) {
      {
        const int seg = kYzCandidates[k][0], bw = kYzCandidates[k][1];
        if (!sweep_shape_ok(plan->nv, 1, seg, bw)) continue;
        plan->seg = seg;
        plan->bw = bw;
        float ms;
        if ((st = time_sweep(1, &ms)) != WCNS_OK) break;
        if (ms < best) {
          best = ms;
          bs = seg;
          bb = bw;
        }
      }
    }
    plan->seg = bs;
    plan->bw = bb;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != WCNS_OK) return st;
  std::lock_guard<std::mutex> g(g_tune_mu);
  TuneKey k{plan->d.ndim, plan->nv, plan->d.weights, plan->d.diff, plan->d.char_proj,
            plan->d.n[0], plan->d.n[1], plan->d.n[2]};
  g_tune_cache[k] = std::make_tuple(plan->tm, plan->seg, plan->bw);
  return WCNS_OK;
}

// ------------------------------------------------------------------ batch --

static wcns_status batch_build_tiles(wcns_batch_plan* B) {
  // Packed tiles over the virtual index space of the problems laid end to
  // end with 2G ghost slots each (BatchArgs): all tiles are full, so only the
  // 2G slots per problem compute midpoints that no node uses.
  const int G = B->d.diff ? 5 : 4;
  const int TL = B->tm - (B->d.diff ? 5 : 3);
  const int64_t np = B->nprob;
  auto start = [&](int64_t p) { return B->h_offset[p] + 2 * G * p; };
  const int64_t V = start(np);
  const int64_t nt = (V + TL - 1) / TL;
  if (nt > INT32_MAX) return fail(WCNS_EUNSUPPORTED, "batch needs %lld tiles", (long long)nt);
  std::vector<int32_t> tp((size_t)nt), tq((size_t)nt);
  int64_t p = 0, q = 0;  // problems holding the first and the last slot of tile k
  for (int64_t k = 0; k < nt; ++k) {
    const int64_t lo = k * TL - G, hi = k * TL + TL + G - 1;
    while (p + 1 < np && start(p + 1) <= lo) ++p;
    while (q + 1 < np && start(q + 1) <= hi) ++q;
    tp[(size_t)k] = (int32_t)p;
    tq[(size_t)k] = (int32_t)q;
  }
  if (B->d_tile_p0) hipFree(B->d_tile_p0);
  if (B->d_tile_p1) hipFree(B->d_tile_p1);
  B->d_tile_p0 = nullptr;
  B->d_tile_p1 = nullptr;
  B->ntiles = (int32_t)nt;
  B->list_work = nullptr;
  WCNS_HIP(hipMalloc(&B->d_tile_p0, sizeof(int32_t) * tp.size()), "hipMalloc tiles");
  WCNS_HIP(hipMalloc(&B->d_tile_p1, sizeof(int32_t) * tq.size()), "hipMalloc tiles");
  WCNS_HIP(hipMemcpy(B->d_tile_p0, tp.data(), sizeof(int32_t) * tp.size(), hipMemcpyHostToDevice), "copy tiles");
  WCNS_HIP(hipMemcpy(B->d_tile_p1, tq.data(), sizeof(int32_t) * tq.size(), hipMemcpyHostToDevice), "copy tiles");
  // one workgroup per tile
  B->grid = B->ntiles;
  if (B->exec) {
    hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  return WCNS_OK;
}

wcns_status wcns_batch_plan_create(const wcns_desc* proto, int64_t nprob, const int64_t* offsets_host,
                                   const double* h_host, wcns_batch_plan** plan) {
  g_err.clear();
  if (!plan) return fail(WCNS_EINVAL, "plan is NULL");
  *plan = nullptr;
  wcns_status st = validate(proto, true);
  if (st != WCNS_OK) return st;
  if (nprob < 1 || nprob > (1 << 30)) return fail(WCNS_EINVAL, "nprob %lld out of range", (long long)nprob);
  if (!offsets_host || !h_host) return fail(WCNS_EINVAL, "NULL offsets or h");
  if (offsets_host[0] != 0) return fail(WCNS_EINVAL, "offsets[0] must be 0");
  for (int64_t p = 0; p < nprob; ++p) {
    const int64_t N = offsets_host[p + 1] - offsets_host[p];
    if (N < 9) return fail(WCNS_EINVAL, "problem %lld has %lld < 9 nodes", (long long)p, (long long)N);
    if (N > (1 << 30)) return fail(WCNS_EINVAL, "problem %lld too long", (long long)p);
    if (!(h_host[p] > 0.0) || !std::isfinite(h_host[p]))
      return fail(WCNS_EINVAL, "h[%lld] must be > 0", (long long)p);
  }
  wcns_batch_plan* B = new (std::nothrow) wcns_batch_plan();
  if (!B) return fail(WCNS_ENOMEM, "host allocation failed");
  B->d = *proto;
  B->nprob = nprob;
  B->total = offsets_host[nprob];
  B->h_offset.assign(offsets_host, offsets_host + nprob + 1);
  B->h_ih.resize(nprob);
  for (int64_t p = 0; p < nprob; ++p) B->h_ih[p] = 1.0 / h_host[p];
  interp_params(proto, &B->ip);
  B->cus = device_cus();
  auto cleanup = [&](wcns_status s) {
    wcns_batch_plan_destroy(B);
    return s;
  };
  hipError_t e;
  if ((e = hipMalloc(&B->d_offset, sizeof(int64_t) * (nprob + 1))) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipMalloc(&B->d_ih, sizeof(double) * nprob)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipMemcpy(B->d_offset, B->h_offset.data(), sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy"));
  if ((e = hipMemcpy(B->d_ih, B->h_ih.data(), sizeof(double) * nprob, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy"));
  if ((st = batch_build_tiles(B)) != WCNS_OK) return cleanup(st);
  {
    // the most tiles any candidate shape needs (the smallest tile)
    const int G = proto->diff ? 5 : 4;
    const int64_t V = B->h_offset[nprob] + 2 * G * nprob;
    for (int tm : kTmCandidates) {
      const int TL = tm - (proto->diff ? 5 : 3);
      B->max_tiles = std::max(B->max_tiles, (V + TL - 1) / TL);
    }
  }
  const size_t state = sizeof(double) * 3 * B->total;
  size_t o = 0;
  B->off_W1 = o; o += align256(state);
  B->off_W2 = o; o += align256(state);
  B->off_dtp = o; o += align256(sizeof(double) * nprob);
  B->off_wmax = o; o += align256(sizeof(unsigned long long) * nprob);
  B->off_live = o; o += align256(sizeof(int32_t) * B->max_tiles);
  B->off_nlive = o; o += 256;
  B->bytes = o;
  *plan = B;
  return WCNS_OK;
}

wcns_status wcns_batch_plan_destroy(wcns_batch_plan* B) {
  if (!B) return WCNS_OK;
  if (B->exec) hipGraphExecDestroy(B->exec);
  if (B->cap_stream) hipStreamDestroy(B->cap_stream);
  if (B->d_offset) hipFree(B->d_offset);
  if (B->d_ih) hipFree(B->d_ih);
  if (B->d_tile_p0) hipFree(B->d_tile_p0);
  if (B->d_tile_p1) hipFree(B->d_tile_p1);
  delete B;
  return WCNS_OK;
}

int64_t wcns_batch_state_elems(const wcns_batch_plan* B) { return B ? 3 * B->total : 0; }
size_t wcns_batch_workspace_bytes(const wcns_batch_plan* B) { return B ? B->bytes : 0; }

static void batch_args(const wcns_batch_plan* B, double* dtp, SweepArgs* a, BatchArgs* b,
                       void* work = nullptr) {
  std::memset(a, 0, sizeof *a);
  std::memset(b, 0, sizeof *b);
  a->npts = B->total;
  a->n[0] = B->total;
  a->n[1] = a->n[2] = 1;
  a->bc = B->d.bc[0];
  a->diff = B->d.diff;
  a->ih = 0.0;
  a->ip = B->ip;
  a->pp.gamma = B->d.gamma;
  a->pp.adv = 0.0;
  a->pp.charproj = B->d.char_proj;
  b->offset = B->d_offset;
  b->ih = B->d_ih;
  b->dtp = dtp;
  b->tile_p0 = B->d_tile_p0;
  b->tile_p1 = B->d_tile_p1;
  b->ntiles = B->ntiles;
  b->nprob = (int32_t)B->nprob;
  // stage launches walk the live-tile list in the workspace
  b->live = work ? (const int32_t*)((const char*)work + B->off_live) : nullptr;
  b->nlive = work ? (const int32_t*)((const char*)work + B->off_nlive) : nullptr;
}

// The live-tile list of the dt just computed (the dt kernel cleared the count).
static wcns_status batch_rebuild_live(wcns_batch_plan* B, const BatchArgs& b, void* work,
                                      hipStream_t s) {
  char* w = (char*)work;
  B->list_work = work;
  B->list_tm = B->tm;
  WCNS_HIP(launch_batch_live(b, (int32_t*)(w + B->off_live), (int32_t*)(w + B->off_nlive), s),
           "batch live-list launch");
  return WCNS_OK;
}

wcns_status wcns_batch_residual(wcns_batch_plan* B, const double* U, double* R, void* work, void* stream) {
  g_err.clear();
  (void)work;
  if (!B || !U || !R) return fail(WCNS_EINVAL, "NULL argument");
  if (U == R) return fail(WCNS_EINVAL, "U and R must not overlap");
  SweepArgs a;
  BatchArgs b;
  batch_args(B, nullptr, &a, &b);
  a.U = U;
  a.out = R;
  WCNS_HIP(launch_batch_sweep(a, b, MODE_RES, B->tm, (hipStream_t)stream), "batch residual launch");
  return WCNS_OK;
}

// One SSP-RK3 step of the batch.  dt comes from a pass over U, or (fused_dt)
// from the per-problem maxima that the previous step's last stage left in
// the workspace; with keep_max this step's last stage leaves them for the
// next step.  With rebuild the live-tile list is rebuilt from this step's
// dt; otherwise the list of an earlier step of the same call is used (a
// superset: problems only finish).
static wcns_status batch_step_enqueue(wcns_batch_plan* B, double* U, void* work, double* t_dev,
                                      double t_end, double cfl, int32_t* status, hipStream_t s,
                                      bool fused_dt = false, bool keep_max = false,
                                      bool rebuild = true, int32_t cap = 0) {
  char* w = (char*)work;
  double* W1 = (double*)(w + B->off_W1);
  double* W2 = (double*)(w + B->off_W2);
  double* dtp = (double*)(w + B->off_dtp);
  unsigned long long* wmax = (unsigned long long*)(w + B->off_wmax);
  int32_t* nlive = rebuild ? (int32_t*)(w + B->off_nlive) : nullptr;
  SweepArgs a;
  BatchArgs b;
  batch_args(B, dtp, &a, &b, work);
  if (fused_dt)
    WCNS_HIP(launch_batch_dt(b, t_dev, t_end, cfl, wmax, status, nlive, s), "batch dt launch");
  else
    WCNS_HIP(launch_batch_cfl(U, B->total, b, B->d.gamma, t_dev, t_end, cfl,
                              keep_max ? wmax : nullptr, status, nlive, s),
             "batch cfl launch");
  if (rebuild) {
    const wcns_status st = batch_rebuild_live(B, b, work, s);
    if (st != WCNS_OK) return st;
  }
  a.status = status;
  a.U0 = U;
  const double* src[3] = {U, W1, W2};
  double* dst[3] = {W1, W2, U};
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int k = 0; k < 3; ++k) {
    a.U = src[k];
    a.out = dst[k];
    a.ca = ca[k];
    a.cb = cb[k];
    a.wmax = (k == 2 && keep_max) ? wmax : nullptr;
    WCNS_HIP(launch_batch_sweep(a, b, MODE_STAGE, B->tm, s, cap), "batch stage launch");
  }
  return WCNS_OK;
}

// Within one wcns_batch_rk3_steps call the live-tile list is rebuilt every
// kLiveEvery steps (and for the first); in between, tiles whose problems
// finished stay listed and leave at once.
static const int32_t kLiveEvery = 4;

static wcns_status batch_rk3_steps(wcns_batch_plan* B, double* U, void* work, double* t_dev,
                                   double t_end, double cfl, int32_t nsteps, int32_t* status_dev,
                                   int32_t cap, void* stream) {
  if (!B || !U || !work || !t_dev) return fail(WCNS_EINVAL, "NULL argument");
  if (!(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0");
  if (!std::isfinite(t_end)) return fail(WCNS_EINVAL, "t_end must be finite");
  if (nsteps < 0) return fail(WCNS_EINVAL, "nsteps %d < 0", nsteps);
  hipStream_t s = (hipStream_t)stream;
  for (int32_t k = 0; k < nsteps; ++k) {
    const wcns_status st = batch_step_enqueue(B, U, work, t_dev, t_end, cfl, status_dev, s, k > 0,
                                              k + 1 < nsteps, k % kLiveEvery == 0, cap);
    if (st != WCNS_OK) return st;
  }
  return WCNS_OK;
}

wcns_status wcns_batch_rk3_steps(wcns_batch_plan* B, double* U, void* work, double* t_dev,
                                 double t_end, double cfl, int32_t nsteps, int32_t* status_dev,
                                 void* stream) {
  g_err.clear();
  return batch_rk3_steps(B, U, work, t_dev, t_end, cfl, nsteps, status_dev, 0, stream);
}

wcns_status wcns_batch_rk3_steps_capped(wcns_batch_plan* B, double* U, void* work, double* t_dev,
                                        double t_end, double cfl, int32_t nsteps,
                                        int32_t* status_dev, int32_t max_live, void* stream) {
  g_err.clear();
  if (!status_dev) return fail(WCNS_EINVAL, "a capped call needs status_dev");
  if (max_live < 1) return fail(WCNS_EINVAL, "max_live %d < 1", max_live);
  return batch_rk3_steps(B, U, work, t_dev, t_end, cfl, nsteps, status_dev, max_live, stream);
}

wcns_status wcns_batch_live_tiles(const wcns_batch_plan* B, const void* work, int32_t* count,
                                  void* stream) {
  g_err.clear();
  if (!B || !work || !count) return fail(WCNS_EINVAL, "NULL argument");
  if (B->list_work != work || B->list_tm != B->tm)
    return fail(WCNS_EINVAL, "no live-tile list in this workspace for the current tile size");
  hipStream_t s = (hipStream_t)stream;
  WCNS_HIP(hipMemcpyAsync(count, (const char*)work + B->off_nlive, sizeof(int32_t),
                          hipMemcpyDeviceToHost, s),
           "live count copy");
  WCNS_HIP(hipStreamSynchronize(s), "live count sync");
  return WCNS_OK;
}

wcns_status wcns_batch_rk3_step(wcns_batch_plan* B, double* U, void* work, double* t_dev, double t_end,
                                double cfl, int32_t* status_dev, void* stream) {
  g_err.clear();
  if (!B || !U || !work || !t_dev) return fail(WCNS_EINVAL, "NULL argument");
  if (!(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0");
  if (!std::isfinite(t_end)) return fail(WCNS_EINVAL, "t_end must be finite");
  hipStream_t s = (hipStream_t)stream;
  if (!B->use_graph) return batch_step_enqueue(B, U, work, t_dev, t_end, cfl, status_dev, s);
  auto key = std::make_tuple((const void*)U, (const void*)work, (const void*)t_dev, t_end, cfl,
                             (const void*)status_dev, B->tm);
  if (!B->exec || key != B->key) {
    if (B->exec) {
      hipGraphExecDestroy(B->exec);
      B->exec = nullptr;
    }
    if (!B->cap_stream) WCNS_HIP(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking), "stream create");
    WCNS_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    wcns_status st = batch_step_enqueue(B, U, work, t_dev, t_end, cfl, status_dev, B->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (st != WCNS_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      B->exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    B->key = key;
  }
  WCNS_HIP(hipGraphLaunch(B->exec, s), "graph launch");
  return WCNS_OK;
}

wcns_status wcns_batch_cfl(wcns_batch_plan* B, const double* U, void* work, double* t_dev,
                           double t_end, double cfl, void* stream) {
  g_err.clear();
  if (!B || !U || !work || !t_dev) return fail(WCNS_EINVAL, "NULL argument");
  if (!(cfl > 0.0)) return fail(WCNS_EINVAL, "cfl must be > 0");
  if (!std::isfinite(t_end)) return fail(WCNS_EINVAL, "t_end must be finite");
  SweepArgs a;
  BatchArgs b;
  batch_args(B, (double*)((char*)work + B->off_dtp), &a, &b, work);
  WCNS_HIP(launch_batch_cfl(U, B->total, b, B->d.gamma, t_dev, t_end, cfl, nullptr, nullptr,
                            (int32_t*)((char*)work + B->off_nlive), (hipStream_t)stream),
           "batch cfl launch");
  return batch_rebuild_live(B, b, work, (hipStream_t)stream);
}

wcns_status wcns_batch_stage(wcns_batch_plan* B, int32_t stage, const double* Uk, const double* U0,
                             double* out, void* work, int32_t* status_dev, void* stream) {
  g_err.clear();
  if (!B || !Uk || !U0 || !out || !work) return fail(WCNS_EINVAL, "NULL argument");
  if (stage < 1 || stage > 3) return fail(WCNS_EINVAL, "stage %d not in 1..3", stage);
  if (out == Uk) return fail(WCNS_EINVAL, "out must not alias Uk");
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  SweepArgs a;
  BatchArgs b;
  // the live list of the last wcns_batch_cfl on this workspace and tiling,
  // else every tile
  const bool list = B->list_work == work && B->list_tm == B->tm;
  batch_args(B, (double*)((char*)work + B->off_dtp), &a, &b, list ? work : nullptr);
  a.status = status_dev;
  a.U = Uk;
  a.U0 = U0;
  a.out = out;
  a.ca = ca[stage - 1];
  a.cb = cb[stage - 1];
  WCNS_HIP(launch_batch_sweep(a, b, MODE_STAGE, B->tm, (hipStream_t)stream),
           "batch stage launch");
  return WCNS_OK;
}

wcns_status wcns_batch_last_dt(const wcns_batch_plan* B, const void* work, double* dt_dev,
                               void* stream) {
  g_err.clear();
  if (!B || !work || !dt_dev) return fail(WCNS_EINVAL, "NULL argument");
  WCNS_HIP(hipMemcpyAsync(dt_dev, (const char*)work + B->off_dtp, sizeof(double) * B->nprob,
                          hipMemcpyDeviceToDevice, (hipStream_t)stream),
           "copy of the per-problem dt");
  return WCNS_OK;
}

wcns_status wcns_batch_set_graph(wcns_batch_plan* B, int32_t enable) {
  g_err.clear();
  if (!B) return fail(WCNS_EINVAL, "NULL plan");
  B->use_graph = enable != 0;
  return WCNS_OK;
}

int32_t wcns_batch_get_tile(const wcns_batch_plan* B) { return B ? B->tm : 0; }

wcns_status wcns_batch_set_tile(wcns_batch_plan* B, int32_t tile) {
  g_err.clear();
  if (!B) return fail(WCNS_EINVAL, "NULL plan");
  if (!in_list(tile, kTmCandidates, 2) || !sweep_shape_ok(3, 0, tile, 1))
    return fail(WCNS_EINVAL, "tile %d not among the candidates", tile);
  if (tile == B->tm) return WCNS_OK;
  B->tm = tile;
  return batch_build_tiles(B);
}

wcns_status wcns_batch_autotune(wcns_batch_plan* B, const double* U, void* work, void* stream) {
  g_err.clear();
  if (!B || !U || !work) return fail(WCNS_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)work;
  double* out = (double*)(w + B->off_W1);
  hipEvent_t e0, e1;
  WCNS_HIP(hipEventCreate(&e0), "event");
  WCNS_HIP(hipEventCreate(&e1), "event");
  float best = 1e30f;
  int best_tm = B->tm;
  wcns_status st = WCNS_OK;
  for (int tm : kTmCandidates) {
    if ((st = wcns_batch_set_tile(B, tm)) != WCNS_OK) break;
    SweepArgs a;
    BatchArgs b;
    batch_args(B, nullptr, &a, &b);
    a.U = U;
    a.out = out;
    for (int r = 0; r < 4 && st == WCNS_OK; ++r) {
      if (r == 1 && hipEventRecord(e0, s) != hipSuccess) st = fail(WCNS_EDEVICE, "event record");
      hipError_t e = launch_batch_sweep(a, b, MODE_RES, B->tm, s);
      if (e != hipSuccess) st = hip_fail(e, "autotune launch");
    }
    if (st != WCNS_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(WCNS_EDEVICE, "event timing");
      break;
    }
    if (ms < best) {
      best = ms;
      best_tm = tm;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != WCNS_OK) return st;
  return wcns_batch_set_tile(B, best_tm);
}

wcns_status wcns_probe_fp64_fma(double* out, int32_t blocks, int32_t iters, void* stream) {
  g_err.clear();
  if (!out) return fail(WCNS_EINVAL, "NULL argument");
  if (blocks < 1 || iters < 1) return fail(WCNS_EINVAL, "blocks and iters must be >= 1");
  WCNS_HIP(launch_probe_fma(out, blocks, iters, (hipStream_t)stream), "probe launch");
  return WCNS_OK;
}

wcns_status wcns_probe_copy(const double* src, double* dst, int64_t n, void* stream) {
  g_err.clear();
  if (!src || !dst) return fail(WCNS_EINVAL, "NULL argument");
  if (n < 0) return fail(WCNS_EINVAL, "n must be >= 0");
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(WCNS_EINVAL, "src and dst must be 16-byte aligned");
  const double *s0 = src, *s1 = src + n, *d0 = dst, *d1 = dst + n;
  if (n > 0 && s0 < d1 && d0 < s1) return fail(WCNS_EINVAL, "src and dst overlap");
  WCNS_HIP(launch_probe_copy(src, dst, n, (hipStream_t)stream), "probe launch");
  return WCNS_OK;
}

wcns_status wcns_probe_math(const double* x, double* out, int64_t n, int32_t fn, void* stream) {
  g_err.clear();
  if (!x || !out) return fail(WCNS_EINVAL, "NULL argument");
  if (n < 0) return fail(WCNS_EINVAL, "n must be >= 0");
  if (fn < WCNS_MATH_EXP_TAB || fn > WCNS_MATH_SQRT) return fail(WCNS_EINVAL, "unknown function %d", fn);
  WCNS_HIP(launch_probe_math(x, out, n, fn, (hipStream_t)stream), "probe launch");
  return WCNS_OK;
}

const char* wcns_status_string(wcns_status s) {
  switch (s) {
    case WCNS_OK: return "ok";
    case WCNS_EINVAL: return "invalid argument";
    case WCNS_ENOMEM: return "out of memory";
    case WCNS_EDEVICE: return "HIP runtime error";
    case WCNS_ENONPHYS: return "non-physical state";
    case WCNS_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* wcns_last_error(void) { return g_err.c_str(); }

}  // extern "C"
