/*
 * wcns.h -- C ABI of the MI355X (gfx950) WCNS-FE residual library.
 *
 * The library evaluates the semi-discrete residual L(U) = -sum_d dF_d/dx_d
 * (eq. 2 of Liu, Min, Cai, Ma, Yan, "A filtered embedded weighted compact
 * nonlinear scheme for hyperbolic conservation law", arXiv 2306.09760) of
 * scalar advection or the Euler equations (eq. 31-32) on uniform 1D/2D/3D
 * grids, and advances it with the three-stage SSP Runge-Kutta scheme.  The
 * residual is, per direction and per midpoint: Roe-averaged characteristic
 * projection, the fifth-order nonlinear interpolation to the midpoint
 * (eq. 5-6) with JS (eq. 11), Z (eq. 14-15) or filtered-embedded (FE,
 * eq. 20-21 and the coefficient table of Sec. 3.1; PFE switch of App. A)
 * weights, a local Lax-Friedrichs midpoint flux, and the sixth-order
 * midpoint-and-node flux difference (or eq. 3's midpoint-only difference).
 *
 * Conventions for every entry point
 *  - Array arguments named U, R, Ubar, Rbar, lambda, work, *_dev are DEVICE
 *    pointers on the current HIP device, owned by the caller (allocate them
 *    with hipMalloc or PyTorch); the library never frees caller memory.
 *    Arguments named *_host are host pointers read during the call only.
 *  - States are float64, variable-major and x-fastest:
 *    U[v*npts + x + nx*(y + ny*z)], npts = nx*ny*nz.  Euler variables are
 *    (rho, rho*u, rho*v, rho*w, E) truncated to ndim + 2; advection has one.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work; none synchronises the device unless stated.
 *  - Host-side validation failures return WCNS_EINVAL before anything is
 *    enqueued; wcns_last_error() then describes the problem.  Device-side
 *    problems (a non-finite value, rho <= 0 or p <= 0 after a stage) are
 *    OR-ed into *status_dev (bit 0) and surface when the caller reads it;
 *    bit 1 reports a capped batch launch shorter than its live-tile list
 *    (wcns_batch_rk3_steps_capped).
 *  - No exception or abort crosses this interface.  A plan must not be used
 *    by two host threads at once, and two calls that share a workspace must
 *    not overlap on the device.
 */
#ifndef WCNS_H
#define WCNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WCNS_OK = 0,
  WCNS_EINVAL = -1,       /* invalid argument (checked on the host)        */
  WCNS_ENOMEM = -2,       /* host or device allocation failed               */
  WCNS_EDEVICE = -3,      /* a HIP runtime call failed                      */
  WCNS_ENONPHYS = -4,     /* value of a status word with bit 0 set          */
  WCNS_EUNSUPPORTED = -5  /* valid but not implemented combination          */
} wcns_status;

typedef enum { WCNS_SYS_ADVECTION = 0, WCNS_SYS_EULER = 1 } wcns_system;
typedef enum { WCNS_BC_PERIODIC = 0, WCNS_BC_TRANSMISSIVE = 1 } wcns_bc;
/* JS: eq. 11.  Z: eq. 14-15.  FE: eq. 20-21 applied to the Z weights, then
   renormalised.  PFE: App. A (FE only outside the |w_k - d_k| <= cv band).
   LINEAR: the ideal weights d = (1/16, 10/16, 5/16) of Sec. 2. */
typedef enum {
  WCNS_W_JS = 0, WCNS_W_Z = 1, WCNS_W_FE = 2, WCNS_W_PFE = 3, WCNS_W_LINEAR = 4
} wcns_weights;
/* MND6: (3/2, -3/10, 1/30) midpoint-and-node difference (WCNS-MND, Sec. 1).
   MD6: eq. 3, midpoint-only (75/64, -25/384, 3/640). */
typedef enum { WCNS_DIFF_MND6 = 0, WCNS_DIFF_MD6 = 1 } wcns_diff;
/* WCNS: interpolation of the (characteristic) state to the midpoints, local
   Lax-Friedrichs flux there and the MND6 / MD6 difference (Sec. 2).
   WENO: the filtered embedded WENO scheme of App. B: finite-difference
   WENO5 reconstruction of the Lax-Friedrichs split flux f+- = (F +- alpha U)/2
   (alpha: largest wave speed over the six stencil nodes), ideal weights
   (1/10, 6/10, 3/10) of Table B.1, FE map with the coefficients of Table B.2,
   conservative difference (F_{i+1/2} - F_{i-1/2}) / h (`diff` unused).  The
   weights, eps, xi, kappa, cv and z_power fields apply to both. */
typedef enum { WCNS_SCHEME_WCNS = 0, WCNS_SCHEME_WENO = 1 } wcns_scheme;

typedef struct wcns_desc {
  int32_t struct_size;   /* = sizeof(wcns_desc)                                */
  int32_t system;        /* wcns_system                                        */
  int32_t ndim;          /* 1, 2 or 3                                          */
  int32_t weights;       /* wcns_weights                                       */
  int64_t n[3];          /* nodes per axis; axes >= ndim must be 1; each used
                            axis needs n >= 9                                  */
  double h[3];           /* grid spacing per used axis, > 0                    */
  double adv_speed[3];   /* advection speed per axis (advection only)          */
  int32_t bc[3];         /* wcns_bc per used axis (same at both ends)          */
  int32_t diff;          /* wcns_diff                                          */
  double gamma;          /* ratio of specific heats, > 1 (Euler)               */
  double eps;            /* epsilon of eq. 11 / eq. 14 (paper: 1e-40), >= 0    */
  double xi;             /* steepness of eq. 20 (paper: 100; 1e6 in Sec. 3.2)  */
  double kappa;          /* null-point parameter of eq. 20 (paper: 0.5)        */
  double cv;             /* PFE switch value of App. A (paper: 1e-3)           */
  int32_t z_power;       /* exponent p of eq. 14, 1..4 (paper leaves it open)  */
  int32_t char_proj;     /* 1: characteristic projection, 0: component-wise    */
  int32_t scheme;        /* wcns_scheme (residual_adjoint, rk3_step_adjoint and
                            the batch support WCNS only: WCNS_EUNSUPPORTED)    */
  int32_t reserved_;     /* 0                                                  */
} wcns_desc;

typedef struct wcns_plan wcns_plan;
typedef struct wcns_batch_plan wcns_batch_plan;

/* Fills *d with the defaults: Euler, 1D, FE weights, MND6, eps = 1e-40,
   xi = 100, kappa = 0.5, cv = 1e-3, p = 2, gamma = 1.4, characteristic
   projection on, periodic.  n and h must still be set. */
void wcns_desc_init(wcns_desc* d);

/* Validates *desc and creates a plan on the current device.  Allocates no
   device memory and does not synchronise.  Errors: WCNS_EINVAL. */
wcns_status wcns_plan_create(const wcns_desc* desc, wcns_plan** plan);
wcns_status wcns_plan_destroy(wcns_plan* plan);

/* Number of float64 values in one state: nv * nx * ny * nz. */
int64_t wcns_state_elems(const wcns_plan* plan);
/* Bytes of device workspace `work` that the calls below need (the caller
   allocates it; 256-byte aligned). */
size_t wcns_workspace_bytes(const wcns_plan* plan);

/* R = L(U): one residual evaluation (all directions).  U and R must not
   overlap.  Uses `work`.  Graph-capturable. */
wcns_status wcns_residual(wcns_plan* plan, const double* U, double* R, void* work,
                          void* stream);

/* *dt_dev = cfl / max_i sum_d (|u_d| + c) / h_d over U (for advection
   sum_d |a_d| / h_d).  Two deterministic kernels (block maxima, then one
   block).  Graph-capturable. */
wcns_status wcns_cfl_dt(wcns_plan* plan, const double* U, double cfl, double* dt_dev,
                        void* work, void* stream);

/* One SSP-RK3 step in place: U <- U^{n+1}.  If dt_dev is NULL the step is
   cfl-limited (computed on the device from U^n and left in the workspace);
   otherwise *dt_dev is used.  status_dev may be NULL; otherwise bit 0 is
   OR-ed in when a stage produced a non-finite value or rho <= 0 or p <= 0.
   No host synchronisation: graph-capturable. */
wcns_status wcns_rk3_step(wcns_plan* plan, double* U, void* work, const double* dt_dev,
                          double cfl, int32_t* status_dev, void* stream);

/* wcns_rk3_step for callers that cannot allocate (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the same
   step, the same kernels and bitwise the same result, with no workspace
   argument.  The stage states, the residual accumulator (2D/3D), the CFL
   block maxima and dt live in a device array inside the library, 48 MiB
   per GPU, held until the process ends: the plan must need at most that
   (2 states, 3 in 2D/3D, plus 16.25 KB: a state of up to about 3.1 M
   doubles in 1D and 2.1 M in 2D/3D), else WCNS_EINVAL before anything is
   enqueued.
   The call allocates nothing (no hipMalloc, no hipFree; the first call on a
   device looks up the array's address there).  Every call on one GPU uses
   the same array: calls that overlap on the device (two streams, two host
   threads) race and must not be issued; nothing in the array needs to be
   zero beforehand (every buffer is written before it is read).  dt_dev,
   cfl, status_dev and stream as for wcns_rk3_step.  Graph-capturable. */
wcns_status wcns_rk3_step_noalloc(wcns_plan* plan, double* U, const double* dt_dev, double cfl,
                                  int32_t* status_dev, void* stream);

/* wcns_rk3_step that also leaves its stage states: U1 <- U^(1) = U^n + dt
   L(U^n), U2 <- U^(2) = 3/4 U^n + 1/4 (U^(1) + dt L(U^(1))), then U <-
   U^{n+1}.  U1, U2: device arrays of wcns_state_elems doubles owned by the
   caller, distinct from U and from each other (WCNS_EINVAL otherwise); kept
   for wcns_rk3_step_adjoint_stages, which then needs no recomputation.  The
   step itself is identical to wcns_rk3_step.  Graph-capturable. */
wcns_status wcns_rk3_step_stages(wcns_plan* plan, double* U, double* U1, double* U2, void* work,
                                 const double* dt_dev, double cfl, int32_t* status_dev,
                                 void* stream);

/* One step in place of the four-stage Runge-Kutta scheme of eq. 16 (the
   paper's integrator, classical RK4): u1 = u + dt/2 L(u), u2 = u + dt/2
   L(u1), u3 = u + dt L(u2), u <- -u/3 + u1/3 + 2 u2/3 + u3/3 + dt/6 L(u3).
   dt_dev, cfl and status_dev as for wcns_rk3_step (the paper runs it at CFL
   0.3).  Uses `work` (three stage states and one combination buffer).  No
   host synchronisation: graph-capturable. */
wcns_status wcns_rk4_step(wcns_plan* plan, double* U, void* work, const double* dt_dev,
                          double cfl, int32_t* status_dev, void* stream);

/* Statistics of the nonlinear weights (App. A): adds to hist the counts of
   every interpolation one residual evaluation of U performs (each
   direction, each distinct midpoint the difference reads, each field, the
   left and the mirrored right stencil).  hist is a device array of
   3 x 3 x nbins uint64 counters, [kind][k][bin], kind 0 = the normalised
   JS/Z weights omega_k, kind 1 = their FE images g_k(omega_k) / sum_l
   g_l(omega_l), kind 2 = the weights the plan's scheme uses (PFE: after the
   switch); bin b covers [b/nbins, (b+1)/nbins) (1.0 in the last bin).  The
   caller zeroes hist; counts accumulate over calls.  nbins in [1, 2^24].
   A diagnostic pass (atomics), not part of the residual. */
wcns_status wcns_weight_histogram(wcns_plan* plan, const double* U, uint64_t* hist,
                                  int32_t nbins, void* stream);

/* Ubar += (dL/dU)^T Rbar at state U: the exact vector-Jacobian product of
   the residual, including the weights, the FE mapping, the Roe-averaged
   projection and the flux (conventions at non-smooth points: d|x|/dx = 0
   at 0, a tie in max goes to the first argument).  Deterministic
   (gather form, no atomics).  Uses `work`. */
wcns_status wcns_residual_adjoint(wcns_plan* plan, const double* U, const double* Rbar,
                                  double* Ubar, void* work, void* stream);

/* Reverse of one SSP-RK3 step at fixed *dt_dev: recomputes the two stage
   states from Un and replaces lambda (in: adjoint of U^{n+1}) by the
   adjoint of U^n.  Uses `work`.  lambda must not overlap Un or `work`
   (WCNS_EINVAL). */
wcns_status wcns_rk3_step_adjoint(wcns_plan* plan, const double* Un, double* lambda,
                                  void* work, const double* dt_dev, void* stream);

/* wcns_rk3_step_adjoint from the stage states U1, U2 that
   wcns_rk3_step_stages wrote for the step from Un with the same *dt_dev:
   the same reverse sweep without recomputing the two stage states (two
   residual evaluations fewer).  Uses `work`.  lambda must not overlap Un,
   U1, U2 or `work`, and U1, U2 may lie in `work` only outside the two
   cotangent buffers the reverse step keeps there (in practice: pass caller
   arrays; WCNS_EINVAL otherwise). */
wcns_status wcns_rk3_step_adjoint_stages(wcns_plan* plan, const double* Un, const double* U1,
                                         const double* U2, double* lambda, void* work,
                                         const double* dt_dev, void* stream);

/* Measures the candidate tile shapes of this plan's kernels on U (timed with
   HIP events; synchronises the stream) and keeps the fastest in the plan and
   in a per-process cache keyed by shape.  U is not modified.  A WENO plan
   has one compiled shape: the call returns WCNS_OK and changes nothing. */
wcns_status wcns_plan_autotune(wcns_plan* plan, const double* U, void* work, void* stream);
/* Current tile shapes: [0] midpoints per tile of the x sweep (128 or 256);
   [1], [2] midpoints along the line and adjacent x-columns per tile of the
   y/z sweeps, one of (16,8), (32,4), (32,8), (64,4), (128,2), (256,1). */
void wcns_plan_get_tiles(const wcns_plan* plan, int32_t tiles[3]);
/* Sets tile shapes (WCNS_EINVAL if not among the candidates or if the tile
   would exceed 64 KB of LDS for this system). */
wcns_status wcns_plan_set_tiles(wcns_plan* plan, const int32_t tiles[3]);

/* ----- ragged batch of independent 1D problems (one launch per
   stage; one graph-captured step) --------------------------------------- */
/* proto: a 1D descriptor (its n[0] and h[0] are ignored).  Problem p holds
   offsets_host[p+1] - offsets_host[p] >= 9 nodes at columns
   offsets_host[p] .. offsets_host[p+1]-1 of every variable of the batch
   state U[v*total + column], total = offsets_host[nprob]; its spacing is
   h_host[p].  The library copies offsets and h to small device tables of
   its own (synchronously; freed by wcns_batch_plan_destroy). */
wcns_status wcns_batch_plan_create(const wcns_desc* proto, int64_t nprob,
                                   const int64_t* offsets_host, const double* h_host,
                                   wcns_batch_plan** plan);
wcns_status wcns_batch_plan_destroy(wcns_batch_plan* plan);
int64_t wcns_batch_state_elems(const wcns_batch_plan* plan);
size_t wcns_batch_workspace_bytes(const wcns_batch_plan* plan);

/* R = L(U) of every problem (per-problem spacing and boundaries). */
wcns_status wcns_batch_residual(wcns_batch_plan* plan, const double* U, double* R,
                                void* work, void* stream);

/* One SSP-RK3 step of every problem whose time t_dev[p] < t_end, each with
   its own dt_p = min(cfl-limited step, t_end - t_dev[p]); t_dev[p] += dt_p.
   Finished problems are left untouched.  status_dev as in wcns_rk3_step;
   a problem whose maximum wave rate is not a positive finite number (its
   state went non-physical) is stopped where it is: dt_p = 0, t_dev[p]
   unchanged, bit 0 of *status_dev set.  The stage kernels take only the
   tiles of problems with dt_p > 0 (a list that the step builds in `work`
   after computing dt_p), so finished problems cost nothing.
   With wcns_batch_set_graph(plan, 1) the step's kernels are captured into
   a HIP graph on first use (for the given pointers and scalars) and
   replayed afterwards. */
wcns_status wcns_batch_rk3_step(wcns_batch_plan* plan, double* U, void* work, double* t_dev,
                                double t_end, double cfl, int32_t* status_dev, void* stream);
wcns_status wcns_batch_set_graph(wcns_batch_plan* plan, int32_t enable);
/* Copies the step size dt_p each problem took in the last step (or that the
   last wcns_batch_cfl set; 0 for a finished or stopped problem) from `work`
   to dt_dev, a device array of nprob doubles: an asynchronous
   device-to-device copy on `stream`. */
wcns_status wcns_batch_last_dt(const wcns_batch_plan* plan, const void* work, double* dt_dev,
                               void* stream);
/* nsteps >= 0 calls of wcns_batch_rk3_step in one (never graph-captured):
   the same states and times bit for bit for physical states.  Each step's
   dt_p still comes from the CFL bound on that step's starting state (the
   time-step restriction of the scheme, Sec. 4); from the second step on,
   the maximum wave rate of problem p is taken by the previous step's last
   stage as it writes the state, instead of by a separate pass over U.  U
   must not be changed by others during the call's execution.  Returns
   WCNS_EINVAL for nsteps < 0 or the arguments wcns_batch_rk3_step rejects. */
wcns_status wcns_batch_rk3_steps(wcns_batch_plan* plan, double* U, void* work, double* t_dev,
                                 double t_end, double cfl, int32_t nsteps, int32_t* status_dev,
                                 void* stream);

/* The length of the live-tile list in `work` (the tiles of the problems
   with dt_p > 0 at the last rebuild), copied to the host *count: blocks
   until the work on `stream` is done.  WCNS_EINVAL if `work` holds no list
   for the plan's current tile size (no wcns_batch_cfl, wcns_batch_rk3_step
   or wcns_batch_rk3_steps on it since the last tile change). */
wcns_status wcns_batch_live_tiles(const wcns_batch_plan* plan, const void* work, int32_t* count,
                                  void* stream);

/* wcns_batch_rk3_steps with every stage launch sized to max_live
   workgroups instead of one per tile: near the end of a run, when few
   problems are live, the full-size launches spend most of their time on
   workgroups that only read the list's length and leave (4096 tubes of
   256-4096 nodes: ~35 000 tiles, ~20 us per step of such launches).  The caller
   bounds the list: within one run towards a fixed t_end problems only
   finish, so a count from wcns_batch_live_tiles, taken after any earlier
   step of that run, bounds every later list.  A launch whose list is
   longer than max_live sets bit 1 (value 2) of *status_dev (required
   here) and leaves tiles out of that stage.  WCNS_EINVAL for max_live < 1
   or a NULL status_dev, else as wcns_batch_rk3_steps. */
wcns_status wcns_batch_rk3_steps_capped(wcns_batch_plan* plan, double* U, void* work,
                                        double* t_dev, double t_end, double cfl, int32_t nsteps,
                                        int32_t* status_dev, int32_t max_live, void* stream);

/* The two kernels of wcns_batch_rk3_step, for callers composing their own
   step.  wcns_batch_cfl: per-problem dt_p (as above) into the workspace and
   t_dev[p] += dt_p.  wcns_batch_stage: SSP-RK3 stage `stage` (1, 2 or 3) of
   every problem with dt_p > 0, out = a*U0 + b*(Uk + dt_p*L(Uk)) with
   (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3); Uk, U0 and out are batch states,
   out may alias U0 but not Uk.  dt_p is the one the last wcns_batch_cfl
   (or wcns_batch_rk3_step) left in `work`, and so is the list of live
   tiles the stage takes (every tile, if the tile size changed since). */
wcns_status wcns_batch_cfl(wcns_batch_plan* plan, const double* U, void* work, double* t_dev,
                           double t_end, double cfl, void* stream);
wcns_status wcns_batch_stage(wcns_batch_plan* plan, int32_t stage, const double* Uk,
                             const double* U0, double* out, void* work, int32_t* status_dev,
                             void* stream);
/* Candidate midpoints per tile (128, 256) are timed on U as in
   wcns_plan_autotune. */
wcns_status wcns_batch_autotune(wcns_batch_plan* plan, const double* U, void* work,
                                void* stream);
int32_t wcns_batch_get_tile(const wcns_batch_plan* plan);
wcns_status wcns_batch_set_tile(wcns_batch_plan* plan, int32_t tile);

/* ----- roof probes (measurement of the machine, not part of the method) -- */
/* FP64 vector-FMA throughput: `blocks` workgroups of 256 lanes each run
   `iters` rounds of eight independent chains x <- fma(x, 1 - 2^-30, 2^-30)
   (16 flops per lane per round) from x0 = 1 + (g mod 1024)/1024 + k/16
   (g the lane's global index, k the chain) and write each lane's sum of its
   chains to out[g] (device, blocks * 256 doubles).  The caller times it.
   WCNS_EINVAL for a NULL out or blocks, iters < 1. */
wcns_status wcns_probe_fp64_fma(double* out, int32_t blocks, int32_t iters, void* stream);
/* HBM streaming copy dst[i] = src[i], i < n, 16 bytes per lane per access
   (device arrays, 16-byte aligned, not overlapping; WCNS_EINVAL otherwise).
   The caller times it: 16 n bytes move. */
wcns_status wcns_probe_copy(const double* src, double* dst, int64_t n, void* stream);
/* The device's elementary functions, out[i] = f(x[i]) for i < n (device
   arrays of doubles, owned by the caller), so that their error bounds can be
   checked against a reference: e^z through the 2^(k/64) table (Tang's
   method, |z| <= 708), e^z by Cody-Waite reduction and a degree-13 Taylor
   polynomial (|z| <= 708), 1/x with two and with one Newton step from the
   hardware seed (x normal), and the square root of 0 or of x in
   [2^-760, inf).  These are the exponentials, reciprocals and square roots
   of the residual (Sec. 2, eq. 20; the Roe average and the fluxes).
   WCNS_EINVAL for a NULL pointer, n < 0 or an unknown fn. */
typedef enum {
  WCNS_MATH_EXP_TAB = 0,
  WCNS_MATH_EXP_CW = 1,
  WCNS_MATH_RCP = 2,
  WCNS_MATH_RCP1 = 3,
  WCNS_MATH_SQRT = 4
} wcns_math_fn;
wcns_status wcns_probe_math(const double* x, double* out, int64_t n, int32_t fn, void* stream);

const char* wcns_status_string(wcns_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char* wcns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WCNS_H */
