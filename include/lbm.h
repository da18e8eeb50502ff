/*
 * lbm.h - C ABI of the MI355X (gfx950) library for the wall-modelled MRT
 * lattice Boltzmann channel with a synthetic-turbulence-generator inlet
 * (Xue, Yao, Davidson, arXiv 2304.04214).
 *
 * Conventions
 *  - Every call returns lbm_status (0 = LBM_OK).  Nothing throws or aborts
 *    across the ABI.  Argument and shape errors are returned synchronously;
 *    errors detected on the device (non-finite or non-positive density, inlet
 *    Mach limit, invalid Reynolds stresses or per-row spectrum inputs of a
 *    bound lbm_stg) are
 *    latched in a device word and returned by lbm_sync() or
 *    lbm_stats(LBM_STATS_READ).
 *  - Pointers named "device" are HIP device pointers.  Population and
 *    outlet-history buffers are CALLER-OWNED: the library never frees them,
 *    and they must outlive the work enqueued on them.  The handle owns only
 *    small tables (STG trigonometric tables, Cholesky factors, statistics
 *    accumulators, an error word).
 *  - All work is enqueued, in order, on the HIP stream given to lbm_create()
 *    (asynchronous to the host).  A handle is not thread-safe.
 *  - Lattice: x streamwise (nx), y wall-normal (ny), z spanwise (nz, periodic).
 *    Node (x, y, z) has linear index n = (x*ny + y)*nz + z in every
 *    node-field argument ("SoA [c][N]": component c of node n at c*N + n,
 *    N = nx*ny*nz).  i is the D3Q19 index in the paper's order (Sec. II.A,
 *    Eq. (1): lexicographic in (c_z, c_y, c_x), opposite of i is 18 - i).
 *  - Population buffers use 64-node bricks: with zc = ceil(nz/64), population
 *    i of node (x, y, z) is element ((x*zc + z/64)*ny + y)*1216 + 64*i + z%64
 *    (1216 = 19*64); a buffer holds 19*nx*ny*zc*64 elements (lbm_state_elems).
 *    Elements of the padding nodes z >= nz are never read.  lbm_import_f32 /
 *    lbm_export_f32 convert from / to SoA float [19][N].  The stored state is
 *    the post-collision population set s_n of time n.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx* lbm_handle;

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = 1,       /* bad argument (NULL, out of range, unsupported combination) */
  LBM_ERR_SHAPE = 2,     /* sizes out of range or buffers misaligned */
  LBM_ERR_HIP = 3,       /* a HIP runtime call failed */
  LBM_ERR_MACH = 4,      /* inlet |u_in,x| >= 0.3 c_s (Sec. III.A, below Eq. (30)) */
  LBM_ERR_NONFINITE = 5, /* a node's density became non-finite or non-positive */
  LBM_ERR_STATE = 6      /* call out of order (no STG bound, statistics not attached, ...) */
} lbm_status;

enum { LBM_STORE_F32 = 0, LBM_STORE_F16DEV = 1 };
enum { LBM_Y_PERIODIC = 0, LBM_Y_BOUNCEBACK = 1, LBM_Y_SLIP = 2 };
enum { LBM_X_PERIODIC = 0, LBM_X_INFLOW = 1 };
enum { LBM_OUTLET_CONVECTIVE = 0, LBM_OUTLET_ZERO_GRADIENT = 1 };
enum { LBM_WALL_REICHARDT = 0, LBM_WALL_MUSKER = 1 };
enum { LBM_WALL_AVG_LOCAL = 0, LBM_WALL_AVG_LINE = 1 };
enum { LBM_STATS_ATTACH = 1, LBM_STATS_DETACH = 2, LBM_STATS_RESET = 3, LBM_STATS_READ = 4, LBM_STATS_READ_WALL = 5 };

/*
 * Problem statement (Sec. II, Sec. IV.A).
 *  storage     LBM_STORE_F32: populations as float.  LBM_STORE_F16DEV:
 *              populations stored as IEEE half deviations h_i = f_i - w_i
 *              (rounded to nearest even); collision is computed in float.
 *  ywall       walls halfway below y = 0 and above y = ny-1: LBM_Y_SLIP is the
 *              paper's slip wall (specular reflection), LBM_Y_BOUNCEBACK is
 *              halfway bounce-back; LBM_Y_PERIODIC has no walls.
 *  xbc         LBM_X_INFLOW: STG inlet at x = 0 (regularised populations,
 *              Sec. III.A, Eq. (26)-(31)) and an outlet at x = nx-1 for the
 *              unknown c_x < 0 populations (Sec. IV.A calls it pressure-free;
 *              the rule is a reading):
 *  outlet      LBM_OUTLET_CONVECTIVE: f_i = (f_i^prev + u_conv f_i(x-1)) /
 *              (1 + u_conv); LBM_OUTLET_ZERO_GRADIENT: f_i = f_i(x-1) (the
 *              limit u_conv -> infinity), with f(x-1) the post-streaming value.
 *  wall_law    the law of the wall in Eq. (20): LBM_WALL_REICHARDT (Eq. (16),
 *              with kappa and b_reich) or LBM_WALL_MUSKER (the explicit profile of
 *              Musker's law that Sec. II.C names as the alternative:
 *              u+ = 5.424 atan((2y+ - 8.15)/16.7) + log10((y+ + 10.6)^9.6 /
 *              (y+^2 - 8.15y+ + 86)^2) + C, with C = -3.5113 so that u+(0) = 0;
 *              the rounded -3.52 often printed would leave no positive u_tau
 *              below y+ = 0.009).
 *  wall_avg    LBM_WALL_AVG_LOCAL: u_tau from each cell's own u_hat (Sec. II.C);
 *              LBM_WALL_AVG_LINE: the plane-averaged u_tau that Sec. II.C
 *              contrasts with its local one, averaged over the homogeneous
 *              direction z of each wall line (x, wall): u_hat = u_w . e_x
 *              (Eq. (19); 0 where u_2 has no tangential part) is averaged over
 *              z in the same step, Eq. (20) is solved once per line for the
 *              mean's magnitude, and each cell of the line takes
 *              F_w = -sign(mean) rho u_tau^2 e_x with its own rho and e_x; the
 *              wall statistics then report the line's u_tau at every cell.
 *              Costs one extra launch per step reading the two rows next to
 *              each wall (lbm_adjoint_step: two, over the wall blocks).
 *  wall_model  1: Reichardt wall force in the first off-wall cells (Sec. II.C,
 *              Eq. (16)-(21)), u_tau by newton_iters Newton steps from the
 *              viscous-sublayer estimate (0: 4; in FP32 the iteration reaches
 *              rounding level after three steps for nu0 in [1e-5, 2e-2] and
 *              |u_hat| in [1e-6, 0.3]).
 *  tau0        molecular relaxation time (> 1/2), nu0 = (tau0 - 1/2)/3 (Eq. (5)).
 *  cs_smag     Smagorinsky C_s, C_smag = C_s^2 (Sec. II.B).  0 disables it.
 *  s[19]       MRT relaxation rates (Appendix A.1); s[9], s[11], s[13], s[14],
 *              s[15] are replaced per node by 1/tau_eff (Eq. (15)).
 *  kappa, b_reich, y_wall  Reichardt constants (0.41, 7.8) and the distance of
 *              the first cell centre from the wall (0.5).
 *  u_conv      outlet convection speed.
 *  g[3]        uniform body acceleration; force density rho g (Eq. (9), (11)).
 *  sponge_cells, sponge_nu  outlet sponge (Sec. IV.A; its law is not given
 *              there, this is the library's reading): over the last
 *              sponge_cells x planes the molecular viscosity rises as
 *              nu(x) = nu0 + (sponge_nu - nu0) r^2, r = (x - nx + sponge_cells + 1)
 *              / sponge_cells, i.e. tau0(x) = 1/2 + 3 nu(x).  0 cells: no sponge;
 *              otherwise LBM_X_INFLOW, sponge_cells <= nx - 1, sponge_nu > 0.
 */
typedef struct {
  int32_t nx, ny, nz;
  int32_t storage;
  int32_t ywall;
  int32_t xbc;
  int32_t wall_model;
  int32_t newton_iters;
  int32_t sponge_cells;
  int32_t outlet;
  int32_t wall_law;
  int32_t wall_avg;
  double tau0;
  double cs_smag;
  double s[19];
  double kappa, b_reich, y_wall;
  double u_conv;
  double g[3];
  double sponge_nu;
} lbm_config;

/*
 * Inlet synthetic turbulence (Sec. III.A, Eq. (22)-(25)).  All pointers are
 * device pointers; the arrays are read when the table is bound (every call
 * that receives a non-NULL lbm_stg binds it again).
 *  q[N], sigma[3][N], kmag[N], d[3][N], phi[N], omega[N]   mode table: weights
 *      (sum 1), unit amplitude directions (sigma . d = 0), wavenumbers, unit
 *      wave directions, phases, temporal frequencies (rad per step).  The mode
 *      phase at inlet node (y, z) and time t is
 *      kmag (d_y (y + 1/2) + d_z z) + omega t + phi.
 *  u_rans[3][ny]  mean inflow;  R[6][ny] Reynolds stresses (R11 R21 R22 R31 R32 R33,
 *      symmetric positive definite: a row that is not, or holds a non-finite
 *      entry, is reported as LBM_ERR_ARG by the next lbm_sync and takes a zero
 *      factor, u' = 0); amp_bin[n_bins] amplitude scalings s_b;
 *      bin_of_y[ny] bin of each row.  u' = s_b(y) a(y) v', a = chol(R).
 *  k_rans[ny], omega_rans[ny]   optional (both NULL or both set): RANS
 *      turbulent kinetic energy and specific dissipation rate of each inlet
 *      row.  When set, q is not read: each row y takes its own weights
 *      q^n(y) = E(k_n; y) dk_n / sum_m E(k_m; y) dk_m from the modified von
 *      Karman spectrum of the STG that Eq. (25) cites,
 *        E(k) = (k/k_e)^4 / (1 + 2.4 (k/k_e)^2)^(17/6) exp(-(12 k/k_eta)^2)
 *               exp(-(4 max(k - 0.9 k_cut, 0)/k_cut)^3),
 *      k_e = 2 pi / min(2 d_w, 3 sqrt(k)/(0.09 omega)), k_eta = 2 pi / eta,
 *      eta = (nu0^3 / (0.09 k omega))^(1/4), k_cut = pi (l_cut = 2 cells), d_w =
 *      min(y + 1/2, ny - y - 1/2), dk_n centred differences of kmag (one-sided
 *      at the ends).  kmag must then be strictly ascending and k, omega
 *      positive, and the y walls must not be periodic (LBM_ERR_ARG: the
 *      lattice's y walls, at bind time; the table values, reported by the
 *      next lbm_sync, with the rows' weights left unspecified).
 *  u_in[3][ny][nz]   (written) inlet velocity plane;  fluct[3][ny][nz] (written,
 *      optional, may be NULL) a(y) v' before the s_b scaling.
 *  1 <= n_modes <= LBM_MAX_MODES.
 */
#define LBM_MAX_MODES 1024
typedef struct {
  int32_t n_modes, n_bins;
  const double *q, *sigma, *kmag, *d, *phi, *omega;
  const double *u_rans, *R, *amp_bin;
  const int32_t* bin_of_y;
  const double *k_rans, *omega_rans;
  float* u_in;
  float* fluct;
} lbm_stg;

/* Number of elements of one population buffer for cfg (19*nx*ny*zc*64);
   validates cfg like lbm_create (no device work). */
lbm_status lbm_state_elems(const lbm_config* cfg, int64_t* elems);

/*
 * Create a handle.  f_a, f_b: device population buffers of lbm_state_elems()
 * elements (float for LBM_STORE_F32, 16-bit for LBM_STORE_F16DEV), 256-byte
 * aligned; the state lives in f_a first and moves between the two each step.
 * hist_a, hist_b: device float buffers [5][ny][nz] for the outlet history
 * (required when xbc = LBM_X_INFLOW, else may be NULL), alternating with the
 * populations.  hip_stream: the hipStream_t all work goes on (NULL = default).
 * Limits: nx >= 1 (>= 3 with LBM_X_INFLOW), ny >= 4, nz >= 1, N < 2^31,
 * lbm_state_elems() < 2^32.
 */
lbm_status lbm_create(const lbm_config* cfg, void* f_a, void* f_b, float* hist_a, float* hist_b,
                      void* hip_stream, lbm_handle* out);
lbm_status lbm_destroy(lbm_handle h);

/* Point the handle at another pair of buffers (checkpoint restore); the state
   is taken to be in f_a / hist_a at time index `time`. */
lbm_status lbm_set_state(lbm_handle h, void* f_a, void* f_b, float* hist_a, float* hist_b, int64_t time);
/* The buffers that currently hold the state, and its time index n. */
lbm_status lbm_get_state(lbm_handle h, void** f_cur, float** hist_cur, int64_t* time);

/*
 * Initial state f_i = f_eq_i(rho, u) + eps w_i pert_i (second-order
 * equilibrium, Sec. III.A Eq. (27)), written into the current buffer; the
 * outlet history is taken from the same state at x = nx-1.  rho [N] (NULL:
 * 1), u [3][N], pert [19][N] (NULL: none): device float arrays.
 */
lbm_status lbm_init_equilibrium(lbm_handle h, const float* rho, const float* u, const float* pert, float eps);
/* The same from device double arrays, the equilibrium formed in FP64 and
   rounded once to the storage (with FP16 storage, the deviation f - w - r
   formed in FP64): a state that matches an FP64 computation of Eq. (27) from
   the same fields up to that rounding. */
lbm_status lbm_init_equilibrium_f64(lbm_handle h, const double* rho, const double* u, const double* pert,
                                    double eps);

/* Mean inflow U(y) = u_tau u+(d u_tau / nu0), d = min(y + 1/2, ny - y - 1/2),
   with the Reichardt law of Sec. II.C; writes device double u_rans[3][ny]. */
lbm_status lbm_inflow_reichardt(lbm_handle h, double u_tau, double* u_rans);

/*
 * Inlet velocity at time t (Algorithm 1 steps 4-5, Eq. (22)-(25)) into
 * stg->u_in (and stg->fluct).  Binds stg when non-NULL.  Mach violations are
 * latched (LBM_ERR_MACH at the next lbm_sync()).
 */
lbm_status stg_inlet_fill(lbm_handle h, const lbm_stg* stg, double t);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): stg_inlet_fill
 * without any device allocation or free.  The inputs stg (required) are bound
 * for this call only, into the library's static device scratch of
 * LBM_NOALLOC_STG_BYTES per device (held from the first lbm_create on that
 * device until the process ends), and the plane at time t is written to
 * stg->u_in (and stg->fluct); the handle's own bound inputs and tables are
 * neither read nor changed.  The tables need
 * 8 N nz + 20 N + 40 ny bytes (+ 4 ny N with k_rans / omega_rans), each of the
 * seven rounded up to 256: LBM_ERR_SHAPE when that exceeds the scratch (e.g.
 * N = 1024 modes with nz = 512).  Every table is written by the call before it
 * is read, so nothing must start at zero.  All calls on one device share its
 * scratch: calls whose work can overlap in time (other streams, other threads)
 * race and must not be issued; calls ordered on one stream are safe.  Errors as
 * stg_inlet_fill (LBM_ERR_ARG for invalid inputs; device-detected ones at the
 * next lbm_sync).  Asynchronous on the handle's stream.
 */
#define LBM_NOALLOC_STG_BYTES (4u << 20)
lbm_status stg_inlet_fill_noalloc(lbm_handle h, const lbm_stg* stg, double t);

/*
 * Advance nsteps time steps (Algorithm 1): for each step n -> n+1 the inlet
 * plane is filled for t = n+1 (when xbc = LBM_X_INFLOW), then one fused
 * pull-stream / boundary / wall-model / MRT-Smagorinsky collision runs over
 * all nodes, on the handle's stream.  With LBM_STORE_F16DEV the blocks away
 * from the inlet, outlet and statistics planes (wall rows included) run in a
 * lean kernel after a general kernel for the other blocks (one fused launch on
 * lattices of up to 2^24 nodes); with LBM_STORE_F32 the general kernel covers
 * all blocks, one dispatch per range of x-planes (lbm_collide_dispatches).
 * stg: bound when non-NULL; required (now or earlier) with LBM_X_INFLOW.
 * Asynchronous on the handle's stream.
 */
lbm_status lbm_step(lbm_handle h, const lbm_stg* stg, int32_t nsteps);

/* Streaming with the wall rules only, current buffer -> other buffer, no
   collision; populations with no source (outside the x range) are set to -1.
   The state then lives in the other buffer (time index unchanged).
   LBM_STORE_F32 only. */
lbm_status lbm_stream_only(lbm_handle h);

/* Current state as float populations, SoA [19][N] (f_i = w_i + h_i for
   LBM_STORE_F16DEV), into device buffer out. */
lbm_status lbm_export_f32(lbm_handle h, float* out);
/* Overwrite the current state from float populations, SoA [19][N] (device
   buffer in; rounded to h_i = f_i - w_i in half for LBM_STORE_F16DEV). */
lbm_status lbm_import_f32(lbm_handle h, const float* in);

/*
 * LBM_STORE_F16DEV only: store the populations as half deviations from a
 * per-row reference equilibrium instead of the weights,
 *   h_i = f_i - w_i - r_i(y),  r_i(y) = f_eq_i(1, u_ref(y)) - w_i
 * (second-order equilibrium, Eq. (27) with rho = 1), u_ref: device double
 * [3][ny] reference velocity profile (e.g. the mean inflow), or NULL for
 * r = 0 (deviations from the weights, the default).  With u_ref near the
 * mean flow the stored deviations, and so their rounding, shrink by about
 * |u'| / |U|.  The arithmetic is unchanged (FP32); the current state is
 * re-encoded in place (one more rounding); population buffers saved earlier
 * (checkpoints, the other buffer) keep the old encoding.  Synchronises the
 * handle's stream.  On a HIP error the old reference stays in force.
 */
lbm_status lbm_set_reference(lbm_handle h, const double* u_ref);

/*
 * Plane statistics (Sec. IV.A: statistics over a time window).  For each x
 * in x_planes (host array), per row y, the sums over z and over steps of
 * u, v, w, uu, vv, ww, uv, uw, vw of the force-corrected velocity
 * (Eq. (11)) are accumulated in FP64 on the device during lbm_step.
 *   ATTACH  x_planes[n_planes] (distinct, in [0, nx)); allocates and zeroes
 *           the accumulators and starts accumulating.
 *   DETACH  stop accumulating (accumulators kept).
 *   RESET   zero the accumulators and the sample count.
 *   READ    synchronise; host_out[n_planes][ny][9] = the means over z and the
 *           sampled steps; *n_samples = number of steps accumulated.  Returns
 *           any latched device error.
 *   READ_WALL  (wall_model = 1) synchronise; host_out[2][nx] = the mean over z
 *           and the sampled steps of the wall law's u_tau (Eq. (20)) in the first
 *           off-wall cells, bottom (y = 0) then top (y = ny-1), at every x.
 */
lbm_status lbm_stats(lbm_handle h, int32_t op, const int32_t* x_planes, int32_t n_planes, double* host_out,
                     int64_t* n_samples);

/* Set the Smagorinsky constant C_s (C_smag = C_s^2, Sec. II.B, Eq. (13)-(15))
   used by later steps and adjoint steps; cs_smag >= 0. */
lbm_status lbm_set_cs_smag(lbm_handle h, double cs_smag);

/*
 * Discrete adjoint of one step n -> n+1: the transpose of the step's
 * linearisation (the step of Algorithm 1 with the rules of Sec. II-III), for
 * gradients of a loss L of the plane statistics with respect to the STG
 * amplitude scalings s_b (Sec. III.A, Eq. (22)) and C_s (Sec. II.B, Eq. (14)).
 *  s_n      device buffer of the post-collision state at time n (storage type
 *           and brick layout of the handle), 256-byte aligned;
 *  hist_n   device float [5][ny][nz], its outlet history (LBM_X_INFLOW);
 *  t_next   n + 1, the STG time of the step (the inlet plane is recomputed);
 *  lam_next dL/ds_{n+1}: device float bricks (lbm_state_elems() elements,
 *           256-byte aligned; padding nodes are neither read nor written);
 *  eta_next dL/dhist_{n+1}: device float [5][ny][nz] (LBM_X_INFLOW);
 *  lam_prev (written) dL/ds_n, float bricks, must not alias lam_next;
 *  eta_prev (written) dL/dhist_n (LBM_X_INFLOW), must not alias eta_next;
 *  coef     device float [n_planes][ny][9]: dL/d(the sums over z of u, v, w,
 *           uu, vv, ww, uv, uw, vw that step n -> n+1 adds at the attached
 *           statistics planes, see lbm_stats), or NULL when the step is not
 *           sampled;
 *  g_uin    (written, optional) dL/du_in(t_next), device float [3][ny][nz];
 *  u_in_next, fluct_next  (optional, both or neither) the inlet plane of the
 *           step (u_in and a v' at t_next, device float [3][ny][nz], as
 *           lbm_step_record keeps them); when NULL it is recomputed;
 *  grad     (optional) device double [n_bins + 1].  Every step adds its
 *           dL/ds_b (the bins of the bound STG inputs; n_bins = 0 with
 *           LBM_X_PERIODIC) and dL/dC_s to accumulators in the handle; a call
 *           with grad != NULL adds all that was accumulated since the last
 *           such call, this step included, to grad[b] and grad[n_bins] and
 *           clears the accumulators.  Pass it on the last step of a sweep.
 *           FP64, fixed-order sums: the result does not depend on scheduling.
 * Chaining calls backwards from lam = eta = 0, with the states of the forward
 * run, gives the gradient of a loss of the accumulated statistics.  The wall
 * law's u_tau is differentiated at its root.  Uses the handle's configuration
 * (C_s, rates, STG tables) and statistics planes; the handle's own state is
 * neither read nor changed.  Without u_in_next, overwrites the bound
 * stg->u_in (and stg->fluct) with the plane at t_next.  Errors: LBM_ERR_ARG (NULL or aliasing
 * buffers), LBM_ERR_SHAPE (alignment, ny > 4096), LBM_ERR_STATE
 * (LBM_X_INFLOW without bound STG inputs, coef without statistics planes).
 * Asynchronous on the handle's stream; the first call allocates the handle's
 * adjoint scratch (accumulators and the block dispatch order) and copies the
 * latter to the device synchronously.
 */
lbm_status lbm_adjoint_step(lbm_handle h, const lbm_stg* stg, const void* s_n, const float* hist_n, double t_next,
                            const float* lam_next, const float* eta_next, float* lam_prev, float* eta_prev,
                            const float* coef, float* g_uin, double* grad, const float* u_in_next,
                            const float* fluct_next);

/*
 * Forward recompute for an adjoint sweep (Algorithm 1 steps, as lbm_step):
 * nsteps steps from the state s_start (device, 256-byte aligned, time
 * t_start) with outlet history hist_start, writing the state after step k
 * (time t_start + k + 1) to f_out[k] and its history to hist_out[k], and the
 * inlet plane that step k used (t = t_start + k + 1) to uin_out[k] and
 * fluct_out[k].  f_out, hist_out, uin_out, fluct_out are host arrays of
 * nsteps device pointers (buffers as for lbm_create / lbm_stg); uin_out and
 * fluct_out may be NULL (planes not kept); hist_out is required with
 * LBM_X_INFLOW.  Consecutive buffers must differ.  Statistics are not
 * accumulated; the handle's own state is neither read nor changed.
 */
lbm_status lbm_step_record(lbm_handle h, const lbm_stg* stg, const void* s_start, const float* hist_start,
                           double t_start, int32_t nsteps, void* const* f_out, float* const* hist_out,
                           float* const* uin_out, float* const* fluct_out);

/* Float brick field (an adjoint field lam) <-> float SoA [19][N], device buffers. */
lbm_status lbm_field_export(lbm_handle h, const float* bricks, float* soa);
lbm_status lbm_field_import(lbm_handle h, const float* soa, float* bricks);

/* Wait for the handle's stream; return and clear any latched device error. */
lbm_status lbm_sync(lbm_handle h);
const char* lbm_status_str(lbm_status s);

/* When enabled, every launch of the dominant collide-stream kernel (with
   LBM_STORE_F32 the general kernel over all nodes, one launch being the
   step's dispatches over its x-chunks (lbm_collide_dispatches); with
   LBM_STORE_F16DEV the bulk kernel over the nodes away from the inlet, outlet
   and statistics planes, or on lattices of up to 2^24 nodes the one kernel
   over all nodes) is bracketed by HIP events on the handle's stream;
   *total_ms and *launches report the summed kernel time since the last
   reset, and *nodes_per_launch the nodes one launch updates (reading
   synchronises).  enable = 2 resets. */
lbm_status lbm_kernel_timing(lbm_handle h, int32_t enable, double* total_ms, int64_t* launches,
                             int64_t* nodes_per_launch);

/* Shape of one step's general-kernel dispatches (host only, no device work).
   With LBM_STORE_F32 the step goes out as one dispatch per range of
   *planes x-planes (the last range may be shorter), the ranges holding about
   30000 blocks of 256 nodes each, so *dispatches = ceil(nx / *planes); with
   LBM_STORE_F16DEV the general blocks, if any, are one dispatch
   (*dispatches = 1, or 0 without such blocks; *planes = nx).  Either pointer
   may be NULL. */
lbm_status lbm_collide_dispatches(lbm_handle h, int32_t* dispatches, int32_t* planes);

/* Plain device copy kernel (bandwidth calibration): dst[0:bytes) = src[0:bytes),
   bytes a multiple of 16, both 16-byte aligned. */
lbm_status lbm_copy_probe(const void* src, void* dst, int64_t bytes, void* hip_stream);

/* Host copies of the library's lattice tables (no device work): c[19][3]
   (c_x, c_y, c_z), w[19], opp[19], y-mirror[19]. */
void lbm_lattice_tables(int32_t* c, double* w, int32_t* opp, int32_t* refl_y);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
