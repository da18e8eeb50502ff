// C ABI of the library: argument checking, handle state, launch sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using lbm::Q;

namespace {

#define HIPCHK(expr)                        \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return LBM_ERR_HIP; \
  } while (0)

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

lbm_status check_config(const lbm_config* c) {
  if (!c) return LBM_ERR_ARG;
  if (c->nx < 1 || c->ny < lbm::YROWS || c->nz < 1) return LBM_ERR_SHAPE;
  if (c->xbc == LBM_X_INFLOW && c->nx < 3) return LBM_ERR_SHAPE;
  const int64_t N = (int64_t)c->nx * c->ny * c->nz;
  if (N >= (int64_t(1) << 31)) return LBM_ERR_SHAPE;
  const int64_t zc = (c->nz + lbm::ZT - 1) / lbm::ZT;
  if ((int64_t)c->nx * c->ny * zc * lbm::ZT * Q >= (int64_t(1) << 32)) return LBM_ERR_SHAPE;
  if (c->storage != LBM_STORE_F32 && c->storage != LBM_STORE_F16DEV) return LBM_ERR_ARG;
  if (c->ywall < LBM_Y_PERIODIC || c->ywall > LBM_Y_SLIP) return LBM_ERR_ARG;
  if (c->xbc != LBM_X_PERIODIC && c->xbc != LBM_X_INFLOW) return LBM_ERR_ARG;
  if (c->wall_model != 0 && c->wall_model != 1) return LBM_ERR_ARG;
  if (c->wall_model == 1 && c->ywall == LBM_Y_PERIODIC) return LBM_ERR_ARG;
  if (c->newton_iters < 0 || c->newton_iters > 64) return LBM_ERR_ARG;
  if (!(c->tau0 > 0.5) || !(c->cs_smag >= 0.0)) return LBM_ERR_ARG;
  if (c->wall_model == 1 && (!(c->kappa > 0.0) || !(c->y_wall > 0.0))) return LBM_ERR_ARG;
  if (c->xbc == LBM_X_INFLOW && !(c->u_conv >= 0.0)) return LBM_ERR_ARG;
  if (c->outlet != LBM_OUTLET_CONVECTIVE && c->outlet != LBM_OUTLET_ZERO_GRADIENT) return LBM_ERR_ARG;
  if (c->wall_law != LBM_WALL_REICHARDT && c->wall_law != LBM_WALL_MUSKER) return LBM_ERR_ARG;
  if (c->wall_avg != LBM_WALL_AVG_LOCAL && c->wall_avg != LBM_WALL_AVG_LINE) return LBM_ERR_ARG;
  if (c->sponge_cells < 0 || c->sponge_cells > c->nx - 1) return LBM_ERR_ARG;
  if (c->sponge_cells > 0 && (c->xbc != LBM_X_INFLOW || !(c->sponge_nu > 0.0))) return LBM_ERR_ARG;
  return LBM_OK;
}

lbm_status check_stg(const lbm_ctx* h, const lbm_stg* s) {
  if (!s) return LBM_ERR_ARG;
  if (s->n_modes < 1 || s->n_modes > LBM_MAX_MODES || s->n_bins < 1) return LBM_ERR_ARG;
  if (!s->sigma || !s->kmag || !s->d || !s->phi || !s->omega || !s->u_rans || !s->R || !s->amp_bin ||
      !s->bin_of_y || !s->u_in)
    return LBM_ERR_ARG;
  if (!s->k_rans != !s->omega_rans) return LBM_ERR_ARG;
  if (s->k_rans ? h->cfg.ywall == LBM_Y_PERIODIC : !s->q) return LBM_ERR_ARG;
  return LBM_OK;
}

lbm_status bind_stg(lbm_ctx* h, const lbm_stg* s) {
  lbm_status st = check_stg(h, s);
  if (st != LBM_OK) return st;
  h->stg = *s;
  HIPCHK(lbm::launch_stg_bind(h, s));
  h->stg_bound = true;
  return LBM_OK;
}

lbm_status take_error(lbm_ctx* h) {
  int err = 0;
  HIPCHK(hipMemcpyAsync(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (err) {
    HIPCHK(hipMemsetAsync(h->d_err, 0, sizeof(int), h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  if (err & lbm::ERRBIT_NONFINITE) return LBM_ERR_NONFINITE;
  if (err & lbm::ERRBIT_MACH) return LBM_ERR_MACH;
  if (err & lbm::ERRBIT_STG_TABLE) return LBM_ERR_ARG;
  return LBM_OK;
}

void free_tables(lbm_ctx* h) {
  lbm::StgTables& t = h->tab;
  if (t.amp3) (void)hipFree(t.amp3);
  if (t.ky) (void)hipFree(t.ky);
  if (t.trigz) (void)hipFree(t.trigz);
  if (t.chol) (void)hipFree(t.chol);
  if (t.sb) (void)hipFree(t.sb);
  if (t.urans) (void)hipFree(t.urans);
  if (t.rowamp_buf) (void)hipFree(t.rowamp_buf);
  t = lbm::StgTables();
}

// The timed collide launch (the bulk kernel with FP16 storage, or the fused
// kernel on small lattices; with FP32 storage the general kernel's dispatches
// over the step's x-chunks), bracketed by events when enabled.
hipError_t timed_launch(lbm_ctx* h, int src, int dst, const float* u_in, hipStream_t st) {
  auto launch = [&]() {
    return h->split ? lbm::launch_bulk(h, src, dst, st, u_in)
                    : lbm::launch_boundary(h, src, dst, st, u_in);
  };
  if (!h->timing) return launch();
  const size_t need = 2 * (size_t)(h->ev_used + 1);
  while (h->ev.size() < need) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    h->ev.push_back(e);
  }
  hipError_t r = hipEventRecord(h->ev[2 * h->ev_used], st);
  if (r != hipSuccess) return r;
  r = launch();
  if (r != hipSuccess) return r;
  r = hipEventRecord(h->ev[2 * h->ev_used + 1], st);
  if (r != hipSuccess) return r;
  ++h->ev_used;
  return hipSuccess;
}

hipError_t harvest_timing(lbm_ctx* h) {
  if (h->ev_used == 0) return hipSuccess;
  hipError_t r = hipEventSynchronize(h->ev[2 * h->ev_used - 1]);
  if (r != hipSuccess) return r;
  for (int64_t k = 0; k < h->ev_used; ++k) {
    float ms = 0.f;
    r = hipEventElapsedTime(&ms, h->ev[2 * k], h->ev[2 * k + 1]);
    if (r != hipSuccess) return r;
    h->timed_ms += ms;
    ++h->timed_launches;
  }
  h->ev_used = 0;
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* lbm_status_str(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_ARG: return "invalid argument";
    case LBM_ERR_SHAPE: return "invalid shape or alignment";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_MACH: return "inlet velocity above 0.3 c_s";
    case LBM_ERR_NONFINITE: return "non-finite or non-positive density";
    case LBM_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

lbm_status lbm_state_elems(const lbm_config* cfg, int64_t* elems) {
  if (!elems) return LBM_ERR_ARG;
  lbm_status st = check_config(cfg);
  if (st != LBM_OK) return st;
  *elems = (int64_t)Q * cfg->nx * cfg->ny * ((cfg->nz + lbm::ZT - 1) / lbm::ZT) * lbm::ZT;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_config* cfg, void* f_a, void* f_b, float* hist_a, float* hist_b, void* hip_stream,
                      lbm_handle* out) {
  if (!out) return LBM_ERR_ARG;
  *out = nullptr;
  lbm_status st = check_config(cfg);
  if (st != LBM_OK) return st;
  if (!f_a || !f_b || f_a == f_b) return LBM_ERR_ARG;
  if (!aligned256(f_a) || !aligned256(f_b)) return LBM_ERR_SHAPE;
  if (cfg->xbc == LBM_X_INFLOW && (!hist_a || !hist_b || hist_a == hist_b)) return LBM_ERR_ARG;
  lbm_ctx* h = new (std::nothrow) lbm_ctx();
  if (!h) return LBM_ERR_ARG;
  h->cfg = *cfg;
  if (h->cfg.newton_iters == 0 && h->cfg.wall_model) h->cfg.newton_iters = 4;
  h->stream = static_cast<hipStream_t>(hip_stream);
  // the device's address of the static scratch of stg_inlet_fill_noalloc (once per device)
  if (hipGetDevice(&h->device) != hipSuccess || lbm::noalloc_scratch_setup(h->device) != hipSuccess) {
    delete h;
    return LBM_ERR_HIP;
  }
  h->f[0] = f_a;
  h->f[1] = f_b;
  h->hist[0] = hist_a;
  h->hist[1] = hist_b;
  h->N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  h->zc = (cfg->nz + lbm::ZT - 1) / lbm::ZT;
  h->yg = (cfg->ny + lbm::YROWS - 1) / lbm::YROWS;
  h->split = cfg->storage == LBM_STORE_F16DEV;
  h->fused = h->split && h->N <= lbm::FUSED_MAX_NODES;
  const int64_t nb = (int64_t)cfg->nx * h->yg * h->zc;
  if (nb >= (int64_t(1) << 31)) {
    delete h;
    return LBM_ERR_SHAPE;
  }
  h->nblocks = (int)nb;
  if (hipMalloc(&h->d_err, sizeof(int)) != hipSuccess) {
    delete h;
    return LBM_ERR_HIP;
  }
  if (hipMalloc(&h->d_plane_of_x, sizeof(int) * cfg->nx) != hipSuccess) {
    (void)hipFree(h->d_err);
    delete h;
    return LBM_ERR_HIP;
  }
  std::vector<int> none(cfg->nx, -1);
  if (hipMemcpy(h->d_plane_of_x, none.data(), sizeof(int) * cfg->nx, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->d_err, 0, sizeof(int)) != hipSuccess || lbm::build_block_lists(h, none) != hipSuccess) {
    (void)hipFree(h->d_err);
    (void)hipFree(h->d_plane_of_x);
    if (h->d_blist_int) (void)hipFree(h->d_blist_int);
    if (h->d_blist_bnd) (void)hipFree(h->d_blist_bnd);
    delete h;
    return LBM_ERR_HIP;
  }
  h->plane_of_x = none;
  *out = h;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_handle h) {
  if (!h) return LBM_ERR_ARG;
  (void)hipStreamSynchronize(h->stream);
  free_tables(h);
  if (h->d_stats) (void)hipFree(h->d_stats);
  if (h->d_wall_acc) (void)hipFree(h->d_wall_acc);
  if (h->d_wall_line) (void)hipFree(h->d_wall_line);
  if (h->d_line_part) (void)hipFree(h->d_line_part);
  if (h->d_dref) (void)hipFree(h->d_dref);
  if (h->d_plane_of_x) (void)hipFree(h->d_plane_of_x);
  if (h->d_blist_int) (void)hipFree(h->d_blist_int);
  if (h->d_blist_bnd) (void)hipFree(h->d_blist_bnd);
  if (h->d_err) (void)hipFree(h->d_err);
  if (h->d_cs_part) (void)hipFree(h->d_cs_part);
  if (h->d_amp_part) (void)hipFree(h->d_amp_part);
  if (h->d_fluct) (void)hipFree(h->d_fluct);
  if (h->d_guin) (void)hipFree(h->d_guin);
  if (h->d_uin_ring) (void)hipFree(h->d_uin_ring);
  if (h->d_fl_ring) (void)hipFree(h->d_fl_ring);
  if (h->d_ablist) (void)hipFree(h->d_ablist);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  delete h;
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_handle h, void* f_a, void* f_b, float* hist_a, float* hist_b, int64_t time) {
  if (!h || !f_a || !f_b || f_a == f_b) return LBM_ERR_ARG;
  if (!aligned256(f_a) || !aligned256(f_b)) return LBM_ERR_SHAPE;
  if (h->cfg.xbc == LBM_X_INFLOW && (!hist_a || !hist_b || hist_a == hist_b)) return LBM_ERR_ARG;
  if (time < 0) return LBM_ERR_ARG;
  h->f[0] = f_a;
  h->f[1] = f_b;
  h->hist[0] = hist_a;
  h->hist[1] = hist_b;
  h->cur = 0;
  h->time = time;
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_handle h, void** f_cur, float** hist_cur, int64_t* time) {
  if (!h) return LBM_ERR_ARG;
  if (f_cur) *f_cur = h->f[h->cur];
  if (hist_cur) *hist_cur = h->hist[h->cur];
  if (time) *time = h->time;
  return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_handle h, const float* rho, const float* u, const float* pert, float eps) {
  if (!h || !u) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_init(h, rho, u, pert, eps));
  return LBM_OK;
}

lbm_status lbm_init_equilibrium_f64(lbm_handle h, const double* rho, const double* u, const double* pert,
                                     double eps) {
  if (!h || !u) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_init(h, rho, u, pert, eps));
  return LBM_OK;
}

lbm_status lbm_inflow_reichardt(lbm_handle h, double u_tau, double* u_rans) {
  if (!h || !u_rans || !(u_tau >= 0.0)) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_inflow_reichardt(h, u_tau, u_rans));
  return LBM_OK;
}

lbm_status stg_inlet_fill(lbm_handle h, const lbm_stg* stg, double t) {
  if (!h) return LBM_ERR_ARG;
  if (stg) {
    lbm_status st = bind_stg(h, stg);
    if (st != LBM_OK) return st;
  }
  if (!h->stg_bound) return LBM_ERR_STATE;
  HIPCHK(lbm::launch_stg_fill(h, t, h->stream));
  return LBM_OK;
}

lbm_status stg_inlet_fill_noalloc(lbm_handle h, const lbm_stg* stg, double t) {
  if (!h) return LBM_ERR_ARG;
  lbm_status st = check_stg(h, stg);
  if (st != LBM_OK) return st;
  if (lbm::noalloc_stg_bytes(h, stg) > lbm::NOALLOC_STG_BYTES) return LBM_ERR_SHAPE;
  HIPCHK(lbm::launch_stg_fill_noalloc(h, stg, t));
  return LBM_OK;
}

// nsteps steps from state parity cur at time index `time`, enqueued on st
// (the handle's state is not advanced).  Everything on one stream: FP32
// storage the general kernel, one dispatch per x-chunk; FP16 storage the
// boundary blocks (with the line-averaged wall model the line kernel first),
// then the bulk blocks, both reading s_n and writing disjoint nodes of
// s_{n+1}, as two launches or, on lattices up to FUSED_MAX_NODES, one
// (running the boundary blocks concurrently on a second stream cost more in
// cross-stream waits than it hid).  The inlet planes of up to STG_BATCH steps
// come from one launch into a ring; the plane of the last step also goes to
// the bound u_in / fluct.
hipError_t enqueue_steps(lbm_ctx* h, int cur, int64_t time, int32_t nsteps, hipStream_t st) {
  const bool inflow = h->cfg.xbc == LBM_X_INFLOW;
  const size_t plane = (size_t)3 * h->cfg.ny * h->cfg.nz;
  hipError_t e;
  for (int32_t n = 0; n < nsteps; ++n) {
    const float* ring = inflow ? h->d_uin_ring + plane * (size_t)(n % lbm::STG_BATCH) : nullptr;
    if (inflow && n % lbm::STG_BATCH == 0) {
      const int nb = (int)std::min<int64_t>(lbm::STG_BATCH, nsteps - n);
      const double t0 = (double)(time + n + 1);
      e = lbm::launch_stg_fill_batch(h, t0, nb, st, h->d_uin_ring, h->stg.fluct ? h->d_fl_ring : nullptr,
                                     n + nb == nsteps ? nb - 1 : -1);
      if (e != hipSuccess) return e;
    }
    if (h->split && (e = lbm::launch_boundary(h, cur, 1 - cur, st, ring)) != hipSuccess) return e;
    if ((e = timed_launch(h, cur, 1 - cur, ring, st)) != hipSuccess) return e;
    cur = 1 - cur;
  }
  return hipSuccess;
}

lbm_status lbm_step(lbm_handle h, const lbm_stg* stg, int32_t nsteps) {
  if (!h || nsteps < 0) return LBM_ERR_ARG;
  if (stg) {
    lbm_status st = bind_stg(h, stg);
    if (st != LBM_OK) return st;
  }
  const bool inflow = h->cfg.xbc == LBM_X_INFLOW;
  if (inflow && !h->stg_bound) return LBM_ERR_STATE;
  if (nsteps == 0) return LBM_OK;
  // The inlet planes of up to STG_BATCH steps are computed by one launch into
  // a ring (the plane of the call's last step also into the bound u_in /
  // fluct); the steps' kernels then read their plane from the ring.
  const size_t plane = (size_t)3 * h->cfg.ny * h->cfg.nz;
  if (inflow && !h->d_uin_ring) HIPCHK(hipMalloc(&h->d_uin_ring, sizeof(float) * plane * lbm::STG_BATCH));
  if (inflow && h->stg.fluct && !h->d_fl_ring) HIPCHK(hipMalloc(&h->d_fl_ring, sizeof(float) * plane * lbm::STG_BATCH));
  HIPCHK(enqueue_steps(h, h->cur, h->time, nsteps, h->stream));
  if (nsteps & 1) h->cur = 1 - h->cur;
  h->time += nsteps;
  if (h->stats_on) h->n_samples += nsteps;
  return LBM_OK;
}

lbm_status lbm_stream_only(lbm_handle h) {
  if (!h) return LBM_ERR_ARG;
  if (h->cfg.storage != LBM_STORE_F32) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_stream_only(h, h->cur, 1 - h->cur));
  h->cur = 1 - h->cur;
  return LBM_OK;
}

lbm_status lbm_export_f32(lbm_handle h, float* out) {
  if (!h || !out) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_export(h, out));
  return LBM_OK;
}

lbm_status lbm_import_f32(lbm_handle h, const float* in) {
  if (!h || !in) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_import(h, in));
  return LBM_OK;
}

lbm_status lbm_set_reference(lbm_handle h, const double* u_ref) {
  if (!h || h->cfg.storage != LBM_STORE_F16DEV) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_set_reference(h, u_ref));
  return LBM_OK;
}

lbm_status lbm_stats(lbm_handle h, int32_t op, const int32_t* x_planes, int32_t n_planes, double* host_out,
                     int64_t* n_samples) {
  if (!h) return LBM_ERR_ARG;
  const int nx = h->cfg.nx, ny = h->cfg.ny;
  switch (op) {
    case LBM_STATS_ATTACH: {
      if (!x_planes || n_planes < 1 || n_planes > nx) return LBM_ERR_ARG;
      std::vector<int> map(nx, -1);
      for (int p = 0; p < n_planes; ++p) {
        const int x = x_planes[p];
        if (x < 0 || x >= nx || map[x] >= 0) return LBM_ERR_ARG;
        map[x] = p;
      }
      HIPCHK(hipStreamSynchronize(h->stream));
      if (h->d_stats) {
        HIPCHK(hipFree(h->d_stats));
        h->d_stats = nullptr;
      }
      const size_t bytes = sizeof(double) * (size_t)n_planes * ny * h->zc * 9;
      HIPCHK(hipMalloc(&h->d_stats, bytes));
      HIPCHK(hipMemsetAsync(h->d_stats, 0, bytes, h->stream));
      if (h->cfg.wall_model && !h->d_wall_acc) HIPCHK(hipMalloc(&h->d_wall_acc, sizeof(double) * 2 * nx * h->zc));
      if (h->d_wall_acc) HIPCHK(hipMemsetAsync(h->d_wall_acc, 0, sizeof(double) * 2 * nx * h->zc, h->stream));
      HIPCHK(hipMemcpyAsync(h->d_plane_of_x, map.data(), sizeof(int) * nx, hipMemcpyHostToDevice, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      h->n_planes = n_planes;
      h->n_samples = 0;
      h->stats_on = 1;
      h->plane_of_x = map;
      HIPCHK(lbm::build_block_lists(h, h->plane_of_x));
      return LBM_OK;
    }
    case LBM_STATS_DETACH:
      // the planes keep their block routing (general kernel with FP16 storage), so a step's
      // result does not depend on whether its statistics are accumulated
      h->stats_on = 0;
      return LBM_OK;
    case LBM_STATS_RESET: {
      if (!h->d_stats) return LBM_ERR_STATE;
      const size_t bytes = sizeof(double) * (size_t)h->n_planes * ny * h->zc * 9;
      HIPCHK(hipMemsetAsync(h->d_stats, 0, bytes, h->stream));
      if (h->d_wall_acc) HIPCHK(hipMemsetAsync(h->d_wall_acc, 0, sizeof(double) * 2 * nx * h->zc, h->stream));
      h->n_samples = 0;
      return LBM_OK;
    }
    case LBM_STATS_READ: {
      if (!h->d_stats) return LBM_ERR_STATE;
      if (!host_out) return LBM_ERR_ARG;
      const size_t cnt = (size_t)h->n_planes * ny * h->zc * 9;
      std::vector<double> raw(cnt);
      HIPCHK(hipMemcpyAsync(raw.data(), h->d_stats, sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream));
      lbm_status st = take_error(h);
      // fixed-order sum over the z-chunks, then the mean over z and samples
      const double denom = (double)h->n_samples * h->cfg.nz;
      for (int p = 0; p < h->n_planes; ++p)
        for (int y = 0; y < ny; ++y)
          for (int k = 0; k < 9; ++k) {
            double acc = 0.0;
            for (int c = 0; c < h->zc; ++c) acc += raw[(((size_t)p * ny + y) * h->zc + c) * 9 + k];
            host_out[((size_t)p * ny + y) * 9 + k] = denom > 0 ? acc / denom : 0.0;
          }
      if (n_samples) *n_samples = h->n_samples;
      return st;
    }
    case LBM_STATS_READ_WALL: {
      if (!h->d_wall_acc) return LBM_ERR_STATE;
      if (!host_out) return LBM_ERR_ARG;
      const size_t cnt = (size_t)2 * nx * h->zc;
      std::vector<double> raw(cnt);
      HIPCHK(hipMemcpyAsync(raw.data(), h->d_wall_acc, sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream));
      lbm_status st = take_error(h);
      const double denom = (double)h->n_samples * h->cfg.nz;
      for (int w = 0; w < 2; ++w)
        for (int x = 0; x < nx; ++x) {
          double acc = 0.0;  // fixed-order sum over the z-chunks
          for (int c = 0; c < h->zc; ++c) acc += raw[((size_t)w * nx + x) * h->zc + c];
          host_out[(size_t)w * nx + x] = denom > 0 ? acc / denom : 0.0;
        }
      if (n_samples) *n_samples = h->n_samples;
      return st;
    }
    default:
      return LBM_ERR_ARG;
  }
}

lbm_status lbm_set_cs_smag(lbm_handle h, double cs_smag) {
  if (!h || !(cs_smag >= 0.0)) return LBM_ERR_ARG;
  h->cfg.cs_smag = cs_smag;
  return LBM_OK;
}

lbm_status lbm_step_record(lbm_handle h, const lbm_stg* stg, const void* s_start, const float* hist_start,
                           double t_start, int32_t nsteps, void* const* f_out, float* const* hist_out,
                           float* const* uin_out, float* const* fluct_out) {
  if (!h || !s_start || nsteps < 0 || (nsteps > 0 && !f_out)) return LBM_ERR_ARG;
  const bool inflow = h->cfg.xbc == LBM_X_INFLOW;
  if (inflow && (!hist_start || (nsteps > 0 && !hist_out))) return LBM_ERR_ARG;
  if (!aligned256(s_start)) return LBM_ERR_SHAPE;
  for (int32_t k = 0; k < nsteps; ++k) {
    const void* src = k == 0 ? s_start : f_out[k - 1];
    if (!f_out[k] || f_out[k] == src) return LBM_ERR_ARG;
    if (!aligned256(f_out[k])) return LBM_ERR_SHAPE;
    if (inflow) {
      const float* hsrc = k == 0 ? hist_start : hist_out[k - 1];
      if (!hist_out[k] || hist_out[k] == hsrc) return LBM_ERR_ARG;
      if (uin_out && !uin_out[k]) return LBM_ERR_ARG;
    }
  }
  if (stg) {
    lbm_status st = bind_stg(h, stg);
    if (st != LBM_OK) return st;
  }
  if (inflow && !h->stg_bound) return LBM_ERR_STATE;
  // with every plane kept, the planes of up to STG_BATCH steps come from one launch
  bool batch = inflow && uin_out && fluct_out;
  for (int32_t k = 0; batch && k < nsteps; ++k) batch = fluct_out[k] != nullptr;
  for (int32_t k = 0; k < nsteps; ++k) {
    const void* src = k == 0 ? s_start : f_out[k - 1];
    float* uin = uin_out ? uin_out[k] : h->stg.u_in;
    float* fl = fluct_out ? fluct_out[k] : nullptr;
    if (batch && k % lbm::STG_BATCH == 0) {
      const int nb = (int)std::min<int64_t>(lbm::STG_BATCH, nsteps - k);
      lbm::PlaneDst dst{};
      for (int j = 0; j < nb; ++j) {
        dst.u[j] = uin_out[k + j];
        dst.f[j] = fluct_out[k + j];
      }
      HIPCHK(lbm::launch_stg_fill_to(h, t_start + k + 1, nb, h->stream, dst));
    } else if (inflow && !batch) {
      HIPCHK(lbm::launch_stg_fill(h, t_start + k + 1, h->stream, fl, uin));
    }
    const float* hsrc = inflow ? (k == 0 ? hist_start : hist_out[k - 1]) : nullptr;
    HIPCHK(lbm::launch_step_explicit(h, src, f_out[k], hsrc, inflow ? hist_out[k] : nullptr, inflow ? uin : nullptr,
                                     h->stream));
  }
  return LBM_OK;
}

lbm_status lbm_adjoint_step(lbm_handle h, const lbm_stg* stg, const void* s_n, const float* hist_n, double t_next,
                            const float* lam_next, const float* eta_next, float* lam_prev, float* eta_prev,
                            const float* coef, float* g_uin, double* grad, const float* u_in_next,
                            const float* fluct_next) {
  if (!h || !s_n || !lam_next || !lam_prev || lam_next == lam_prev) return LBM_ERR_ARG;
  if (!aligned256(s_n) || !aligned256(lam_next) || !aligned256(lam_prev)) return LBM_ERR_SHAPE;
  const bool inflow = h->cfg.xbc == LBM_X_INFLOW;
  if (inflow && (!hist_n || !eta_next || !eta_prev || eta_next == eta_prev)) return LBM_ERR_ARG;
  if (!u_in_next != !fluct_next) return LBM_ERR_ARG;  // the inlet plane is given whole or recomputed
  if (stg) {
    lbm_status st = bind_stg(h, stg);
    if (st != LBM_OK) return st;
  }
  if (inflow && !h->stg_bound) return LBM_ERR_STATE;
  if (coef && h->n_planes < 1) return LBM_ERR_STATE;
  const size_t plane = (size_t)3 * h->cfg.ny * h->cfg.nz;
  if (h->cfg.ny > LBM_ADJ_MAX_NY) return LBM_ERR_SHAPE;
  if (!h->d_cs_part) {  // accumulators start at zero; each reduction clears them
    HIPCHK(hipMalloc(&h->d_cs_part, sizeof(double) * h->nblocks));
    HIPCHK(hipMemset(h->d_cs_part, 0, sizeof(double) * h->nblocks));
  }
  if (!h->d_amp_part) {
    HIPCHK(hipMalloc(&h->d_amp_part, sizeof(double) * h->cfg.ny * h->zc));
    HIPCHK(hipMemset(h->d_amp_part, 0, sizeof(double) * h->cfg.ny * h->zc));
  }
  if (inflow && !h->stg.fluct && !h->d_fluct) HIPCHK(hipMalloc(&h->d_fluct, sizeof(float) * plane));
  if (inflow && !g_uin && !h->d_guin) HIPCHK(hipMalloc(&h->d_guin, sizeof(float) * plane));
  lbm::AdjointArgs A;
  lbm::fill_args(h, A.c, h->cur, h->cur);
  A.c.src = s_n;
  A.c.dst = nullptr;
  A.c.hist_in = inflow ? hist_n : nullptr;
  A.c.hist_out = nullptr;
  A.c.stats = nullptr;
  A.c.stats_on = 0;
  A.c.u_in = inflow ? (u_in_next ? u_in_next : h->stg.u_in) : nullptr;
  A.lam_next = lam_next;
  A.lam_prev = lam_prev;
  A.eta_next = inflow ? eta_next : nullptr;
  A.eta_prev = inflow ? eta_prev : nullptr;
  A.coef = coef;
  A.g_uin = inflow ? (g_uin ? g_uin : h->d_guin) : nullptr;
  A.cs_part = h->d_cs_part;
  A.amp_part = h->d_amp_part;
  A.line_part = nullptr;  // set by launch_adjoint with the line-averaged wall model
  A.dsmag = (float)(36.0 * std::sqrt(2.0) * h->cfg.cs_smag);  // d(18 sqrt(2) C_s^2)/dC_s
  float* fluct = inflow ? (h->stg.fluct ? h->stg.fluct : h->d_fluct) : nullptr;
  A.fluct = fluct_next ? fluct_next : fluct;
  HIPCHK(lbm::launch_adjoint(h, A, h->cfg.storage == LBM_STORE_F16DEV, t_next, inflow && !u_in_next, nullptr, fluct));
  if (grad) HIPCHK(lbm::launch_adjoint_reduce(h, grad));
  return LBM_OK;
}

lbm_status lbm_field_export(lbm_handle h, const float* bricks, float* soa) {
  if (!h || !bricks || !soa) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_field_export(h, bricks, soa));
  return LBM_OK;
}

lbm_status lbm_field_import(lbm_handle h, const float* soa, float* bricks) {
  if (!h || !bricks || !soa) return LBM_ERR_ARG;
  HIPCHK(lbm::launch_field_import(h, soa, bricks));
  return LBM_OK;
}

lbm_status lbm_sync(lbm_handle h) {
  if (!h) return LBM_ERR_ARG;
  HIPCHK(hipStreamSynchronize(h->stream));
  return take_error(h);
}

lbm_status lbm_kernel_timing(lbm_handle h, int32_t enable, double* total_ms, int64_t* launches,
                              int64_t* nodes_per_launch) {
  if (!h) return LBM_ERR_ARG;
  HIPCHK(harvest_timing(h));
  if (total_ms) *total_ms = h->timed_ms;
  if (launches) *launches = h->timed_launches;
  if (nodes_per_launch) *nodes_per_launch = h->split && !h->fused ? h->int_nodes : h->N;
  if (enable == 2) {
    h->timed_ms = 0.0;
    h->timed_launches = 0;
    h->timing = 1;
  } else {
    h->timing = enable ? 1 : 0;
  }
  return LBM_OK;
}

lbm_status lbm_collide_dispatches(lbm_handle h, int32_t* dispatches, int32_t* planes) {
  if (!h) return LBM_ERR_ARG;
  if (dispatches) *dispatches = (int32_t)h->bnd_off.size() - 1;
  if (planes) *planes = h->chunk_planes;
  return LBM_OK;
}

lbm_status lbm_copy_probe(const void* src, void* dst, int64_t bytes, void* hip_stream) {
  if (!src || !dst || bytes <= 0 || (bytes & 15) != 0) return LBM_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(src) & 15u) || (reinterpret_cast<uintptr_t>(dst) & 15u)) return LBM_ERR_SHAPE;
  HIPCHK(lbm::launch_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

void lbm_lattice_tables(int32_t* c, double* w, int32_t* opp, int32_t* refl_y) {
  for (int i = 0; i < Q; ++i) {
    if (c) {
      c[3 * i] = lbm::CX[i];
      c[3 * i + 1] = lbm::CY[i];
      c[3 * i + 2] = lbm::CZ[i];
    }
    if (w) w[i] = lbm::WD[i];
    if (opp) opp[i] = lbm::opp(i);
    if (refl_y) refl_y[i] = lbm::REFLY[i];
  }
}

}  // extern "C"
